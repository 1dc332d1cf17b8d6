// Left-to-right sweep of two-site local solves (Implementation section: one tensor is
// optimised at a time, the others fixed, sweeping over the sites).
//
// After the local problem at (l, l+1) is solved, the two-site tensor is split per middle-bond
// sector by an SVD (X_q = U_q S_q V_q^T), the m_max largest singular values over all sectors
// are kept, U becomes the new left-canonical tensor of site l, the left environment is
// extended by that site on the device, and S V^T contracted with the right-canonical tensor of
// site l+2 is the initial guess of the next local problem at (l+1, l+2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "state.h"

namespace lcc {
namespace {

// dst[i*cols + c] = s[i] * src[i*ld + c]  (i < rows)
__global__ void scale_rows_kernel(double* __restrict__ dst, const double* __restrict__ src, const double* __restrict__ s,
                                  int rows, int cols, int ld) {
  const int64_t n = (int64_t)rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / cols), c = (int)(e % cols);
    dst[e] = s[i] * src[(int64_t)i * ld + c];
  }
}

// ---------------------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi SVD of every middle-bond sector, blocked over workgroups.
//
// The sector block X (row-major nrows x ncols) is copied into a column-major m x n workspace
// W with n = min(nrows, ncols): W = X if nrows >= ncols, else W = X^T; V (n x n, column j
// contiguous) starts as the identity.  Pairs of columns are rotated until every pair is
// orthogonal to a relative tolerance; the rotations accumulate in V, so that W V_0 ... =
// U diag(s).  Singular values are the final column norms, written in descending order
// together with the matching vectors:
//   left vectors of X  (row-major nrows x n)  -> L,   right vectors (row-major n x ncols) -> R.
//
// Blocking: the n columns are cut into nb blocks of w columns.  One outer sweep is a
// round-robin over the blocks (nb - 1 rounds, one more with a dummy when nb is odd); in a
// round, every pair of blocks goes to one workgroup, which copies the pair's columns into LDS,
// runs one-sided Jacobi sweeps among them (rotation angles from the columns' own dot
// products, as in the unblocked method, so small singular values keep their relative
// accuracy), accumulates the rotations in a small matrix Q, writes the columns back and
// applies Q to the same columns of V.  A sector has converged when a whole outer sweep finds
// no pair to rotate.  One launch per round, all sectors together; sectors with fewer rounds or
// already converged leave their workgroups idle.
// ---------------------------------------------------------------------------------------
struct SvdJob {
  int64_t x_off;                // the block in the two-site vector
  int64_t w_off;                // workspace: W (m n), V (n n), norms (n), ranks (n)
  int64_t s_off, l_off, r_off;  // outputs
  int32_t nrows, ncols;
  int32_t w, nb;                // columns per block, blocks
};
struct SvdSlot {  // one workgroup of a round: job and pair index in the round-robin
  int32_t job, k;
};
constexpr int kSvdThreads = 1024;
constexpr int kSvdMaxSweeps = 60;
constexpr double kSvdTol = 1e-14;  // |w_i . w_j| <= tol ||w_i|| ||w_j|| counts as orthogonal
constexpr int kSvdMaxW = 8;        // columns per block (a pair of blocks: at most 16 columns)
constexpr int kSvdLdsCols = 120 * 1024 / (int)sizeof(double);  // LDS budget for a pair's columns, elements
constexpr int kSvdInner = 1;       // Jacobi sweeps per visit of a block pair (more when it is the whole matrix)
constexpr int kSvdRoundThreads = 64 * kSvdMaxW;  // one wave per column pair of a block pair

constexpr int kSvdGroup = 64;  // lanes (one wave) per column pair inside a block pair

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// sum over the kSvdGroup lanes of a group (groups are aligned within the wave)
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = kSvdGroup / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// players i, j of pair k in round r of a round-robin over N (even) players
__device__ __forceinline__ void round_robin(int N, int r, int k, int& i, int& j) {
  i = k == 0 ? N - 1 : (r + k) % (N - 1);
  j = k == 0 ? r : (r - k + N - 1) % (N - 1);
}

__global__ void __launch_bounds__(kSvdThreads)
svd_setup_kernel(const SvdJob* __restrict__ jobs, const double* __restrict__ x, double* __restrict__ work) {
  const SvdJob jb = jobs[blockIdx.x];
  const bool tall = jb.nrows >= jb.ncols;
  const int m = tall ? jb.nrows : jb.ncols, n = tall ? jb.ncols : jb.nrows;
  double* W = work + jb.w_off;
  double* V = W + (int64_t)m * n;
  const double* X = x + jb.x_off;
  for (int64_t e = threadIdx.x; e < (int64_t)m * n; e += blockDim.x) {
    const int j = (int)(e / m), i = (int)(e % m);
    W[e] = tall ? X[(int64_t)i * jb.ncols + j] : X[(int64_t)j * jb.ncols + i];
  }
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += blockDim.x) V[e] = (e / n == e % n) ? 1.0 : 0.0;
}

// One round of the blocked sweep.  rot[job] is set when a pair of the job needed a rotation;
// done[job] marks converged jobs.
__global__ void __launch_bounds__(kSvdRoundThreads)
svd_round_kernel(const SvdJob* __restrict__ jobs, const SvdSlot* __restrict__ slots, int round,
                 double* __restrict__ work, int* __restrict__ rot, const int* __restrict__ done) {
  extern __shared__ double cols[];  // the pair's columns, column-major m x cnt
  __shared__ double Q[2 * kSvdMaxW][2 * kSvdMaxW];
  __shared__ int col_of[2 * kSvdMaxW];
  __shared__ int rotated, any;
  const SvdSlot sl = slots[blockIdx.x];
  if (done[sl.job]) return;
  const SvdJob jb = jobs[sl.job];
  const int N = jb.nb + (jb.nb & 1);
  if (round >= N - 1 && !(jb.nb == 1 && round == 0)) return;  // this job has fewer rounds
  int bp = 0, bq = 1;
  if (jb.nb > 1) round_robin(N, round, sl.k, bp, bq);
  const bool tall = jb.nrows >= jb.ncols;
  const int m = tall ? jb.nrows : jb.ncols, n = tall ? jb.ncols : jb.nrows;
  double* W = work + jb.w_off;
  double* V = W + (int64_t)m * n;
  // columns of the pair: block bp, then block bq (a dummy block, index >= nb, has none)
  const int np = bp < jb.nb ? min(n, (bp + 1) * jb.w) - bp * jb.w : 0;
  const int nq = bq < jb.nb ? min(n, (bq + 1) * jb.w) - bq * jb.w : 0;
  const int cnt = np + nq;
  if (cnt < 2) return;  // a lone column: nothing to rotate
  if (threadIdx.x < cnt) col_of[threadIdx.x] = threadIdx.x < np ? bp * jb.w + threadIdx.x : bq * jb.w + threadIdx.x - np;
  if (threadIdx.x == 0) {
    rotated = 0;
    any = 0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < m * cnt; e += blockDim.x) cols[e] = W[(int64_t)col_of[e / m] * m + e % m];
  for (int e = threadIdx.x; e < 4 * kSvdMaxW * kSvdMaxW; e += blockDim.x) {
    const int a = e / (2 * kSvdMaxW), b = e % (2 * kSvdMaxW);
    Q[a][b] = a == b ? 1.0 : 0.0;
  }
  __syncthreads();
  const int gl = threadIdx.x % kSvdGroup, grp = threadIdx.x / kSvdGroup;
  const int N2 = cnt + (cnt & 1);
  const int inner = jb.nb == 1 ? kSvdMaxSweeps : kSvdInner;
  for (int sweep = 0; sweep < inner; ++sweep) {
    for (int r = 0; r < N2 - 1; ++r) {
      if (grp < N2 / 2) {
        int i, j;
        round_robin(N2, r, grp, i, j);
        if (i < cnt && j < cnt) {
          if (i > j) {
            const int t = i;
            i = j;
            j = t;
          }
          double* wi = cols + i * m;
          double* wj = cols + j * m;
          double a = 0, b = 0, g = 0;
          for (int t = gl; t < m; t += kSvdGroup) {
            const double u = wi[t], v = wj[t];
            a += u * u;
            b += v * v;
            g += u * v;
          }
          a = group_sum(a);
          b = group_sum(b);
          g = group_sum(g);
          if (fabs(g) > kSvdTol * sqrt(a * b)) {
            const double zeta = (b - a) / (2.0 * g);
            const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
            for (int q = gl; q < m; q += kSvdGroup) {
              const double u = wi[q], v = wj[q];
              wi[q] = c * u - s * v;
              wj[q] = s * u + c * v;
            }
            for (int q = gl; q < cnt; q += kSvdGroup) {
              const double u = Q[q][i], v = Q[q][j];
              Q[q][i] = c * u - s * v;
              Q[q][j] = s * u + c * v;
            }
            if (gl == 0) rotated = 1;
          }
        }
      }
      __syncthreads();
    }
    const int rs = rotated;
    __syncthreads();
    if (rs == 0) break;
    if (threadIdx.x == 0) {
      any = 1;
      rotated = 0;
    }
    __syncthreads();
  }
  if (any == 0) return;  // the pair was orthogonal: W and V unchanged
  if (threadIdx.x == 0) rot[sl.job] = 1;
  for (int e = threadIdx.x; e < m * cnt; e += blockDim.x) W[(int64_t)col_of[e / m] * m + e % m] = cols[e];
  __syncthreads();
  // V(:, C) <- V(:, C) Q, through LDS (n <= m, so the pair's V columns fit where W's were)
  for (int e = threadIdx.x; e < n * cnt; e += blockDim.x) cols[e] = V[(int64_t)col_of[e / n] * n + e % n];
  __syncthreads();
  for (int e = threadIdx.x; e < n * cnt; e += blockDim.x) {
    const int c = e / n, t = e % n;
    double v = 0;
    for (int k = 0; k < cnt; ++k) v += cols[k * n + t] * Q[k][c];
    V[(int64_t)col_of[c] * n + t] = v;
  }
}

// Singular values (column norms, descending) and vectors of every converged job.
__global__ void __launch_bounds__(kSvdThreads)
svd_finalize_kernel(const SvdJob* __restrict__ jobs, double* __restrict__ work, double* __restrict__ S,
                    double* __restrict__ L, double* __restrict__ R) {
  const SvdJob jb = jobs[blockIdx.x];
  const bool tall = jb.nrows >= jb.ncols;
  const int m = tall ? jb.nrows : jb.ncols, n = tall ? jb.ncols : jb.nrows;
  double* W = work + jb.w_off;
  double* V = W + (int64_t)m * n;
  double* nrm = V + (int64_t)n * n;
  double* rank = nrm + n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  for (int j = wave; j < n; j += nwaves) {
    const double* wj = W + (int64_t)j * m;
    double a = 0;
    for (int t = lane; t < m; t += 64) a += wj[t] * wj[t];
    a = wave_sum(a);
    if (lane == 0) nrm[j] = sqrt(a);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    int rk = 0;
    for (int k = 0; k < n; ++k) rk += (nrm[k] > nrm[j]) || (nrm[k] == nrm[j] && k < j);
    rank[j] = rk;
    S[jb.s_off + rk] = nrm[j];
  }
  __syncthreads();
  // tall: X = (W/s) diag(s) V^T -> L from W, R from V;  wide: X^T = (W/s) diag(s) V^T -> L from V, R from W
  for (int64_t e = threadIdx.x; e < (int64_t)m * n; e += blockDim.x) {
    const int j = (int)(e / m), i = (int)(e % m);
    const double u = nrm[j] > 0.0 ? W[e] / nrm[j] : 0.0;
    const int rk = (int)rank[j];
    if (tall) L[jb.l_off + (int64_t)i * n + rk] = u;
    else R[jb.r_off + (int64_t)rk * jb.ncols + i] = u;
  }
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += blockDim.x) {
    const int j = (int)(e / n), i = (int)(e % n);
    const int rk = (int)rank[j];
    if (tall) R[jb.r_off + (int64_t)rk * jb.ncols + i] = V[e];
    else L[jb.l_off + (int64_t)i * n + rk] = V[e];
  }
}

}  // namespace

struct Sweep {
  Context* ctx = nullptr;
  const Hamiltonian* ham = nullptr;
  DeviceMps mps;
  std::vector<Environment> R;  // R[j]: right environment at MPS bond j (j >= first + 2)
  Environment L;
  Bond bl;  // current left bond of the block
  int site = 0, first = 0;
  std::unique_ptr<Env> env;
  DevBuf guess;      // initial guess of the current local problem (n_elements), valid if have_guess
  bool have_guess = false;
  std::vector<double> last_sv;  // singular values of the last split, descending
};

Sweep* sweep_create(Context* ctx, const Hamiltonian& ham, const lcc_mps_desc& md, int first) {
  hipStream_t st = ctx->stream;
  const Mpo& mpo = ham.mpo;
  const int K = mpo.K;
  if (md.n_sites != K) throw Error{LCC_ERR_ARG, "MPS length differs from the Hamiltonian's orbital count"};
  if (first < 0 || first + 1 >= K) throw Error{LCC_ERR_ARG, "first two-site block must satisfy 0 <= site < K-1"};
  std::unique_ptr<Sweep> S(new Sweep());
  S->ctx = ctx;
  S->ham = &ham;
  S->first = S->site = first;
  load_mps(md, ham.desc.N, ham.desc.two_sz, st, S->mps);
  S->L = unit_env(st);
  for (int j = 0; j < first; ++j) S->L = left_step(S->L, S->mps, j, mpo, st);
  S->R.resize(K + 1);
  S->R[K] = unit_env(st);
  for (int j = K - 1; j >= first + 2; --j) S->R[j] = right_step(S->R[j + 1], S->mps, j, mpo, st);
  const int wl = channel_of_kind(mpo, first, 0), wr = channel_of_kind(mpo, first + 2, 1);
  if (first > 0 && wl >= 0) check_identity(S->L, wl, S->mps.bonds[first], st, "left");
  if (first + 2 < K && wr >= 0) check_identity(S->R[first + 2], wr, S->mps.bonds[first + 2], st, "right");
  S->bl = S->mps.bonds[first];
  S->env.reset(make_env(ctx, mpo, first, S->bl, S->mps.bonds[first + 2], S->L, S->R[first + 2]));
  return S.release();
}

void sweep_destroy(Sweep* s) { delete s; }
Env* sweep_env(Sweep& s) { return s.env.get(); }

void sweep_advance(Sweep& S, const double* x, int m_max, lcc_sweep_info* info) {
  hipStream_t st = S.ctx->stream;
  typedef std::chrono::steady_clock clk;
  const auto ms_since = [](clk::time_point t) {
    return (float)std::chrono::duration<double, std::milli>(clk::now() - t).count();
  };
  const clk::time_point t_start = clk::now();
  const Mpo& mpo = S.ham->mpo;
  const int K = mpo.K;
  if (S.site + 2 >= K) throw Error{LCC_ERR_STATE, "the sweep is already at the last two-site block"};
  if (m_max < 1) throw Error{LCC_ERR_ARG, "m_max must be >= 1"};
  Env& E = *S.env;
  const int nsec = (int)E.sectors.size();
  // ---- SVD per middle sector (one workgroup each): singular values descending at s_off, left
  // vectors as a row-major nrows x r matrix at v_off, right vectors as a row-major r x ncols
  // matrix at u_off (r = min(nrows, ncols)).
  struct Split { int r; int64_t s_off, u_off, v_off; };
  std::vector<Split> sp(nsec);
  std::vector<SvdJob> jobs(nsec);
  int64_t s_tot = 0, u_tot = 0, v_tot = 0, w_tot = 0;
  for (int q = 0; q < nsec; ++q) {
    const MiddleSector& M = E.sectors[q];
    Split& p = sp[q];
    p.r = std::min(M.nrows, M.ncols);
    p.s_off = s_tot; s_tot += p.r;
    p.u_off = u_tot; u_tot += (int64_t)M.ncols * p.r;
    p.v_off = v_tot; v_tot += (int64_t)p.r * M.nrows;
    SvdJob& j = jobs[q];
    j.x_off = M.off;
    j.w_off = w_tot;
    const int mm = std::max(M.nrows, M.ncols);
    w_tot += (int64_t)mm * p.r + (int64_t)p.r * p.r + 2 * (int64_t)p.r;
    j.s_off = p.s_off;
    j.l_off = p.v_off;
    j.r_off = p.u_off;
    j.nrows = M.nrows;
    j.ncols = M.ncols;
    // a pair of blocks (2w columns of mm rows) must fit the LDS budget of the round kernel
    if (2 * mm > kSvdLdsCols) throw Error{LCC_ERR_ARG, "a middle-bond sector is too tall for the blocked SVD"};
    j.w = std::max(1, std::min(kSvdMaxW, kSvdLdsCols / (2 * mm)));
    j.nb = std::max(1, (p.r + j.w - 1) / j.w);
  }
  // workgroups of a round: the pairs of each job's round-robin over its blocks
  std::vector<SvdSlot> slots;
  int rounds = 1;
  int64_t lds_cols = 1;  // LDS of the round kernel: the largest pair of blocks
  for (int q = 0; q < nsec; ++q) {
    lds_cols = std::max<int64_t>(lds_cols, 2 * (int64_t)jobs[q].w * std::max(jobs[q].nrows, jobs[q].ncols));
    const int N = jobs[q].nb + (jobs[q].nb & 1);
    rounds = std::max(rounds, N - 1);
    for (int k = 0; k < std::max(1, N / 2); ++k) slots.push_back(SvdSlot{q, k});
  }
  DevBuf Sv, U, V, Wk, rot, done, djobs, dslots;
  Sv.alloc(sizeof(double) * std::max<int64_t>(s_tot, 1));
  U.alloc(sizeof(double) * std::max<int64_t>(u_tot, 1));
  V.alloc(sizeof(double) * std::max<int64_t>(v_tot, 1));
  Wk.alloc(sizeof(double) * std::max<int64_t>(w_tot, 1));
  rot.alloc(sizeof(int) * std::max(nsec, 1));
  done.alloc(sizeof(int) * std::max(nsec, 1));
  upload(djobs, jobs, st);
  upload(dslots, slots, st);
  std::vector<double> hs(s_tot);
  if (nsec > 0) {
    const size_t lds = sizeof(double) * lds_cols;
    check_hip(hipFuncSetAttribute((const void*)svd_round_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
              "svd lds");
    hipLaunchKernelGGL(svd_setup_kernel, dim3(nsec), dim3(kSvdThreads), 0, st, djobs.as<SvdJob>(), x, Wk.as<double>());
    check_hip(hipMemsetAsync(done.p, 0, sizeof(int) * nsec, st), "svd flags");
    std::vector<int> hrot(nsec), hdone(nsec, 0);
    bool converged = false;
    for (int sweep = 0; sweep < kSvdMaxSweeps && !converged; ++sweep) {
      check_hip(hipMemsetAsync(rot.p, 0, sizeof(int) * nsec, st), "svd flags");
      for (int r = 0; r < rounds; ++r)
        hipLaunchKernelGGL(svd_round_kernel, dim3((unsigned)slots.size()), dim3(kSvdRoundThreads), lds, st,
                           djobs.as<SvdJob>(), dslots.as<SvdSlot>(), r, Wk.as<double>(), rot.as<int>(),
                           (const int*)done.as<int>());
      check_hip(hipGetLastError(), "jacobi svd round");
      check_hip(hipMemcpyAsync(hrot.data(), rot.p, sizeof(int) * nsec, hipMemcpyDeviceToHost, st), "svd flag copy");
      check_hip(hipStreamSynchronize(st), "svd sweep");
      converged = true;
      for (int q = 0; q < nsec; ++q) {
        if (hrot[q] == 0) hdone[q] = 1;
        converged = converged && hdone[q];
      }
      if (!converged)
        check_hip(hipMemcpyAsync(done.p, hdone.data(), sizeof(int) * nsec, hipMemcpyHostToDevice, st), "svd flags");
    }
    if (!converged) throw Error{LCC_ERR_NAN, "Jacobi SVD did not converge in a sector (non-finite input?)"};
    hipLaunchKernelGGL(svd_finalize_kernel, dim3(nsec), dim3(kSvdThreads), 0, st, djobs.as<SvdJob>(), Wk.as<double>(),
                       Sv.as<double>(), V.as<double>(), U.as<double>());
    check_hip(hipGetLastError(), "jacobi svd finalize");
  }
  check_hip(hipMemcpyAsync(hs.data(), Sv.p, sizeof(double) * s_tot, hipMemcpyDeviceToHost, st), "sv copy");
  check_hip(hipStreamSynchronize(st), "svd");
  const float ms_svd = ms_since(t_start);
  // ---- global truncation: the m_max largest singular values; ties by sector (N, 2Sz), then index
  struct Cand { double v; int q, i; };
  std::vector<Cand> cand;
  for (int q = 0; q < nsec; ++q)
    for (int i = 0; i < sp[q].r; ++i) cand.push_back(Cand{hs[sp[q].s_off + i], q, i});
  std::stable_sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) {
    if (a.v != b.v) return a.v > b.v;
    if (a.q != b.q) return a.q < b.q;
    return a.i < b.i;
  });
  std::vector<int> keep(nsec, 0);
  double total = 0, kept_w = 0, largest_dropped = 0;
  for (size_t c = 0; c < cand.size(); ++c) {
    total += cand[c].v * cand[c].v;
    if ((int)c < m_max && cand[c].v > 0.0) {
      keep[cand[c].q] = std::max(keep[cand[c].q], cand[c].i + 1);
      kept_w += cand[c].v * cand[c].v;
    } else if (largest_dropped == 0.0) {
      largest_dropped = cand[c].v;
    }
  }
  S.last_sv.clear();
  for (const Cand& c : cand) S.last_sv.push_back(c.v);
  // ---- new bond l+1 and the left-canonical site tensor A_l
  Bond nb;
  std::vector<int> new_index(nsec, -1);
  for (int q = 0; q < nsec; ++q)
    if (keep[q] > 0) {
      new_index[q] = (int)nb.q.size();
      nb.index[E.sectors[q].q] = (int)nb.q.size();
      nb.q.push_back(E.sectors[q].q);
      nb.dim.push_back(keep[q]);
    }
  if (nb.q.empty()) throw Error{LCC_ERR_ARG, "the two-site tensor is zero"};
  DeviceMps one;
  one.K = K;
  one.bonds.resize(K + 1);
  one.bonds[S.site] = S.bl;
  one.bonds[S.site + 1] = nb;
  one.sites.resize(K);
  int64_t a_site = 0;
  std::vector<std::pair<int, int>> src;  // (sector, row) of each block
  for (int q = 0; q < nsec; ++q) {
    if (keep[q] == 0) continue;
    const MiddleSector& M = E.sectors[q];
    for (size_t i = 0; i < M.rows.size(); ++i) {
      const int a = M.rows[i].first, s1 = M.rows[i].second;
      SiteBlock b{a, s1, new_index[q], a_site, S.bl.dim[a], keep[q]};
      a_site += (int64_t)b.rows * b.cols;
      one.sites[S.site].push_back(b);
      src.push_back({q, (int)i});
    }
  }
  one.data.alloc(sizeof(double) * std::max<int64_t>(a_site, 1));
  for (size_t k = 0; k < src.size(); ++k) {
    const SiteBlock& b = one.sites[S.site][k];
    const MiddleSector& M = E.sectors[src[k].first];
    const Split& p = sp[src[k].first];
    // rows row_off .. row_off + M_a of the row-major nrows x r left-vector matrix, first keep columns
    check_hip(hipMemcpy2DAsync(one.data.as<double>() + b.off, sizeof(double) * b.cols,
                               V.as<double>() + p.v_off + (int64_t)M.row_off[src[k].second] * p.r, sizeof(double) * p.r,
                               sizeof(double) * b.cols, b.rows, hipMemcpyDeviceToDevice, st),
              "A block copy");
  }
  // ---- extend the left environment by the new site tensor
  const clk::time_point t_env = clk::now();
  Environment Lnew = left_step(S.L, one, S.site, mpo, st);
  // ---- next block (l+1, l+2)
  const int next = S.site + 1;
  std::unique_ptr<Env> nenv(make_env(S.ctx, mpo, next, nb, S.mps.bonds[next + 2], Lnew, S.R[next + 2]));
  const float ms_env = ms_since(t_env);
  const clk::time_point t_guess = clk::now();
  // ---- next guess: rows (q, s2) x cols (s3, c) = sum_b (S V^T)_q[:, (s2, b)] B_{l+2}^{s3}[b -> c]
  DevBuf C;
  std::vector<int64_t> c_off(nsec, -1);
  int64_t c_tot = 0;
  for (int q = 0; q < nsec; ++q)
    if (keep[q] > 0) {
      c_off[q] = c_tot;
      c_tot += (int64_t)keep[q] * E.sectors[q].ncols;
    }
  C.alloc(sizeof(double) * std::max<int64_t>(c_tot, 1));
  for (int q = 0; q < nsec; ++q) {
    if (keep[q] == 0) continue;
    const MiddleSector& M = E.sectors[q];
    const int64_t n = (int64_t)keep[q] * M.ncols;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(scale_rows_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, st, C.as<double>() + c_off[q],
                       U.as<double>() + sp[q].u_off, Sv.as<double>() + sp[q].s_off, keep[q], M.ncols, M.ncols);
  }
  check_hip(hipGetLastError(), "scale rows");
  S.guess.alloc(sizeof(double) * std::max<int64_t>(nenv->n_elements, 1));
  check_hip(launch_fill_f64(S.guess.as<double>(), nenv->n_elements, 0.0, st), "zero guess");
  {
    // site l+2 tensor blocks by (left sector b, s3)
    std::map<std::pair<int, int>, const SiteBlock*> B;
    for (const SiteBlock& b : S.mps.sites[next + 1]) B[{b.l, b.s}] = &b;
    GemmBuilder gb;
    for (const lcc_block_entry& e : nenv->layout) {
      // e.left = new sector index (q), e.s1 = s2, e.s2 = s3, e.right = c
      int q_old = -1;
      for (int q = 0; q < nsec; ++q)
        if (new_index[q] == e.left) q_old = q;
      const MiddleSector& M = E.sectors[q_old];
      const QN qc = S.mps.bonds[next + 2].q[e.right];
      const QN qb = qc - local_qn(e.s2);
      const int b = S.mps.bonds[next + 1].find(qb);
      if (b < 0) continue;
      auto it = B.find({b, e.s2});
      if (it == B.end()) continue;
      int col = -1;
      for (size_t j = 0; j < M.cols.size(); ++j)
        if (M.cols[j].first == e.s1 && M.cols[j].second == b) col = (int)j;
      if (col < 0) continue;
      const SiteBlock& Bb = *it->second;
      gb.group(BASE_Y, e.offset, e.ld, e.rows, e.cols, false);
      gb.term(BASE_X, c_off[q_old] + M.col_off[col], M.ncols, BASE_MPS, Bb.off, Bb.cols, Bb.rows, 1.0);
    }
    if (!gb.groups.empty()) {
      const std::vector<GemmLaunch> Ls = finalize(gb, false, false, st);
      Bases<double> bs{};
      bs.p[BASE_X] = C.as<double>();
      bs.p[BASE_MPS] = S.mps.data.as<double>();
      bs.p[BASE_Y] = S.guess.as<double>();
      run_gemm64(Ls, bs, st);
      check_hip(hipStreamSynchronize(st), "guess");
    }
  }
  S.have_guess = true;
  if (info) {
    *info = lcc_sweep_info{};
    info->site = S.site;
    info->kept = 0;
    for (int q = 0; q < nsec; ++q) info->kept += keep[q];
    info->n_singular = (int32_t)cand.size();
    info->discarded_weight = total > 0 ? (total - kept_w) / total : 0.0;
    info->largest_discarded = largest_dropped;
    info->ms_svd = ms_svd;
    info->ms_env = ms_env;
    info->ms_guess = ms_since(t_guess);
    info->ms_total = ms_since(t_start);
  }
  S.L = std::move(Lnew);
  S.bl = nb;
  S.env = std::move(nenv);
  S.site = next;
}

void sweep_copy_guess(Sweep& S, double* x) {
  hipStream_t st = S.ctx->stream;
  if (S.have_guess)
    check_hip(hipMemcpyAsync(x, S.guess.p, sizeof(double) * S.env->n_elements, hipMemcpyDeviceToDevice, st), "guess");
  else
    check_hip(launch_fill_f64(x, S.env->n_elements, 0.0, st), "zero guess");
  check_hip(hipStreamSynchronize(st), "guess sync");
}

const std::vector<double>& sweep_singular_values(Sweep& S) { return S.last_sv; }

}  // namespace lcc
