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
constexpr double kSvCut = 1e-10;  // singular values below kSvCut * the largest count as zero
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

// Environments of one operator between the sweep's MPS (the bra) and a ket: the reference MPS
// of a first-order problem (transition families) or the sweep's own MPS.
struct Family {
  Mpo own;                        // the identity operator of the overlap family
  const Mpo* mpo = nullptr;
  bool transition = false;
  std::vector<Environment> L, R;  // L[j], R[j]: environments at MPS bond j
};

struct Sweep {
  Context* ctx = nullptr;
  int K = 0, N = 0, two_sz = 0;
  std::vector<Bond> bonds;     // current bonds of the MPS
  std::vector<DeviceMps> t;    // site tensors, one buffer each; t[site], t[site+1] are the block's
  Family h;                    // the operator of the local problem
  int site = 0, first = 0;
  std::unique_ptr<Env> env;
  DevBuf guess;      // initial guess of the current local problem (n_elements), valid if have_guess
  bool have_guess = false;
  std::vector<double> last_sv;  // singular values of the last split, descending
  // first-order problems: the reference MPS and the operator O of the right-hand side (transition
  // families), the overlap with the reference, and the perturbation U on the sweep's own MPS
  bool have_ref = false;
  DeviceMps ref;
  Family op, ov, u;
  bool have_u = false;
  std::unique_ptr<Env> env_op, env_ov, env_u;
};

namespace {

// Site j of an MPS as a one-site MPS with its own buffer (bonds j and j + 1 set).
DeviceMps site_copy(const DeviceMps& m, int j, hipStream_t st) {
  DeviceMps o;
  o.K = m.K;
  o.bonds.resize(m.K + 1);
  o.bonds[j] = m.bonds[j];
  o.bonds[j + 1] = m.bonds[j + 1];
  o.sites.resize(m.K);
  int64_t tot = 0;
  for (const SiteBlock& b : m.sites[j]) {
    SiteBlock c = b;
    c.off = tot;
    tot += (int64_t)b.rows * b.cols;
    o.sites[j].push_back(c);
  }
  o.data.alloc(sizeof(double) * std::max<int64_t>(tot, 1));
  for (size_t i = 0; i < m.sites[j].size(); ++i)
    check_hip(hipMemcpyAsync(o.data.as<double>() + o.sites[j][i].off, m.data.as<double>() + m.sites[j][i].off,
                             sizeof(double) * (size_t)m.sites[j][i].rows * m.sites[j][i].cols, hipMemcpyDeviceToDevice,
                             st),
              "site copy");
  return o;
}

const DeviceMps& ket_of(const Sweep& S, const Family& f, int j) { return f.transition ? S.ref : S.t[j]; }

// L[j + 1] from L[j] and the site tensor t[j]
void extend_left(Sweep& S, Family& f, int j) {
  f.L[j + 1] = left_step(f.L[j], S.t[j], ket_of(S, f, j), j, *f.mpo, S.ctx->stream);
}
// R[j] from R[j + 1] and the site tensor t[j]
void extend_right(Sweep& S, Family& f, int j) {
  f.R[j] = right_step(f.R[j + 1], S.t[j], ket_of(S, f, j), j, *f.mpo, S.ctx->stream);
}

// a family's environments left and right of the current block
void build_family(Sweep& S, Family& f) {
  hipStream_t st = S.ctx->stream;
  f.L.clear();
  f.R.clear();
  f.L.resize(S.K + 1);
  f.R.resize(S.K + 1);
  f.L[0] = unit_env(st);
  for (int j = 0; j < S.site; ++j) extend_left(S, f, j);
  f.R[S.K] = unit_env(st);
  for (int j = S.K - 1; j >= S.site + 2; --j) extend_right(S, f, j);
}

void drop_block_envs(Sweep& S) {
  S.env_op.reset();
  S.env_ov.reset();
  S.env_u.reset();
}

// The split of the solved two-site tensor: per middle-bond sector an SVD (singular values
// descending at s_off; left vectors as a row-major nrows x r matrix at v_off; right vectors as a
// row-major r x ncols matrix at u_off; r = min(nrows, ncols)), and the global truncation to the
// m_max largest singular values (ties by sector (N, 2Sz), then index).
struct SplitSector {
  int r;
  int64_t s_off, u_off, v_off;
};
struct SplitResult {
  std::vector<SplitSector> sp;
  DevBuf Sv, U, V;
  std::vector<int> keep;      // kept singular vectors per sector
  Bond nb;                    // the new bond: the sectors with keep > 0
  std::vector<int> new_index; // sector -> index in nb (-1 if dropped)
  std::vector<double> sv;     // all singular values, descending
  double total = 0, kept_w = 0, largest_dropped = 0;
  float ms_svd = 0;
};

SplitResult split_block(Sweep& S, const double* x, int m_max) {
  hipStream_t st = S.ctx->stream;
  typedef std::chrono::steady_clock clk;
  const clk::time_point t_start = clk::now();
  Env& E = *S.env;
  const int nsec = (int)E.sectors.size();
  SplitResult out;
  std::vector<SplitSector>& sp = out.sp;
  sp.resize(nsec);
  std::vector<SvdJob> jobs(nsec);
  int64_t s_tot = 0, u_tot = 0, v_tot = 0, w_tot = 0;
  for (int q = 0; q < nsec; ++q) {
    const MiddleSector& M = E.sectors[q];
    SplitSector& p = sp[q];
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
  DevBuf Wk, rot, done, djobs, dslots;
  out.Sv.alloc(sizeof(double) * std::max<int64_t>(s_tot, 1));
  out.U.alloc(sizeof(double) * std::max<int64_t>(u_tot, 1));
  out.V.alloc(sizeof(double) * std::max<int64_t>(v_tot, 1));
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
                       out.Sv.as<double>(), out.V.as<double>(), out.U.as<double>());
    check_hip(hipGetLastError(), "jacobi svd finalize");
  }
  check_hip(hipMemcpyAsync(hs.data(), out.Sv.p, sizeof(double) * s_tot, hipMemcpyDeviceToHost, st), "sv copy");
  check_hip(hipStreamSynchronize(st), "svd");
  out.ms_svd = (float)std::chrono::duration<double, std::milli>(clk::now() - t_start).count();
  struct Cand { double v; int q, i; };
  std::vector<Cand> cand;
  for (int q = 0; q < nsec; ++q)
    for (int i = 0; i < sp[q].r; ++i) cand.push_back(Cand{hs[sp[q].s_off + i], q, i});
  std::stable_sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) {
    if (a.v != b.v) return a.v > b.v;
    if (a.q != b.q) return a.q < b.q;
    return a.i < b.i;
  });
  out.keep.assign(nsec, 0);
  // singular values at the rounding level of the largest are zeros of the exact tensor: their
  // vectors are not determined (one-sided Jacobi forms them as W / sigma), so they are never kept
  const double cut = kSvCut * (cand.empty() ? 0.0 : cand[0].v);
  for (size_t c = 0; c < cand.size(); ++c) {
    out.total += cand[c].v * cand[c].v;
    if ((int)c < m_max && cand[c].v > cut) {
      out.keep[cand[c].q] = std::max(out.keep[cand[c].q], cand[c].i + 1);
      out.kept_w += cand[c].v * cand[c].v;
    } else if (out.largest_dropped == 0.0) {
      out.largest_dropped = cand[c].v;
    }
  }
  for (const Cand& c : cand) out.sv.push_back(c.v);
  out.new_index.assign(nsec, -1);
  for (int q = 0; q < nsec; ++q)
    if (out.keep[q] > 0) {
      out.new_index[q] = (int)out.nb.q.size();
      out.nb.index[E.sectors[q].q] = (int)out.nb.q.size();
      out.nb.q.push_back(E.sectors[q].q);
      out.nb.dim.push_back(out.keep[q]);
    }
  if (out.nb.q.empty()) throw Error{LCC_ERR_ARG, "the two-site tensor is zero"};
  return out;
}

void fill_info(const SplitResult& R, int site, float ms_env, float ms_guess, float ms_total, lcc_sweep_info* info) {
  if (!info) return;
  *info = lcc_sweep_info{};
  info->site = site;
  info->kept = 0;
  for (int k : R.keep) info->kept += k;
  info->n_singular = (int32_t)R.sv.size();
  info->discarded_weight = R.total > 0 ? (R.total - R.kept_w) / R.total : 0.0;
  info->largest_discarded = R.largest_dropped;
  info->ms_svd = R.ms_svd;
  info->ms_env = ms_env;
  info->ms_guess = ms_guess;
  info->ms_total = ms_total;
}

// dst[i*keep + k] = src[i*ld + k] * s[k]  (i < rows, k < keep)
__global__ void scale_cols_kernel(double* __restrict__ dst, const double* __restrict__ src, const double* __restrict__ s,
                                  int rows, int keep, int ld) {
  const int64_t n = (int64_t)rows * keep;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / keep), k = (int)(e % keep);
    dst[e] = src[(int64_t)i * ld + k] * s[k];
  }
}

}  // namespace

Sweep* sweep_create(Context* ctx, const Hamiltonian& ham, const lcc_mps_desc& md, int first) {
  hipStream_t st = ctx->stream;
  const Mpo& mpo = ham.mpo;
  const int K = mpo.K;
  if (md.n_sites != K) throw Error{LCC_ERR_ARG, "MPS length differs from the Hamiltonian's orbital count"};
  if (first < 0 || first + 1 >= K) throw Error{LCC_ERR_ARG, "first two-site block must satisfy 0 <= site < K-1"};
  std::unique_ptr<Sweep> S(new Sweep());
  S->ctx = ctx;
  S->K = K;
  S->N = ham.desc.N;
  S->two_sz = ham.desc.two_sz;
  S->first = S->site = first;
  DeviceMps mps;
  load_mps(md, ham.desc.N, ham.desc.two_sz, st, mps);
  S->bonds = mps.bonds;
  for (int j = 0; j < K; ++j) S->t.push_back(site_copy(mps, j, st));
  check_hip(hipStreamSynchronize(st), "site copies");
  S->h.mpo = &mpo;
  build_family(*S, S->h);
  const int wl = channel_of_kind(mpo, first, 0), wr = channel_of_kind(mpo, first + 2, 1);
  if (first > 0 && wl >= 0) check_identity(S->h.L[first], wl, S->bonds[first], st, "left");
  if (first + 2 < K && wr >= 0) check_identity(S->h.R[first + 2], wr, S->bonds[first + 2], st, "right");
  S->env.reset(make_env(ctx, mpo, first, S->bonds[first], S->bonds[first + 2], S->h.L[first], S->h.R[first + 2]));
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
  const Mpo& mpo = *S.h.mpo;
  const int K = S.K;
  if (S.site + 2 >= K) throw Error{LCC_ERR_STATE, "the sweep is already at the last two-site block"};
  if (m_max < 1) throw Error{LCC_ERR_ARG, "m_max must be >= 1"};
  Env& E = *S.env;
  const int nsec = (int)E.sectors.size();
  SplitResult R = split_block(S, x, m_max);
  S.last_sv = R.sv;
  const std::vector<int>& keep = R.keep;
  // ---- new bond l+1 and the left-canonical site tensor A_l (left vectors, first keep columns)
  const int l = S.site;
  DeviceMps one;
  one.K = K;
  one.bonds.resize(K + 1);
  one.bonds[l] = S.bonds[l];
  one.bonds[l + 1] = R.nb;
  one.sites.resize(K);
  int64_t a_site = 0;
  std::vector<std::pair<int, int>> src;  // (sector, row) of each block
  for (int q = 0; q < nsec; ++q) {
    if (keep[q] == 0) continue;
    const MiddleSector& M = E.sectors[q];
    for (size_t i = 0; i < M.rows.size(); ++i) {
      const int a = M.rows[i].first, s1 = M.rows[i].second;
      SiteBlock b{a, s1, R.new_index[q], a_site, S.bonds[l].dim[a], keep[q]};
      a_site += (int64_t)b.rows * b.cols;
      one.sites[l].push_back(b);
      src.push_back({q, (int)i});
    }
  }
  one.data.alloc(sizeof(double) * std::max<int64_t>(a_site, 1));
  for (size_t k = 0; k < src.size(); ++k) {
    const SiteBlock& b = one.sites[l][k];
    const MiddleSector& M = E.sectors[src[k].first];
    const SplitSector& p = R.sp[src[k].first];
    check_hip(hipMemcpy2DAsync(one.data.as<double>() + b.off, sizeof(double) * b.cols,
                               R.V.as<double>() + p.v_off + (int64_t)M.row_off[src[k].second] * p.r, sizeof(double) * p.r,
                               sizeof(double) * b.cols, b.rows, hipMemcpyDeviceToDevice, st),
              "A block copy");
  }
  // ---- extend the left environments by the new site tensor
  const clk::time_point t_env = clk::now();
  S.t[l] = std::move(one);
  S.bonds[l + 1] = R.nb;
  extend_left(S, S.h, l);
  if (S.have_ref) {
    extend_left(S, S.op, l);
    extend_left(S, S.ov, l);
    if (S.have_u) extend_left(S, S.u, l);
  }
  drop_block_envs(S);
  // ---- next block (l+1, l+2)
  const int next = l + 1;
  std::unique_ptr<Env> nenv(make_env(S.ctx, mpo, next, R.nb, S.bonds[next + 2], S.h.L[next], S.h.R[next + 2]));
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
                       R.U.as<double>() + R.sp[q].u_off, R.Sv.as<double>() + R.sp[q].s_off, keep[q], M.ncols, M.ncols);
  }
  check_hip(hipGetLastError(), "scale rows");
  S.guess.alloc(sizeof(double) * std::max<int64_t>(nenv->n_elements, 1));
  check_hip(launch_fill_f64(S.guess.as<double>(), nenv->n_elements, 0.0, st), "zero guess");
  {
    const DeviceMps& B3 = S.t[next + 1];  // site l+2 blocks by (left sector b, s3)
    std::map<std::pair<int, int>, const SiteBlock*> B;
    for (const SiteBlock& b : B3.sites[next + 1]) B[{b.l, b.s}] = &b;
    GemmBuilder gb;
    for (const lcc_block_entry& e : nenv->layout) {
      // e.left = new sector index (q), e.s1 = s2, e.s2 = s3, e.right = c
      int q_old = -1;
      for (int q = 0; q < nsec; ++q)
        if (R.new_index[q] == e.left) q_old = q;
      const MiddleSector& M = E.sectors[q_old];
      const QN qc = S.bonds[next + 2].q[e.right];
      const QN qb = qc - local_qn(e.s2);
      const int b = S.bonds[next + 1].find(qb);
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
      bs.p[BASE_MPS] = B3.data.as<double>();
      bs.p[BASE_Y] = S.guess.as<double>();
      run_gemm64(Ls, bs, st);
    }
    check_hip(hipStreamSynchronize(st), "guess");
  }
  S.have_guess = true;
  fill_info(R, l, ms_env, ms_since(t_guess), ms_since(t_start), info);
  S.env = std::move(nenv);
  S.site = next;
}

// The mirror of sweep_advance: the right vectors of the split become the right-canonical tensor
// of site l+1, the right environments are extended by it, and A_{l-1} contracted with U S is the
// initial guess of the local problem at (l-1, l).
void sweep_retreat(Sweep& S, const double* x, int m_max, lcc_sweep_info* info) {
  hipStream_t st = S.ctx->stream;
  typedef std::chrono::steady_clock clk;
  const auto ms_since = [](clk::time_point t) {
    return (float)std::chrono::duration<double, std::milli>(clk::now() - t).count();
  };
  const clk::time_point t_start = clk::now();
  const Mpo& mpo = *S.h.mpo;
  const int K = S.K;
  if (S.site == 0) throw Error{LCC_ERR_STATE, "the sweep is already at the first two-site block"};
  if (m_max < 1) throw Error{LCC_ERR_ARG, "m_max must be >= 1"};
  Env& E = *S.env;
  const int nsec = (int)E.sectors.size();
  SplitResult R = split_block(S, x, m_max);
  S.last_sv = R.sv;
  const std::vector<int>& keep = R.keep;
  const int l = S.site;
  // ---- new bond l+1 and the right-canonical site tensor B_{l+1} (right vectors, first keep rows)
  DeviceMps one;
  one.K = K;
  one.bonds.resize(K + 1);
  one.bonds[l + 1] = R.nb;
  one.bonds[l + 2] = S.bonds[l + 2];
  one.sites.resize(K);
  int64_t b_site = 0;
  std::vector<std::pair<int, int>> src;  // (sector, column block) of each block
  for (int q = 0; q < nsec; ++q) {
    if (keep[q] == 0) continue;
    const MiddleSector& M = E.sectors[q];
    for (size_t i = 0; i < M.cols.size(); ++i) {
      const int s2 = M.cols[i].first, b = M.cols[i].second;
      SiteBlock sb{R.new_index[q], s2, b, b_site, keep[q], S.bonds[l + 2].dim[b]};
      b_site += (int64_t)sb.rows * sb.cols;
      one.sites[l + 1].push_back(sb);
      src.push_back({q, (int)i});
    }
  }
  one.data.alloc(sizeof(double) * std::max<int64_t>(b_site, 1));
  for (size_t k = 0; k < src.size(); ++k) {
    const SiteBlock& b = one.sites[l + 1][k];
    const MiddleSector& M = E.sectors[src[k].first];
    const SplitSector& p = R.sp[src[k].first];
    // rows 0 .. keep of the row-major r x ncols right-vector matrix, columns col_off .. + M_b
    check_hip(hipMemcpy2DAsync(one.data.as<double>() + b.off, sizeof(double) * b.cols,
                               R.U.as<double>() + p.u_off + M.col_off[src[k].second], sizeof(double) * M.ncols,
                               sizeof(double) * b.cols, b.rows, hipMemcpyDeviceToDevice, st),
              "B block copy");
  }
  const clk::time_point t_env = clk::now();
  S.t[l + 1] = std::move(one);
  S.bonds[l + 1] = R.nb;
  extend_right(S, S.h, l + 1);
  if (S.have_ref) {
    extend_right(S, S.op, l + 1);
    extend_right(S, S.ov, l + 1);
    if (S.have_u) extend_right(S, S.u, l + 1);
  }
  drop_block_envs(S);
  // ---- previous block (l-1, l)
  const int prev = l - 1;
  std::unique_ptr<Env> nenv(make_env(S.ctx, mpo, prev, S.bonds[prev], R.nb, S.h.L[prev], S.h.R[l + 1]));
  const float ms_env = ms_since(t_env);
  const clk::time_point t_guess = clk::now();
  // ---- guess: rows (a'', s0) x cols (s1, q) = sum_a A_{l-1}^{s0}[a'' -> a] (U S)_q[(a, s1), :]
  DevBuf C;
  std::vector<int64_t> c_off(nsec, -1);
  int64_t c_tot = 0;
  for (int q = 0; q < nsec; ++q)
    if (keep[q] > 0) {
      c_off[q] = c_tot;
      c_tot += (int64_t)E.sectors[q].nrows * keep[q];
    }
  C.alloc(sizeof(double) * std::max<int64_t>(c_tot, 1));
  for (int q = 0; q < nsec; ++q) {
    if (keep[q] == 0) continue;
    const MiddleSector& M = E.sectors[q];
    const int64_t n = (int64_t)M.nrows * keep[q];
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(scale_cols_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, st, C.as<double>() + c_off[q],
                       R.V.as<double>() + R.sp[q].v_off, R.Sv.as<double>() + R.sp[q].s_off, M.nrows, keep[q], R.sp[q].r);
  }
  check_hip(hipGetLastError(), "scale cols");
  S.guess.alloc(sizeof(double) * std::max<int64_t>(nenv->n_elements, 1));
  check_hip(launch_fill_f64(S.guess.as<double>(), nenv->n_elements, 0.0, st), "zero guess");
  {
    const DeviceMps& A0 = S.t[prev];  // site l-1 blocks by (left sector a'', s0)
    std::map<std::pair<int, int>, const SiteBlock*> A;
    for (const SiteBlock& b : A0.sites[prev]) A[{b.l, b.s}] = &b;
    GemmBuilder gb;
    for (const lcc_block_entry& e : nenv->layout) {
      // e.left = a'' (bond l-1), e.s1 = s0, e.s2 = s1, e.right = new sector index (q)
      int q_old = -1;
      for (int q = 0; q < nsec; ++q)
        if (R.new_index[q] == e.right) q_old = q;
      const MiddleSector& M = E.sectors[q_old];
      auto it = A.find({e.left, e.s1});
      if (it == A.end()) continue;
      const SiteBlock& Ab = *it->second;  // a'' -> a on bond l
      int row = -1;
      for (size_t i = 0; i < M.rows.size(); ++i)
        if (M.rows[i].first == Ab.r && M.rows[i].second == e.s2) row = (int)i;
      if (row < 0) continue;
      gb.group(BASE_Y, e.offset, e.ld, e.rows, e.cols, false);
      gb.term(BASE_MPS, Ab.off, Ab.cols, BASE_X, c_off[q_old] + (int64_t)M.row_off[row] * keep[q_old], keep[q_old],
              Ab.cols, 1.0);
    }
    if (!gb.groups.empty()) {
      const std::vector<GemmLaunch> Ls = finalize(gb, false, false, st);
      Bases<double> bs{};
      bs.p[BASE_X] = C.as<double>();
      bs.p[BASE_MPS] = A0.data.as<double>();
      bs.p[BASE_Y] = S.guess.as<double>();
      run_gemm64(Ls, bs, st);
    }
    check_hip(hipStreamSynchronize(st), "guess");
  }
  S.have_guess = true;
  fill_info(R, l, ms_env, ms_since(t_guess), ms_since(t_start), info);
  S.env = std::move(nenv);
  S.site = prev;
}

// Split the block tensor x in place (no move): site l gets the left-canonical factor, site l+1
// the right factor scaled by the singular values, bond l+1 the kept states.  The environments
// and the local problem of the block stay as they are.
void sweep_split_block(Sweep& S, const double* x, int m_max, lcc_sweep_info* info) {
  hipStream_t st = S.ctx->stream;
  typedef std::chrono::steady_clock clk;
  const clk::time_point t_start = clk::now();
  if (m_max < 1) throw Error{LCC_ERR_ARG, "m_max must be >= 1"};
  const int K = S.K, l = S.site;
  Env& E = *S.env;
  const int nsec = (int)E.sectors.size();
  SplitResult R = split_block(S, x, m_max);
  S.last_sv = R.sv;
  const std::vector<int>& keep = R.keep;
  DeviceMps a, b;
  a.K = b.K = K;
  a.bonds.resize(K + 1);
  b.bonds.resize(K + 1);
  a.bonds[l] = S.bonds[l];
  a.bonds[l + 1] = R.nb;
  b.bonds[l + 1] = R.nb;
  b.bonds[l + 2] = S.bonds[l + 2];
  a.sites.resize(K);
  b.sites.resize(K);
  int64_t na = 0, nb = 0;
  for (int q = 0; q < nsec; ++q) {
    if (keep[q] == 0) continue;
    const MiddleSector& M = E.sectors[q];
    for (size_t i = 0; i < M.rows.size(); ++i) {
      SiteBlock sb{M.rows[i].first, M.rows[i].second, R.new_index[q], na, S.bonds[l].dim[M.rows[i].first], keep[q]};
      na += (int64_t)sb.rows * sb.cols;
      a.sites[l].push_back(sb);
    }
    for (size_t i = 0; i < M.cols.size(); ++i) {
      SiteBlock sb{R.new_index[q], M.cols[i].first, M.cols[i].second, nb, keep[q], S.bonds[l + 2].dim[M.cols[i].second]};
      nb += (int64_t)sb.rows * sb.cols;
      b.sites[l + 1].push_back(sb);
    }
  }
  a.data.alloc(sizeof(double) * std::max<int64_t>(na, 1));
  b.data.alloc(sizeof(double) * std::max<int64_t>(nb, 1));
  // S V^T of each kept sector (keep x ncols, row-major)
  DevBuf C;
  std::vector<int64_t> c_off(nsec, -1);
  int64_t c_tot = 0;
  for (int q = 0; q < nsec; ++q)
    if (keep[q] > 0) {
      c_off[q] = c_tot;
      c_tot += (int64_t)keep[q] * E.sectors[q].ncols;
    }
  C.alloc(sizeof(double) * std::max<int64_t>(c_tot, 1));
  size_t ia = 0, ib = 0;
  for (int q = 0; q < nsec; ++q) {
    if (keep[q] == 0) continue;
    const MiddleSector& M = E.sectors[q];
    const SplitSector& p = R.sp[q];
    const int64_t n = (int64_t)keep[q] * M.ncols;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(scale_rows_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, st, C.as<double>() + c_off[q],
                       R.U.as<double>() + p.u_off, R.Sv.as<double>() + p.s_off, keep[q], M.ncols, M.ncols);
    for (size_t i = 0; i < M.rows.size(); ++i, ++ia) {
      const SiteBlock& sb = a.sites[l][ia];
      check_hip(hipMemcpy2DAsync(a.data.as<double>() + sb.off, sizeof(double) * sb.cols,
                                 R.V.as<double>() + p.v_off + (int64_t)M.row_off[i] * p.r, sizeof(double) * p.r,
                                 sizeof(double) * sb.cols, sb.rows, hipMemcpyDeviceToDevice, st),
                "A block copy");
    }
    for (size_t i = 0; i < M.cols.size(); ++i, ++ib) {
      const SiteBlock& sb = b.sites[l + 1][ib];
      check_hip(hipMemcpy2DAsync(b.data.as<double>() + sb.off, sizeof(double) * sb.cols,
                                 C.as<double>() + c_off[q] + M.col_off[i], sizeof(double) * M.ncols,
                                 sizeof(double) * sb.cols, sb.rows, hipMemcpyDeviceToDevice, st),
                "SV block copy");
    }
  }
  check_hip(hipGetLastError(), "split block");
  check_hip(hipStreamSynchronize(st), "split block");
  S.t[l] = std::move(a);
  S.t[l + 1] = std::move(b);
  S.bonds[l + 1] = R.nb;
  fill_info(R, l, 0.f, 0.f,
            (float)std::chrono::duration<double, std::milli>(clk::now() - t_start).count(), info);
}

const Bond& sweep_bond(const Sweep& S, int j) {
  if (j < 0 || j > S.K) throw Error{LCC_ERR_ARG, "bond index out of range"};
  return S.bonds[j];
}

const DeviceMps& sweep_site_tensor(const Sweep& S, int j) {
  if (j < 0 || j >= S.K) throw Error{LCC_ERR_ARG, "site index out of range"};
  return S.t[j];
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

int sweep_site(const Sweep& S) { return S.site; }

// ---------------------------------------------------------------------------------------
// First-order problems (Theory section, the first-order equation): the reference MPS Phi0 and
// the operator O of the right-hand side -Q O Phi0 (O = U; O = H for the projector approximation),
// the overlap with Phi0, and optionally U on the sweep's own MPS for the third-order energy.
// ---------------------------------------------------------------------------------------
void sweep_attach_reference(Sweep& S, const Hamiltonian& op, const Hamiltonian* u, const lcc_mps_desc& ref) {
  hipStream_t st = S.ctx->stream;
  if (op.mpo.K != S.K || (u && u->mpo.K != S.K) || ref.n_sites != S.K)
    throw Error{LCC_ERR_ARG, "the operators and the reference MPS must have the sweep's orbital count"};
  if (op.desc.N != S.N || op.desc.two_sz != S.two_sz || (u && (u->desc.N != S.N || u->desc.two_sz != S.two_sz)))
    throw Error{LCC_ERR_QN, "the operators must act in the sweep's (N, 2Sz) sector"};
  S.have_ref = false;
  drop_block_envs(S);
  DeviceMps r;
  load_mps(ref, S.N, S.two_sz, st, r);
  S.ref = std::move(r);
  S.op = Family();
  S.op.mpo = &op.mpo;
  S.op.transition = true;
  S.ov = Family();
  {
    // the identity operator through the MPO compiler: no integrals, constant 1
    HamDesc id;
    id.K = S.K;
    id.N = S.N;
    id.two_sz = S.two_sz;
    id.h.assign((size_t)S.K * S.K, 0.0);
    id.e_const = 1.0;
    id.switch_bond = -1;
    const std::string err = build_mpo(id, S.ov.own);
    if (!err.empty()) throw Error{LCC_ERR_STATE, "identity operator: " + err};
  }
  S.ov.mpo = &S.ov.own;
  S.ov.transition = true;
  build_family(S, S.op);
  build_family(S, S.ov);
  S.have_u = u != nullptr;
  S.u = Family();
  if (u) {
    S.u.mpo = &u->mpo;
    build_family(S, S.u);
  }
  S.have_ref = true;
}

namespace {
Env* transition_block(Sweep& S, Family& f) {
  const int l = S.site;
  std::unique_ptr<Env> e(make_env(S.ctx, *f.mpo, l, S.bonds[l], S.bonds[l + 2], S.ref.bonds[l], S.ref.bonds[l + 2],
                                  f.L[l], f.R[l + 2], true));
  build_ket_tensor(*e, S.ref, S.ref, S.ctx->stream);
  return e.release();
}
double dot_dev(Context* c, const double* a, const double* b, int64_t n) {
  hipStream_t st = c->stream;
  check_hip(launch_dot_f64(a, b, n, c->dot_partial.as<double>(), c->dot_out.as<double>(), st), "dot");
  check_hip(hipMemcpyAsync(c->host_scalar, c->dot_out.p, sizeof(double), hipMemcpyDeviceToHost, st), "dot copy");
  check_hip(hipStreamSynchronize(st), "dot sync");
  return c->host_scalar[0];
}
}  // namespace

// b = -(P^T O Phi0 - c v) with v = P^T Phi0 (P: the environment basis of the current block);
// v is returned scaled to norm 1 (as the solver's projection takes it) and |v| in *v_norm
void sweep_first_order_rhs(Sweep& S, double c, double* b, double* v, double* v_norm) {
  if (!S.have_ref) throw Error{LCC_ERR_STATE, "no reference MPS attached to the sweep"};
  hipStream_t st = S.ctx->stream;
  if (!S.env_op) S.env_op.reset(transition_block(S, S.op));
  if (!S.env_ov) S.env_ov.reset(transition_block(S, S.ov));
  const int64_t n = S.env->n_elements;
  if (S.env_op->n_elements != n || S.env_ov->n_elements != n)
    throw Error{LCC_ERR_STATE, "internal: block layouts of the sweep and its transition operators differ"};
  apply_heff(*S.env_ov, LCC_FP64, S.env_ov->x0.p, v);
  apply_heff(*S.env_op, LCC_FP64, S.env_op->x0.p, b);
  // b = -b + c v
  check_hip(launch_axpby_f64(n, c, v, -1.0, b, st), "rhs");
  const double nv = std::sqrt(std::max(0.0, dot_dev(S.ctx, v, v, n)));
  if (nv > 0.0) check_hip(launch_axpby_f64(n, 0.0, v, 1.0 / nv, v, st), "normalise v");
  check_hip(hipStreamSynchronize(st), "rhs");
  *v_norm = nv;
}

// x^T U_eff x and x^T x of the current block's tensor
void sweep_u_expectation(Sweep& S, const double* x, double* xux, double* xx) {
  if (!S.have_ref || !S.have_u) throw Error{LCC_ERR_STATE, "no perturbation operator attached to the sweep"};
  const int l = S.site;
  if (!S.env_u) S.env_u.reset(make_env(S.ctx, *S.u.mpo, l, S.bonds[l], S.bonds[l + 2], S.u.L[l], S.u.R[l + 2]));
  const int64_t n = S.env->n_elements;
  DevBuf y;
  y.alloc(sizeof(double) * std::max<int64_t>(n, 1));
  apply_heff(*S.env_u, LCC_FP64, x, y.p);
  *xux = dot_dev(S.ctx, x, y.as<double>(), n);
  *xx = dot_dev(S.ctx, x, x, n);
}

}  // namespace lcc
