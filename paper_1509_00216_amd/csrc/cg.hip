// Device-side steps of the single-problem conjugate-gradient solve (Implementation section:
// the local problem is solved by CG).  Every scalar of the recurrence (alpha, beta, rho, the
// residual norms) lives in one CgScalars record in device memory.  Each vector update is fused
// with the dot product that follows it and with the scalar step that consumes that dot: the
// blocks of a launch write their partial sums, and the last block to arrive (an atomic ticket)
// adds them in block order -- a fixed order, so results repeat bit for bit -- and advances
// the record.  A plain iteration is then three small launches besides the operator product:
//   shift (+ projection) and p^T A p -> alpha;  x/d and r update and |r|^2 -> stop test, beta;
//   p update, which also writes the status words to mapped host memory.
// A halt word stops the recurrence on the device (converged, refresh due, or an error), so an
// iteration the host has already queued behind it changes nothing (its operator product is
// skipped through the run word); the host reads the status words one iteration late
// (solver.cpp).
#include <cmath>

#include "state.h"

namespace lcc {
namespace {

constexpr int kT = 256;
constexpr int kMaxBlocks = 1024;  // partial sums per fused launch (the context's dot_partial)
static_assert(kMaxBlocks <= kDotBlocks, "the partial-sum buffer holds kDotBlocks entries");

inline dim3 blocks_for(int64_t n) {
  int64_t b = (n + kT - 1) / kT;
  if (b > kMaxBlocks) b = kMaxBlocks;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// sum over the block, valid in thread 0
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();  // red may still be read from a previous call
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < kT / 64; ++i) r += red[i];
  return r;
}

// Partial sum of this block into partial[blockIdx.x]; returns true in thread 0 of the last
// block to arrive, with the total (partials added in block order) in *total.
__device__ bool grid_sum(double v, double* partial, uint32_t* ticket, double* total) {
  __shared__ double red[kT / 64];
  __shared__ int last;
  const double s = block_sum(v, red);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s;
    __threadfence();
    last = atomicAdd(ticket, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  double acc = 0.0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += kT) acc += __builtin_nontemporal_load(partial + i);
  acc = block_sum(acc, red);
  if (threadIdx.x != 0) return false;
  *ticket = 0;
  *total = acc;
  return true;
}

__device__ __forceinline__ void stop(CgScalars* S, int32_t halt) {
  S->halt = halt;
  S->run = 0;
}
__device__ __forceinline__ void fail(CgScalars* S, int code, int why) {
  stop(S, CG_HALT_ERROR);
  S->err = code;
  S->why = why;
}

// alpha = rho / p^T A p
__device__ __forceinline__ void alpha_step(CgScalars* S, double pAp) {
  S->pAp = pAp;
  if (S->halt) return;
  if (!isfinite(pAp)) return fail(S, LCC_ERR_NAN, CG_WHY_PAP_NAN);
  if (pAp <= 0.0) return fail(S, LCC_ERR_NOT_SPD, CG_WHY_PAP_NOT_POSITIVE);
  S->alpha = S->rho / pAp;
}

// After the residual update.  Low-precision recurrence (mixed): the residual is in units of the
// last true residual norm sc; a refresh is due once it has dropped by `delta` since the last
// refresh or below the tolerance.  FP64: converged once |r| <= tol |Q b|.  Without a
// preconditioner rho is |r|^2 and beta follows here; with one, cg_beta_kernel follows the dot
// r^T z.
__device__ __forceinline__ void after_r_step(CgScalars* S, double rrn, int mixed, int preconditioned) {
  S->rr_new = rrn;
  if (S->halt) return;
  S->iters += 1;
  if (!isfinite(rrn)) return fail(S, LCC_ERR_NAN, CG_WHY_RESIDUAL_NAN);
  if (mixed) {
    const double rn = sqrt(rrn) * S->sc;
    S->margin = rn / fmax(S->delta * S->rmax * S->sc, S->tol_bn);
    if (rn < S->delta * S->rmax * S->sc || rn <= S->tol_bn) return stop(S, CG_STOP);
  } else {
    S->margin = sqrt(rrn) / S->tol_bn;
  }
  S->rr = rrn;
  if (!mixed && sqrt(rrn) <= S->tol_bn) return stop(S, CG_STOP);
  if (!preconditioned) {
    S->beta = rrn / S->rho;
    S->rho = rrn;
  }
}

__global__ void cg_set_kernel(CgScalars* S, double rho, double rr, double rmax, double sc, double tol_bn,
                              double delta) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  S->rho = rho;
  S->rr = rr;
  S->rmax = rmax;
  S->sc = sc;
  S->tol_bn = tol_bn;
  S->delta = delta;
  S->margin = HUGE_VAL;
  S->halt = CG_RUNNING;
  S->run = 1;
  S->err = 0;
  S->why = 0;
}

__global__ void cg_reset_kernel(CgScalars* S) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  S->ticket = 0;
  S->iters = 0;
  S->margin = HUGE_VAL;
  S->halt = CG_RUNNING;
  S->run = 1;
  S->err = 0;
  S->why = 0;
}

__global__ void cg_after_r_kernel(CgScalars* S, int mixed, int preconditioned) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  after_r_step(S, S->rr_new, mixed, preconditioned);
}

__global__ void cg_beta_kernel(CgScalars* S) {
  if (blockIdx.x != 0 || threadIdx.x != 0 || S->halt) return;
  S->beta = S->rho_new / S->rho;
  S->rho = S->rho_new;
}

// Ap <- Ap - e0 p, then with v: c = v^T Ap (the projection follows in cg_project_kernel);
// without v: p^T Ap -> alpha.
template <class T>
__global__ void __launch_bounds__(kT) cg_shift_kernel(int64_t n, double e0, const T* __restrict__ p,
                                                      T* __restrict__ Ap, const T* __restrict__ v, CgScalars* S,
                                                      double* __restrict__ partial) {
  const T* w = v ? v : p;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const T a = (T)(-e0 * (double)p[i] + (double)Ap[i]);
    Ap[i] = a;
    s += (double)w[i] * (double)a;
  }
  double total;
  if (!grid_sum(s, partial, &S->ticket, &total)) return;
  if (v) S->c = total;
  else alpha_step(S, total);
}

// Ap <- Ap - c v (c from cg_shift_kernel), then p^T Ap -> alpha
template <class T>
__global__ void __launch_bounds__(kT) cg_project_kernel(int64_t n, const T* __restrict__ v, T* __restrict__ Ap,
                                                        const T* __restrict__ p, CgScalars* S,
                                                        double* __restrict__ partial) {
  const double c = S->c;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const double cv = c == 0.0 ? 0.0 : -c * (double)v[i];
    const T a = (T)(cv + (double)Ap[i]);
    Ap[i] = a;
    s += (double)p[i] * (double)a;
  }
  double total;
  if (grid_sum(s, partial, &S->ticket, &total)) alpha_step(S, total);
}

// s += alpha p, r -= alpha Ap, then |r|^2 -> the stop test and beta.  Nothing changes while the
// recurrence is halted (every block reads the halt word before the last block can change it).
template <class T>
__global__ void __launch_bounds__(kT) cg_update_kernel(int64_t n, const T* __restrict__ p, T* __restrict__ s_,
                                                       const T* __restrict__ Ap, T* __restrict__ r, CgScalars* S,
                                                       double* __restrict__ partial, int mixed, int preconditioned) {
  if (S->halt) return;
  const double a = S->alpha;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    s_[i] = (T)(a * (double)p[i] + (double)s_[i]);
    const T ri = (T)(-a * (double)Ap[i] + (double)r[i]);
    r[i] = ri;
    s += (double)ri * (double)ri;
  }
  double total;
  if (grid_sum(s, partial, &S->ticket, &total)) after_r_step(S, total, mixed, preconditioned);
}

// s += alpha p only (the step whose residual is recomputed from the solution)
template <class T>
__global__ void __launch_bounds__(kT) cg_solution_kernel(int64_t n, const T* __restrict__ p, T* __restrict__ s_,
                                                         const CgScalars* S) {
  if (S->halt) return;
  const double a = S->alpha;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    s_[i] = (T)(a * (double)p[i] + (double)s_[i]);
}

// p <- z + beta p (unless halted); block 0 writes the status to `post` (mapped host memory)
template <class T>
__global__ void __launch_bounds__(kT) cg_direction_kernel(int64_t n, const T* __restrict__ z, T* __restrict__ p,
                                                          const CgScalars* S, CgStatus* post) {
  const int32_t halted = S->halt;
  if (post && blockIdx.x == 0 && threadIdx.x == 0) {
    post->halt = halted;
    post->err = S->err;
    post->why = S->why;
    post->iters = S->iters;
    post->margin = S->margin;
  }
  if (halted) return;
  const double beta = S->beta;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const double by = beta == 0.0 ? 0.0 : beta * (double)p[i];
    p[i] = (T)((double)z[i] + by);
  }
}

// y <- y - c v with c = *cp (projection onto the complement of v)
template <class T>
__global__ void __launch_bounds__(kT) cg_deflate_kernel(int64_t n, const double* __restrict__ cp,
                                                        const T* __restrict__ v, T* __restrict__ y) {
  const double c = *cp;
  if (c == 0.0) return;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    y[i] = (T)(-c * (double)v[i] + (double)y[i]);
}

// copy of the record into mapped host memory
__global__ void cg_copy_kernel(const CgScalars* S, CgScalars* out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *out = *S;
}

}  // namespace

hipError_t launch_cg_set(CgScalars* S, double rho, double rr, double rmax, double sc, double tol_bn, double delta,
                         hipStream_t s) {
  hipLaunchKernelGGL(cg_set_kernel, dim3(1), dim3(64), 0, s, S, rho, rr, rmax, sc, tol_bn, delta);
  return hipGetLastError();
}
hipError_t launch_cg_reset(CgScalars* S, hipStream_t s) {
  hipLaunchKernelGGL(cg_reset_kernel, dim3(1), dim3(64), 0, s, S);
  return hipGetLastError();
}
hipError_t launch_cg_after_r(CgScalars* S, bool mixed, bool preconditioned, hipStream_t s) {
  hipLaunchKernelGGL(cg_after_r_kernel, dim3(1), dim3(64), 0, s, S, (int)mixed, (int)preconditioned);
  return hipGetLastError();
}
hipError_t launch_cg_beta(CgScalars* S, hipStream_t s) {
  hipLaunchKernelGGL(cg_beta_kernel, dim3(1), dim3(64), 0, s, S);
  return hipGetLastError();
}
hipError_t launch_cg_copy(const CgScalars* S, CgScalars* out, hipStream_t s) {
  hipLaunchKernelGGL(cg_copy_kernel, dim3(1), dim3(64), 0, s, S, out);
  return hipGetLastError();
}
template <class T>
hipError_t launch_cg_shift(int64_t n, double e0, const T* p, T* Ap, const T* v, CgScalars* S, double* partial,
                           hipStream_t s) {
  hipLaunchKernelGGL(cg_shift_kernel<T>, blocks_for(n), dim3(kT), 0, s, n, e0, p, Ap, v, S, partial);
  if (v) hipLaunchKernelGGL(cg_project_kernel<T>, blocks_for(n), dim3(kT), 0, s, n, v, Ap, p, S, partial);
  return hipGetLastError();
}
template <class T>
hipError_t launch_cg_update(int64_t n, const T* p, T* s_, const T* Ap, T* r, CgScalars* S, double* partial, bool mixed,
                            bool preconditioned, hipStream_t s) {
  hipLaunchKernelGGL(cg_update_kernel<T>, blocks_for(n), dim3(kT), 0, s, n, p, s_, Ap, r, S, partial, (int)mixed,
                     (int)preconditioned);
  return hipGetLastError();
}
template <class T>
hipError_t launch_cg_solution(int64_t n, const T* p, T* s_, const CgScalars* S, hipStream_t s) {
  hipLaunchKernelGGL(cg_solution_kernel<T>, blocks_for(n), dim3(kT), 0, s, n, p, s_, S);
  return hipGetLastError();
}
template <class T>
hipError_t launch_cg_direction(int64_t n, const T* z, T* p, const CgScalars* S, CgStatus* post, hipStream_t s) {
  hipLaunchKernelGGL(cg_direction_kernel<T>, blocks_for(n), dim3(kT), 0, s, n, z, p, S, post);
  return hipGetLastError();
}
template <class T>
hipError_t launch_cg_deflate(int64_t n, const double* c, const T* v, T* y, hipStream_t s) {
  hipLaunchKernelGGL(cg_deflate_kernel<T>, blocks_for(n), dim3(kT), 0, s, n, c, v, y);
  return hipGetLastError();
}

#define LCC_CG_INSTANTIATE(T)                                                                                      \
  template hipError_t launch_cg_shift<T>(int64_t, double, const T*, T*, const T*, CgScalars*, double*, hipStream_t); \
  template hipError_t launch_cg_update<T>(int64_t, const T*, T*, const T*, T*, CgScalars*, double*, bool, bool,     \
                                          hipStream_t);                                                             \
  template hipError_t launch_cg_solution<T>(int64_t, const T*, T*, const CgScalars*, hipStream_t);                  \
  template hipError_t launch_cg_direction<T>(int64_t, const T*, T*, const CgScalars*, CgStatus*, hipStream_t);      \
  template hipError_t launch_cg_deflate<T>(int64_t, const double*, const T*, T*, hipStream_t);
LCC_CG_INSTANTIATE(double)
LCC_CG_INSTANTIATE(float)
#undef LCC_CG_INSTANTIATE

}  // namespace lcc
