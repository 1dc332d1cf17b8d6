// Lowest eigenvalue of H_eff by Lanczos (the DMRG energy functional of the Implementation
// section) and event timing of the two apply phases.
#include <algorithm>
#include <cmath>
#include <vector>

#include "state.h"

namespace lcc {
namespace {

double dot(Env& env, const double* a, const double* b) {
  Context* c = env.ctx;
  hipStream_t st = c->stream;
  check_hip(launch_dot_f64(a, b, env.n_elements, c->dot_partial.as<double>(), c->dot_out.as<double>(), st), "dot");
  check_hip(hipMemcpyAsync(c->host_scalar, c->dot_out.p, sizeof(double), hipMemcpyDeviceToHost, st), "dot copy");
  check_hip(hipStreamSynchronize(st), "dot sync");
  return c->host_scalar[0];
}

// Eigen-decomposition of a small symmetric matrix by cyclic Jacobi rotations (host, k <= a
// few hundred), in place on caller storage: a (k x k, row-major) is destroyed, w receives the
// eigenvalues and the columns of v (row-major k x k) the eigenvectors.
void jacobi_eigen(double* a, int k, double* w, double* v) {
  for (int i = 0; i < k * k; ++i) v[i] = 0.0;
  for (int i = 0; i < k; ++i) v[(size_t)i * k + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) off += a[(size_t)p * k + q] * a[(size_t)p * k + q];
    if (off < 1e-30) break;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = a[(size_t)p * k + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = a[(size_t)p * k + p], aqq = a[(size_t)q * k + q];
        const double tau = (aqq - app) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int r = 0; r < k; ++r) {
          const double arp = a[(size_t)r * k + p], arq = a[(size_t)r * k + q];
          a[(size_t)r * k + p] = c * arp - s * arq;
          a[(size_t)r * k + q] = s * arp + c * arq;
        }
        for (int r = 0; r < k; ++r) {
          const double apr = a[(size_t)p * k + r], aqr = a[(size_t)q * k + r];
          a[(size_t)p * k + r] = c * apr - s * aqr;
          a[(size_t)q * k + r] = s * apr + c * aqr;
        }
        for (int r = 0; r < k; ++r) {
          const double vrp = v[(size_t)r * k + p], vrq = v[(size_t)r * k + q];
          v[(size_t)r * k + p] = c * vrp - s * vrq;
          v[(size_t)r * k + q] = s * vrp + c * vrq;
        }
      }
  }
  for (int i = 0; i < k; ++i) w[i] = a[(size_t)i * k + i];
}

}  // namespace

// Lanczos cycles with full re-orthogonalisation, each restarted from the Ritz vector of the
// previous one.  Returns true when ||H u - theta u|| <= tol max(1, |theta|).
namespace {
void no_callback(void*, const LaunchRef&) {}
}  // namespace

size_t lanczos_host_elems(int steps) {
  const size_t k = (size_t)std::max(steps, 1);
  return 2 * k * k + 3 * k;
}

int64_t lanczos_workspace_elems(const Env& env, int steps) {
  const int64_t n = env.n_elements;
  return n * (std::min<int64_t>(std::max(steps, 1), n) + 2);
}

bool lowest_eigenpair(Env& env, int steps, int max_restarts, double tol, uint64_t seed, double* x_io, double* theta,
                      double* residual) {
  if (steps < 1) throw Error{LCC_ERR_ARG, "steps must be >= 1"};
  DevBuf ws;
  ws.alloc(sizeof(double) * (size_t)lanczos_workspace_elems(env, steps));
  std::vector<double> host(lanczos_host_elems(steps));
  return lowest_eigenpair_in(env, steps, max_restarts, tol, seed, x_io, theta, residual, ws.as<double>(), host.data(),
                             false);
}

bool lowest_eigenpair_in(Env& env, int steps, int max_restarts, double tol, uint64_t seed, double* x_io,
                         double* theta, double* residual, double* workspace, double* host_ws, bool in_order) {
  hipStream_t st = env.ctx->stream;
  const int64_t n = env.n_elements;
  if (steps < 1) throw Error{LCC_ERR_ARG, "steps must be >= 1"};
  if (max_restarts < 1) throw Error{LCC_ERR_ARG, "max_restarts must be >= 1"};
  if (!(tol >= 0.0)) throw Error{LCC_ERR_ARG, "tol must be >= 0"};
  steps = (int)std::min<int64_t>(steps, n);
  // workspace: steps + 1 Krylov vectors, then w
  double* Q = workspace;
  double* w = workspace + (size_t)n * (steps + 1);
  auto apply = [&](const double* in, double* out) {
    if (in_order) apply_heff_each(env, LCC_FP64, in, out, no_callback, nullptr);  // no side streams
    else apply_heff(env, LCC_FP64, in, out);
  };
  double nrm = 0.0;
  if (x_io) {
    check_hip(hipMemcpyAsync(Q, x_io, sizeof(double) * n, hipMemcpyDeviceToDevice, st), "start vector");
    nrm = std::sqrt(dot(env, Q, Q));
    if (!std::isfinite(nrm)) throw Error{LCC_ERR_NAN, "non-finite start vector"};
  }
  if (nrm == 0.0) {
    check_hip(launch_random_fill_f64(Q, n, seed, st), "start vector");
    nrm = std::sqrt(dot(env, Q, Q));
  }
  check_hip(launch_axpby_f64(n, 0.0, Q, 1.0 / nrm, Q, st), "normalise");
  // host storage (lanczos_host_elems(steps) doubles): alpha, beta, T (overwritten by its
  // eigen-decomposition), eigenvalues, eigenvectors
  const size_t S = (size_t)steps;
  double* alpha = host_ws;
  double* beta = alpha + S;
  double* T = beta + S;
  double* ev = T + S * S;
  double* vec = ev + S;
  bool converged = false;
  for (int cycle = 0; cycle < max_restarts; ++cycle) {
    int k = 0;
    for (; k < steps; ++k) {
      double* qk = Q + (size_t)k * n;
      apply(qk, w);
      const double a = dot(env, qk, w);
      if (!std::isfinite(a)) throw Error{LCC_ERR_NAN, "non-finite Rayleigh quotient"};
      alpha[k] = a;
      // full re-orthogonalisation (twice) against every Krylov vector so far
      for (int pass = 0; pass < 2; ++pass)
        for (int i = 0; i <= k; ++i) {
          const double* qi = Q + (size_t)i * n;
          const double c = dot(env, qi, w);
          check_hip(launch_axpby_f64(n, -c, qi, 1.0, w, st), "reorth");
        }
      const double b = std::sqrt(dot(env, w, w));
      if (k + 1 == steps || b < 1e-12 * std::max(1.0, std::fabs(a))) {
        ++k;
        break;
      }
      beta[k] = b;
      // the next basis vector is written without reading its (uninitialised) slot
      check_hip(launch_axpby_f64(n, 1.0 / b, w, 0.0, Q + (size_t)(k + 1) * n, st), "next vector");
    }
    const int m = k;
    for (int i = 0; i < m * m; ++i) T[i] = 0.0;
    for (int i = 0; i < m; ++i) {
      T[(size_t)i * m + i] = alpha[i];
      if (i + 1 < m) T[(size_t)i * m + i + 1] = T[(size_t)(i + 1) * m + i] = beta[i];
    }
    jacobi_eigen(T, m, ev, vec);
    int lo = 0;
    for (int i = 1; i < m; ++i)
      if (ev[i] < ev[lo]) lo = i;
    // Ritz vector u = Q s (normalised) and its residual; the basis is free afterwards
    check_hip(launch_fill_f64(w, n, 0.0, st), "zero");
    for (int i = 0; i < m; ++i)
      check_hip(launch_axpby_f64(n, vec[(size_t)i * m + lo], Q + (size_t)i * n, 1.0, w, st), "ritz");
    const double un = std::sqrt(dot(env, w, w));
    check_hip(launch_axpby_f64(n, 0.0, w, 1.0 / un, w, st), "normalise ritz");
    double* hu = Q + (size_t)n;  // slot 1 (steps + 1 >= 2 slots)
    apply(w, hu);
    const double th = dot(env, w, hu);
    check_hip(launch_axpby_f64(n, -th, w, 1.0, hu, st), "residual");
    const double res = std::sqrt(dot(env, hu, hu));
    *theta = th;
    *residual = res;
    converged = res <= tol * std::max(1.0, std::fabs(th));
    check_hip(hipMemcpyAsync(Q, w, sizeof(double) * n, hipMemcpyDeviceToDevice, st), "restart vector");
    if (converged) break;
  }
  if (x_io) check_hip(hipMemcpyAsync(x_io, w, sizeof(double) * n, hipMemcpyDeviceToDevice, st), "ritz out");
  check_hip(hipStreamSynchronize(st), "lanczos");
  return converged;
}

void lowest_eigenvalue(Env& env, int steps, uint64_t seed, double* theta, double* residual) {
  (void)lowest_eigenpair(env, steps, 1, 0.0, seed, nullptr, theta, residual);
}

namespace {
struct LaunchTimer {
  hipStream_t st;
  std::vector<hipEvent_t> events;
  std::vector<LaunchRef> refs;
  size_t next = 0;
};
void record_after(void* u, const LaunchRef& r) {
  LaunchTimer* t = static_cast<LaunchTimer*>(u);
  if (t->next >= t->events.size()) {
    hipEvent_t e;
    check_hip(hipEventCreate(&e), "event");
    t->events.push_back(e);
  }
  check_hip(hipEventRecord(t->events[t->next], t->st), "record");
  if (t->refs.size() < t->events.size()) t->refs.push_back(r);
  ++t->next;
}
}  // namespace

std::vector<lcc_launch_profile> profile_launches(Env& env, int precision, const void* x, void* y, int reps) {
  if (reps < 1) throw Error{LCC_ERR_ARG, "reps must be >= 1"};
  LaunchTimer t;
  t.st = env.ctx->stream;
  hipEvent_t start;
  check_hip(hipEventCreate(&start), "event");
  std::vector<double> sum;
  for (int r = 0; r < reps; ++r) {
    t.next = 0;
    check_hip(hipEventRecord(start, t.st), "record");
    apply_heff_each(env, precision, x, y, record_after, &t);
    check_hip(hipEventSynchronize(t.events[t.next - 1]), "sync");
    sum.resize(t.next, 0.0);
    for (size_t i = 0; i < t.next; ++i) {
      float ms = 0;
      check_hip(hipEventElapsedTime(&ms, i == 0 ? start : t.events[i - 1], t.events[i]), "elapsed");
      sum[i] += ms;
    }
  }
  const double esz = precision == LCC_FP64 ? 8.0 : 4.0;
  std::vector<lcc_launch_profile> out;
  for (size_t i = 0; i < t.refs.size(); ++i) {
    lcc_launch_profile p{};
    p.phase = t.refs[i].phase;
    p.kind = t.refs[i].kind;
    if (t.refs[i].gemm) {
      const GemmLaunch& L = *t.refs[i].gemm;
      p.tile_m = kTileShapes[L.shape][0];
      p.tile_n = kTileShapes[L.shape][1];
      p.n_tiles = L.n_tiles;
      p.packed = L.packed[precision] ? 1 : 0;
      p.layout = (L.ta ? 1 : 0) | (L.tb ? 2 : 0);
      p.flops = L.flops;
      p.exec_flops = L.exec_flops[precision][L.packed[precision] ? 1 : 0];
      p.bytes = (L.elems_read + L.elems_written) * esz;
    } else {
      p.n_tiles = env.plan.n_reduce_tiles;
      p.bytes = (double)env.work_elems * esz + (double)env.n_elements * esz;
    }
    p.ms = (float)(sum[i] / reps);
    out.push_back(p);
  }
  for (hipEvent_t e : t.events) (void)hipEventDestroy(e);
  (void)hipEventDestroy(start);
  return out;
}

void profile_apply(Env& env, int precision, const void* x, void* y, int reps, float* ms1, float* ms2) {
  const std::vector<lcc_launch_profile> v = profile_launches(env, precision, x, y, reps);
  double a = 0, b = 0;
  for (const lcc_launch_profile& p : v) (p.phase == 1 ? a : b) += p.ms;
  *ms1 = (float)a;
  *ms2 = (float)b;
}

}  // namespace lcc
