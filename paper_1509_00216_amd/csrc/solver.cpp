// Local LCC solve on the device: Q (H_eff - e0) Q x = Q b by conjugate gradients
// (Implementation section), optionally as FP64 iterative refinement around a
// low-precision CG.  All dot products accumulate in FP64 and every scalar of the
// recurrences is FP64; only the operator products and the vector updates of the inner
// solve run in FP32.
#include <chrono>
#include <cmath>

#include "state.h"

namespace lcc {
namespace {

struct Ops {
  Env& env;
  hipStream_t st;
  int64_t n;
  double e0;
  const double* v64;   // may be null
  float* v32;          // FP32 copy of v (inner solve) or null
  int applies64 = 0, applies_low = 0;

  double dot64(const double* a, const double* b) {
    Context* c = env.ctx;
    check_hip(launch_dot_f64(a, b, n, c->dot_partial.as<double>(), c->dot_out.as<double>(), st), "dot");
    check_hip(hipMemcpyAsync(c->host_scalar, c->dot_out.p, sizeof(double), hipMemcpyDeviceToHost, st), "dot copy");
    check_hip(hipStreamSynchronize(st), "dot sync");
    return c->host_scalar[0];
  }
  double dot32(const float* a, const float* b) {
    Context* c = env.ctx;
    check_hip(launch_dot_f32(a, b, n, c->dot_partial.as<double>(), c->dot_out.as<double>(), st), "dot");
    check_hip(hipMemcpyAsync(c->host_scalar, c->dot_out.p, sizeof(double), hipMemcpyDeviceToHost, st), "dot copy");
    check_hip(hipStreamSynchronize(st), "dot sync");
    return c->host_scalar[0];
  }
  // z <- z - (v.z) v
  void project64(double* z) {
    if (!v64) return;
    const double c = dot64(v64, z);
    check_hip(launch_axpby_f64(n, -c, v64, 1.0, z, st), "project");
  }
  void project32(float* z) {
    if (!v32) return;
    const double c = dot32(v32, z);
    check_hip(launch_axpby_f32(n, -c, v32, 1.0, z, st), "project");
  }
  // out = Q (H - e0) Q in ; `in` is assumed to lie in range(Q) already (all iterates do)
  void A64(const double* in, double* out) {
    apply_heff(env, LCC_FP64, in, out);
    ++applies64;
    check_hip(launch_axpby_f64(n, -e0, in, 1.0, out, st), "shift");
    project64(out);
  }
  void A32(int prec, const float* in, float* out) {
    apply_heff(env, prec, in, out);
    ++applies_low;
    check_hip(launch_axpby_f32(n, -e0, in, 1.0, out, st), "shift");
    project32(out);
  }
};

bool finite(double v) { return std::isfinite(v); }

}  // namespace

lcc_status solve_local(Env& env, const lcc_solve_opts& o, const double* b, double e0, const double* v,
                       double* x, lcc_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = env.ctx->stream;
  const int64_t n = env.n_elements;
  const int prec = o.precision;
  const int max_iter = o.max_iter > 0 ? o.max_iter : 1000;
  const double tol = o.tol > 0 ? o.tol : 1e-10;
  const double inner_tol = o.inner_tol > 0 ? o.inner_tol : 0.1;
  const int max_outer = o.max_outer > 0 ? o.max_outer : 200;
  const int replace_every = o.replace_every > 0 ? o.replace_every : 50;
  if (prec != LCC_FP64 && prec != LCC_FP32 && prec != LCC_BF16X3) throw Error{LCC_ERR_ARG, "unknown precision"};
  if (o.preconditioner != 0 && o.preconditioner != 1) throw Error{LCC_ERR_ARG, "unknown preconditioner"};
  if (!finite(e0)) throw Error{LCC_ERR_NAN, "e0 is not finite"};
  const bool jacobi = o.preconditioner == 1;

  Ops ops{env, st, n, e0, v, nullptr};
  double* bq = env.w64[0].as<double>();
  double* r = env.w64[1].as<double>();
  double* p = env.w64[2].as<double>();
  double* Ap = env.w64[3].as<double>();

  // non-finite inputs
  {
    int* flag = env.flag.as<int>();
    check_hip(launch_fill_f32(reinterpret_cast<float*>(flag), 1, 0.0f, st), "flag clear");
    check_hip(launch_nonfinite_f64(b, n, flag, st), "nan check");
    check_hip(launch_nonfinite_f64(x, n, flag, st), "nan check");
    if (v) check_hip(launch_nonfinite_f64(v, n, flag, st), "nan check");
    int h = 0;
    check_hip(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st), "flag copy");
    check_hip(hipStreamSynchronize(st), "flag sync");
    if (h) throw Error{LCC_ERR_NAN, "non-finite value in b, x or v"};
  }
  // Jacobi preconditioner M^-1 = 1 / (diag(H_eff) - e0); positive whenever H_eff - e0 is positive definite
  double* z = r;  // preconditioned residual (the residual itself without a preconditioner)
  if (jacobi) {
    compute_diagonal(env);
    env.minv64.alloc(sizeof(double) * std::max<int64_t>(n, 1));
    env.minv32.alloc(sizeof(float) * std::max<int64_t>(n, 1));
    int* flag = env.flag.as<int>();
    check_hip(launch_fill_f32(reinterpret_cast<float*>(flag), 1, 0.0f, st), "flag clear");
    check_hip(launch_jacobi_inverse(n, env.diag64.as<double>(), e0, env.minv64.as<double>(), env.minv32.as<float>(),
                                    flag, st), "jacobi");
    int h = 0;
    check_hip(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st), "flag copy");
    check_hip(hipStreamSynchronize(st), "flag sync");
    if (h) throw Error{LCC_ERR_NOT_SPD, "diag(H_eff) - e0 has an entry <= 0: H_eff - e0 is not positive definite"};
    z = env.w64[4].as<double>();
  }
  // z = Q M^-1 r (kept in the range of Q, where every iterate lives)
  auto precondition64 = [&]() {
    if (!jacobi) return;
    check_hip(launch_mul_f64(n, env.minv64.as<double>(), r, z, st), "precondition");
    ops.project64(z);
  };
  // bq = Q b ; x <- Q x
  check_hip(hipMemcpyAsync(bq, b, sizeof(double) * n, hipMemcpyDeviceToDevice, st), "copy b");
  ops.project64(bq);
  ops.project64(x);
  const double bn = std::sqrt(ops.dot64(bq, bq));
  lcc_solve_info inf{};
  lcc_status status = LCC_OK;
  auto residual64 = [&]() {  // r = bq - A x, returns ||r||
    ops.A64(x, r);
    check_hip(launch_axpby_f64(n, 1.0, bq, -1.0, r, st), "residual");
    return std::sqrt(ops.dot64(r, r));
  };
  if (bn == 0.0) {
    check_hip(launch_fill_f64(x, n, 0.0, st), "zero x");
    check_hip(launch_fill_f64(r, n, 0.0, st), "zero r");
  } else if (prec == LCC_FP64) {
    // (preconditioned) conjugate gradients: rho = r^T z with z = Q M^-1 r (z = r without M)
    double rnorm = residual64();
    precondition64();
    check_hip(hipMemcpyAsync(p, z, sizeof(double) * n, hipMemcpyDeviceToDevice, st), "p = z");
    double rr = rnorm * rnorm;
    double rho = jacobi ? ops.dot64(r, z) : rr;
    int it = 0;
    while (std::sqrt(rr) > tol * bn) {
      if (it >= max_iter) { status = LCC_NOT_CONVERGED; break; }
      ops.A64(p, Ap);
      const double pAp = ops.dot64(p, Ap);
      if (!finite(pAp)) throw Error{LCC_ERR_NAN, "non-finite p^T A p"};
      if (pAp <= 0.0) throw Error{LCC_ERR_NOT_SPD, "p^T A p <= 0: Q (H_eff - e0) Q is not positive definite"};
      const double alpha = rho / pAp;
      check_hip(launch_axpby_f64(n, alpha, p, 1.0, x, st), "x update");
      ++it;
      double rr_new;
      if (it % replace_every == 0) {
        const double rn = residual64();
        rr_new = rn * rn;
      } else {
        check_hip(launch_axpby_f64(n, -alpha, Ap, 1.0, r, st), "r update");
        rr_new = ops.dot64(r, r);
      }
      if (!finite(rr_new)) throw Error{LCC_ERR_NAN, "non-finite residual"};
      precondition64();
      const double rho_new = jacobi ? ops.dot64(r, z) : rr_new;
      const double beta = rho_new / rho;
      check_hip(launch_axpby_f64(n, 1.0, z, beta, p, st), "p update");
      rr = rr_new;
      rho = rho_new;
    }
    inf.iterations = it;
    inf.outer = 1;
    residual64();
  } else {
    // FP64 iterative refinement with a low-precision CG for each correction
    ensure_fp32(env);
    float* r32 = env.w32[0].as<float>();
    float* d32 = env.w32[1].as<float>();
    float* p32 = env.w32[2].as<float>();
    float* Ap32 = env.w32[3].as<float>();
    float* v32 = nullptr;
    if (v) {
      v32 = env.w32[4].as<float>();
      check_hip(launch_convert_f64_f32(n, v, v32, st), "v32");
    }
    ops.v32 = v32;
    float* z32 = jacobi ? env.w32[5].as<float>() : r32;
    auto precondition32 = [&]() {
      if (!jacobi) return;
      check_hip(launch_mul_f32(n, env.minv32.as<float>(), r32, z32, st), "precondition");
      ops.project32(z32);
    };
    // Reliable-update CG: one low-precision Krylov recurrence, with the FP64 true residual
    // r = Q b - A x recomputed (and the accumulated correction folded into the FP64 x)
    // whenever the recurrence residual has dropped by `inner_tol` since the last refresh.
    // The search direction is kept across refreshes, so the iteration count stays close to
    // FP64 CG while almost every operator product runs in low precision.  The low-precision
    // vectors are kept in units of the last true residual norm (scale sc).
    int total_it = 0, outer = 0;
    double rnorm = residual64();
    if (rnorm > tol * bn) {
      double sc = rnorm;
      check_hip(launch_convert_f64_f32(n, r, r32, st), "r32");
      check_hip(launch_axpby_f32(n, 0.0, r32, 1.0 / sc, r32, st), "scale r32");
      check_hip(launch_fill_f32(d32, n, 0.0f, st), "d = 0");
      precondition32();
      check_hip(hipMemcpyAsync(p32, z32, sizeof(float) * n, hipMemcpyDeviceToDevice, st), "p = z");
      double rr = ops.dot32(r32, r32);
      double rho = jacobi ? ops.dot32(r32, z32) : rr;
      double rmax = std::sqrt(rr);
      while (true) {
        if (total_it >= max_iter || outer >= max_outer) { status = LCC_NOT_CONVERGED; break; }
        ops.A32(prec, p32, Ap32);
        const double pAp = ops.dot32(p32, Ap32);
        if (!finite(pAp)) throw Error{LCC_ERR_NAN, "non-finite p^T A p"};
        if (pAp <= 0.0) throw Error{LCC_ERR_NOT_SPD, "p^T A p <= 0: Q (H_eff - e0) Q is not positive definite"};
        const double alpha = rho / pAp;
        check_hip(launch_axpby_f32(n, alpha, p32, 1.0, d32, st), "d update");
        check_hip(launch_axpby_f32(n, -alpha, Ap32, 1.0, r32, st), "r update");
        double rr_new = ops.dot32(r32, r32);
        if (!finite(rr_new)) throw Error{LCC_ERR_NAN, "non-finite residual"};
        ++total_it;
        const double rn = std::sqrt(rr_new) * sc;
        double p_scale = 1.0;
        if (rn < inner_tol * rmax * sc || rn <= tol * bn) {
          // refresh: x += sc d (FP64), true residual in FP64, continue in the new units
          check_hip(launch_axpy_f32_into_f64(n, sc, d32, x, st), "x += d");
          ops.project64(x);
          check_hip(launch_fill_f32(d32, n, 0.0f, st), "d = 0");
          rnorm = residual64();
          ++outer;
          if (rnorm <= tol * bn) break;
          const double sc_new = rnorm;
          check_hip(launch_convert_f64_f32(n, r, r32, st), "r32");
          check_hip(launch_axpby_f32(n, 0.0, r32, 1.0 / sc_new, r32, st), "scale r32");
          // beta from the refreshed residual (rho in true units); p rescaled to the new units
          precondition32();
          const double rho_new_units = jacobi ? ops.dot32(r32, z32) : ops.dot32(r32, r32);
          const double beta = (rho_new_units * sc_new * sc_new) / (rho * sc * sc);
          p_scale = beta * sc / sc_new;
          check_hip(launch_axpby_f32(n, 1.0, z32, p_scale, p32, st), "p update");
          sc = sc_new;
          rr = ops.dot32(r32, r32);
          rho = rho_new_units;
          rmax = std::sqrt(rr);
          continue;
        }
        precondition32();
        const double rho_new = jacobi ? ops.dot32(r32, z32) : rr_new;
        check_hip(launch_axpby_f32(n, 1.0, z32, rho_new / rho, p32, st), "p update");
        rr = rr_new;
        rho = rho_new;
      }
      if (status == LCC_NOT_CONVERGED) {
        check_hip(launch_axpy_f32_into_f64(n, sc, d32, x, st), "x += d");
        ops.project64(x);
        rnorm = residual64();
      }
    }
    inf.iterations = total_it;
    inf.outer = outer;
  }
  // energy from the last FP64 residual r = bq - A x:  J = x^T A x - 2 bq^T x = -x^T r - bq^T x
  const double xr = ops.dot64(x, r);
  const double bx = ops.dot64(bq, x);
  const double rn = std::sqrt(ops.dot64(r, r));
  inf.rel_residual = bn > 0 ? rn / bn : 0.0;
  inf.hylleraas = -xr - bx;
  inf.e2 = -bx;
  inf.applies_fp64 = ops.applies64;
  inf.applies_low = ops.applies_low;
  inf.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  return status;
}

}  // namespace lcc
