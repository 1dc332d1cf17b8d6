// Local LCC solve on the device: Q (H_eff - e0) Q x = Q b by conjugate gradients
// (Implementation section), optionally as FP64 iterative refinement around a
// low-precision CG.  All dot products accumulate in FP64 and every scalar of the
// recurrences is FP64; only the operator products and the vector updates of the inner
// solve run in FP32.
//
// Inside an iteration nothing returns to the host.  The scalars live in a CgScalars record in
// device memory, and each vector update is fused with the dot product after it and the scalar
// step that uses it (cg.hip): an iteration is the operator product plus three small launches,
// and the low-precision iteration is replayed from a captured graph.
// The last of them writes the status words to mapped host memory; after queueing iteration
// i the host waits for the status of iteration i-1, so the device has the next iteration
// queued (near the end of the recurrence it waits for iteration i itself).  The device halts the recurrence itself (converged, refresh due, error),
// which makes the iteration queued behind the halt change nothing; its operator product
// returns at once.  Refreshes of the mixed solve (FP64 residual, rescaling) and the final
// energy read scalars back synchronously; they happen a few times per solve.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>

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
  CgScalars* S;        // device record of the recurrence
  int applies64 = 0, applies_low = 0;

  double* partial() const { return env.ctx->dot_partial.as<double>(); }
  // dot products read back to the host through mapped memory (set-up, refreshes, final energy)
  double dot64(const double* a, const double* b) {
    Context* c = env.ctx;
    check_hip(launch_dot_f64(a, b, n, partial(), c->host_scalar_dev, st), "dot");
    check_hip(hipStreamSynchronize(st), "dot sync");
    return c->host_scalar[0];
  }
  double dot32(const float* a, const float* b) {
    Context* c = env.ctx;
    check_hip(launch_dot_f32(a, b, n, partial(), c->host_scalar_dev, st), "dot");
    check_hip(hipStreamSynchronize(st), "dot sync");
    return c->host_scalar[0];
  }
  // z <- z - (v.z) v, with v.z kept on the device
  void project64(double* z) {
    if (!v64) return;
    check_hip(launch_dot_f64(v64, z, n, partial(), &S->c, st), "dot");
    check_hip(launch_cg_deflate<double>(n, &S->c, v64, z, st), "project");
  }
  void project32(float* z) {
    if (!v32) return;
    check_hip(launch_dot_f32(v32, z, n, partial(), &S->c, st), "dot");
    check_hip(launch_cg_deflate<float>(n, &S->c, v32, z, st), "project");
  }
  // out = Q (H - e0) Q in ; `in` is assumed to lie in range(Q) already (all iterates do)
  void A64(const double* in, double* out, bool guarded = false) {
    apply_heff(env, LCC_FP64, in, out, guarded ? &S->run : nullptr);
    ++applies64;
    check_hip(launch_axpby_f64(n, -e0, in, 1.0, out, st), "shift");
    project64(out);
  }
  // Ap = Q (H - e0) p and alpha = rho / p^T Ap on the device; the product is skipped while the
  // recurrence is halted
  void Ap64(const double* p, double* Ap) {
    apply_heff(env, LCC_FP64, p, Ap, &S->run);
    ++applies64;
    check_hip(launch_cg_shift<double>(n, e0, p, Ap, v64, S, partial(), st), "shift, p^T A p");
  }
};

// Status of the recurrence.  The direction update of every iteration posts a CgStatus into
// one of two mapped slots.  Before queueing the next iteration the host waits for the
// iteration before the last one queued, so that the device keeps one iteration in its queue.
// An iteration queued behind a halt does nothing, but still dispatches the launches of its
// operator product; so when the last status seen puts the residual within a few of its
// latest per-iteration drops of the threshold that stops the recurrence, the host waits for
// the last iteration as well.
struct StatusPoll {
  static constexpr double kSafety = 2.0;  // drops larger than kSafety x the last one are rare
  hipStream_t st;
  Context* ctx;
  const CgScalars* S;
  int64_t posted = 0;
  int64_t seen = -1;    // last iteration whose status was read
  double margin = 0.0;  // its margin
  bool near = true;     // no status seen yet
  CgStatus* slot_dev() { return reinterpret_cast<CgStatus*>(ctx->host_scalar_dev + 4) + (posted & 1); }
  void posted_one() {
    check_hip(hipEventRecord(ctx->ev_status[posted & 1], st), "status event");
    ++posted;
  }
  // waits for the status of queued iteration k (0-based since the last now()); true if halted
  bool halted_at(int64_t k) {
    if (k == seen) return false;
    check_hip(hipEventSynchronize(ctx->ev_status[k & 1]), "status wait");
    const CgStatus& s = reinterpret_cast<const CgStatus*>(ctx->host_scalar + 4)[k & 1];
    if (s.halt != CG_RUNNING) return true;
    const double drop = seen == k - 1 && s.margin > 0.0 ? std::max(margin / s.margin, 1.0) : HUGE_VAL;
    near = s.margin < kSafety * drop;
    seen = k;
    margin = s.margin;
    return false;
  }
  // true when the recurrence has halted (queue nothing more)
  bool halted() {
    if (posted >= 2 && halted_at(posted - 2)) return true;
    return near && halted_at(posted - 1);
  }
  // all queued work done: the record as the device holds it now; the next post starts anew
  CgScalars now() {
    CgScalars* whole = reinterpret_cast<CgScalars*>(ctx->host_scalar + 12);
    check_hip(launch_cg_copy(S, reinterpret_cast<CgScalars*>(ctx->host_scalar_dev + 12), st), "record copy");
    check_hip(hipStreamSynchronize(st), "record sync");
    posted = 0;
    seen = -1;
    near = true;
    return *whole;
  }
};

[[noreturn]] void raise_halt(const CgScalars& w) {
  const int code = w.err, why = w.why;
  if (why == CG_WHY_PAP_NAN) throw Error{code, "non-finite p^T A p"};
  if (why == CG_WHY_PAP_NOT_POSITIVE) throw Error{code, "p^T A p <= 0: Q (H_eff - e0) Q is not positive definite"};
  if (why == CG_WHY_RESIDUAL_NAN) throw Error{code, "non-finite residual"};
  throw Error{code, "conjugate gradients stopped with status " + std::to_string(code)};
}

bool finite(double v) { return std::isfinite(v); }

}  // namespace

lcc_status solve_local(Env& env, const lcc_solve_opts& o, const double* b, double e0, const double* v,
                       double* x, lcc_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  Context* ctx = env.ctx;
  hipStream_t st = ctx->stream;
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

  if (!env.cg.p) env.cg.alloc(sizeof(CgScalars));
  CgScalars* S = env.cg.as<CgScalars>();
  for (int k = 0; k < 2; ++k)
    if (!ctx->ev_status[k]) check_hip(hipEventCreateWithFlags(&ctx->ev_status[k], hipEventDisableTiming), "event");
  StatusPoll poll{st, ctx, S};
  check_hip(launch_cg_reset(S, st), "cg reset");

  Ops ops{env, st, n, e0, v, nullptr, S};
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
  // r = bq - A x (queued only)
  auto residual64_queue = [&]() {
    ops.A64(x, r);
    check_hip(launch_axpby_f64(n, 1.0, bq, -1.0, r, st), "residual");
  };
  auto residual64 = [&]() {  // r = bq - A x, returns ||r||
    residual64_queue();
    return std::sqrt(ops.dot64(r, r));
  };
  if (bn == 0.0) {
    check_hip(launch_fill_f64(x, n, 0.0, st), "zero x");
    check_hip(launch_fill_f64(r, n, 0.0, st), "zero r");
  } else if (prec == LCC_FP64) {
    // (preconditioned) conjugate gradients: rho = r^T z with z = Q M^-1 r (z = r without M)
    const double rnorm = residual64();
    precondition64();
    check_hip(hipMemcpyAsync(p, z, sizeof(double) * n, hipMemcpyDeviceToDevice, st), "p = z");
    const double rr = rnorm * rnorm;
    const double rho = jacobi ? ops.dot64(r, z) : rr;
    if (std::sqrt(rr) > tol * bn) {
      check_hip(launch_cg_set(S, rho, rr, 0.0, 1.0, tol * bn, 0.0, st), "cg set");
      for (int it = 0; it < max_iter; ++it) {
        ops.Ap64(p, Ap);
        if ((it + 1) % replace_every == 0) {
          // x += alpha p, then the true residual replaces the recurrence one (after a halt the
          // recomputed r is discarded: the final residual is formed again below)
          check_hip(launch_cg_solution<double>(n, p, x, S, st), "x update");
          ops.A64(x, r, true);
          check_hip(launch_axpby_f64(n, 1.0, bq, -1.0, r, st), "residual");
          check_hip(launch_dot_f64(r, r, n, ops.partial(), &S->rr_new, st), "dot");
          check_hip(launch_cg_after_r(S, false, jacobi, st), "after r");
        } else {
          check_hip(launch_cg_update<double>(n, p, x, Ap, r, S, ops.partial(), false, jacobi, st), "x, r update");
        }
        if (jacobi) {
          precondition64();
          check_hip(launch_dot_f64(r, z, n, ops.partial(), &S->rho_new, st), "dot");
          check_hip(launch_cg_beta(S, st), "beta");
        }
        check_hip(launch_cg_direction<double>(n, z, p, S, poll.slot_dev(), st), "p update");
        poll.posted_one();
        if (poll.halted()) break;
      }
      const CgScalars w = poll.now();
      if (w.halt == CG_HALT_ERROR) raise_halt(w);
      if (w.halt != CG_STOP) status = LCC_NOT_CONVERGED;
      inf.iterations = w.iters;
    }
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
      check_hip(launch_cg_set(S, rho, rr, std::sqrt(rr), sc, tol * bn, inner_tol, st), "cg set");
      // One low-precision iteration (operator product, update, direction), posting its status to
      // slot k.  It reads and writes only the environment's own buffers and CG record, so it is
      // captured as a graph once per slot and replayed, in this and later solves, until
      // something it baked in changes.
      // recorded on the graph stream gs: the context stream may be the legacy default stream,
      // which cannot be captured; launches inside go to ctx->stream, pointed at gs meanwhile
      if (!ctx->graph_stream) check_hip(hipStreamCreateWithFlags(&ctx->graph_stream, hipStreamNonBlocking), "stream");
      if (!ctx->ev_gate) check_hip(hipEventCreateWithFlags(&ctx->ev_gate, hipEventDisableTiming), "event");
      hipStream_t gs = ctx->graph_stream;
      poll.st = gs;  // status events, record copies and waits follow the iterations onto gs
      auto iteration = [&](int k) {
        apply_heff(env, prec, p32, Ap32, &S->run);
        check_hip(launch_cg_shift<float>(n, e0, p32, Ap32, v32, S, ops.partial(), gs), "shift, p^T A p");
        check_hip(launch_cg_update<float>(n, p32, d32, Ap32, r32, S, ops.partial(), true, jacobi, gs),
                  "d, r update");
        if (jacobi) {  // z = Q M^-1 r, rho_new = r^T z
          check_hip(launch_mul_f32(n, env.minv32.as<float>(), r32, z32, gs), "precondition");
          if (v32) {
            check_hip(launch_dot_f32(v32, z32, n, ops.partial(), &S->c, gs), "dot");
            check_hip(launch_cg_deflate<float>(n, &S->c, v32, z32, gs), "project");
          }
          check_hip(launch_dot_f32(r32, z32, n, ops.partial(), &S->rho_new, gs), "dot");
          check_hip(launch_cg_beta(S, gs), "beta");
        }
        check_hip(launch_cg_direction<float>(n, z32, p32, S, reinterpret_cast<CgStatus*>(ctx->host_scalar_dev + 4) + k,
                                             gs),
                  "p update");
      };
      CgGraph& G = env.cg_graph;
      uint64_t e0_bits;
      std::memcpy(&e0_bits, &e0, sizeof e0_bits);  // e0 is an argument of the shift launch
      const std::vector<uintptr_t> key = {
          (uintptr_t)e0_bits, (uintptr_t)n, (uintptr_t)prec, (uintptr_t)jacobi, (uintptr_t)env.plan_epoch, (uintptr_t)ctx->overlap, (uintptr_t)gs,
          (uintptr_t)p32, (uintptr_t)Ap32, (uintptr_t)d32, (uintptr_t)r32, (uintptr_t)z32, (uintptr_t)v32,
          (uintptr_t)env.minv32.p, (uintptr_t)env.env32.p, (uintptr_t)env.merged32.p, (uintptr_t)env.tbuf.p,
          (uintptr_t)env.work.p, (uintptr_t)S, (uintptr_t)ctx->host_scalar_dev, (uintptr_t)ops.partial()};
      if (G.key != key) {
        G.release();
        for (int k = 0; k < 2; ++k) {
          check_hip(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal), "begin capture");
          hipGraph_t graph = nullptr;
          ctx->stream = gs;
          try {
            iteration(k);
          } catch (...) {
            ctx->stream = st;
            (void)hipStreamEndCapture(gs, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipGetLastError();
            throw;
          }
          ctx->stream = st;
          check_hip(hipStreamEndCapture(gs, &graph), "end capture");
          const hipError_t e = hipGraphInstantiate(&G.exec[k], graph, nullptr, nullptr, 0);
          (void)hipGraphDestroy(graph);
          check_hip(e, "instantiate");
        }
        G.key = key;
      }
      while (true) {
        // low-precision iterations, until the device halts the recurrence (refresh due,
        // converged, error) or max_iter iterations have run
        // the iterations run on gs, after the work queued on the context stream
        check_hip(hipEventRecord(ctx->ev_gate, st), "gate");
        check_hip(hipStreamWaitEvent(gs, ctx->ev_gate, 0), "gate wait");
        for (; total_it < max_iter; ++total_it) {
          check_hip(hipGraphLaunch(G.exec[poll.posted & 1], gs), "iteration");
          ++ops.applies_low;
          poll.posted_one();
          if (poll.halted()) break;
        }
        const CgScalars w = poll.now();
        if (w.halt == CG_HALT_ERROR) raise_halt(w);
        total_it = w.iters;  // iterations the device performed (a queued one behind a halt does nothing)
        rho = w.rho;         // rho of the last completed iteration
        if (w.halt != CG_STOP) { status = LCC_NOT_CONVERGED; break; }
        // refresh: x += sc d (FP64), true residual in FP64, continue in the new units
        check_hip(launch_axpy_f32_into_f64(n, sc, d32, x, st), "x += d");
        ops.project64(x);
        check_hip(launch_fill_f32(d32, n, 0.0f, st), "d = 0");
        rnorm = residual64();
        ++outer;
        if (rnorm <= tol * bn) break;
        if (total_it >= max_iter || outer >= max_outer) { status = LCC_NOT_CONVERGED; break; }
        const double sc_new = rnorm;
        check_hip(launch_convert_f64_f32(n, r, r32, st), "r32");
        check_hip(launch_axpby_f32(n, 0.0, r32, 1.0 / sc_new, r32, st), "scale r32");
        // beta from the refreshed residual (rho in true units); p rescaled to the new units
        precondition32();
        rr = ops.dot32(r32, r32);
        const double rho_new_units = jacobi ? ops.dot32(r32, z32) : rr;
        const double beta = (rho_new_units * sc_new * sc_new) / (rho * sc * sc);
        check_hip(launch_axpby_f32(n, 1.0, z32, beta * sc / sc_new, p32, st), "p update");
        sc = sc_new;
        rho = rho_new_units;
        check_hip(launch_cg_set(S, rho, rr, std::sqrt(rr), sc, tol * bn, inner_tol, st), "cg set");
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
