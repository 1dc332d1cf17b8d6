// C ABI entry points: argument checks, error capture, and dispatch into the planner,
// kernels and solver.  No exception crosses this boundary.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "state.h"

using namespace lcc;

namespace {

std::mutex g_err_mu;
std::string g_last_error;

lcc_status fail(lcc_context ctx, lcc_status code, const std::string& msg) {
  if (ctx) ctx->c.err = msg;
  std::lock_guard<std::mutex> lk(g_err_mu);
  g_last_error = msg;
  return code;
}

template <class F>
lcc_status guarded(lcc_context ctx, F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    return fail(ctx, e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(ctx, LCC_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(ctx, LCC_ERR_ARG, e.what());
  } catch (...) {
    return fail(ctx, LCC_ERR_ARG, "unknown failure");
  }
}

void require_device(lcc_context ctx) {
  if (!ctx || ctx->c.device < 0) throw Error{LCC_ERR_STATE, "this call needs a context on a device"};
  check_hip(hipSetDevice(ctx->c.device), "hipSetDevice");
}

}  // namespace

extern "C" {

lcc_status lcc_context_create(int32_t device, void* stream, lcc_context* out) {
  if (!out) return fail(nullptr, LCC_ERR_ARG, "out is NULL");
  *out = nullptr;
  return guarded(nullptr, [&]() -> lcc_status {
    std::unique_ptr<lcc_context_s> c(new lcc_context_s());
    c->c.device = device;
    c->c.handle = c.get();
    if (device >= 0) {
      int n = 0;
      if (hipGetDeviceCount(&n) != hipSuccess || device >= n) {
        (void)hipGetLastError();
        throw Error{LCC_ERR_NODEV, "no HIP device " + std::to_string(device)};
      }
      hipDeviceProp_t prop;
      check_hip(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
      if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        throw Error{LCC_ERR_NODEV, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950"};
      check_hip(hipSetDevice(device), "hipSetDevice");
      scratch_register_current_device();
      c->c.stream = static_cast<hipStream_t>(stream);
      c->c.dot_partial.alloc(sizeof(double) * kDotBlocks);
      c->c.dot_out.alloc(sizeof(double) * 8);
      check_hip(hipHostMalloc(reinterpret_cast<void**>(&c->c.host_scalar), sizeof(double) * kHostScalars,
                              hipHostMallocMapped | hipHostMallocCoherent),
                "hipHostMalloc");
      check_hip(hipHostGetDevicePointer(reinterpret_cast<void**>(&c->c.host_scalar_dev), c->c.host_scalar, 0),
                "hipHostGetDevicePointer");
    }
    *out = c.release();
    return LCC_OK;
  });
}

void lcc_context_destroy(lcc_context ctx) {
  if (!ctx) return;
  if (ctx->c.device >= 0) {
    (void)hipSetDevice(ctx->c.device);
    if (ctx->c.stream) (void)hipStreamSynchronize(ctx->c.stream);
    if (ctx->c.host_scalar) (void)hipHostFree(ctx->c.host_scalar);
    for (hipStream_t s : ctx->c.side) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
    for (hipEvent_t e : ctx->c.ev_join) (void)hipEventDestroy(e);
    if (ctx->c.ev_fork) (void)hipEventDestroy(ctx->c.ev_fork);
    for (hipEvent_t e : ctx->c.ev_status)
      if (e) (void)hipEventDestroy(e);
    if (ctx->c.ev_gate) (void)hipEventDestroy(ctx->c.ev_gate);
    if (ctx->c.graph_stream) {
      (void)hipStreamSynchronize(ctx->c.graph_stream);
      (void)hipStreamDestroy(ctx->c.graph_stream);
    }
    if (ctx->c.own_stream) (void)hipStreamDestroy(ctx->c.stream);
  }
  delete ctx;
}

const char* lcc_last_error(lcc_context ctx) {
  if (ctx) return ctx->c.err.c_str();
  std::lock_guard<std::mutex> lk(g_err_mu);
  return g_last_error.c_str();
}

lcc_status lcc_context_synchronize(lcc_context ctx) {
  return guarded(ctx, [&]() -> lcc_status {
    require_device(ctx);
    check_hip(hipStreamSynchronize(ctx->c.stream), "hipStreamSynchronize");
    return LCC_OK;
  });
}

lcc_status lcc_context_set_intermediate_limit(lcc_context ctx, int64_t bytes) {
  if (!ctx) return fail(nullptr, LCC_ERR_ARG, "ctx is NULL");
  if (bytes < 8) return fail(ctx, LCC_ERR_ARG, "limit must hold at least one element");
  ctx->c.t_budget_elems = bytes / 8;
  return LCC_OK;
}

lcc_status lcc_context_set_overlap(lcc_context ctx, int32_t side_streams) {
  if (!ctx) return fail(nullptr, LCC_ERR_ARG, "ctx is NULL");
  if (side_streams < 0 || side_streams > 8) return fail(ctx, LCC_ERR_ARG, "side_streams must be in [0, 8]");
  return guarded(ctx, [&]() -> lcc_status {
    if (ctx->c.device >= 0) check_hip(hipSetDevice(ctx->c.device), "hipSetDevice");
    for (hipStream_t s : ctx->c.side) check_hip(hipStreamSynchronize(s), "side stream sync");
    ctx->c.overlap = side_streams;
    return LCC_OK;
  });
}

lcc_status lcc_context_set_plan(lcc_context ctx, double tile_overhead, int64_t split_k, int32_t p2_order,
                                int32_t t_colmajor) {
  if (!ctx) return fail(nullptr, LCC_ERR_ARG, "ctx is NULL");
  if (!(tile_overhead >= 0) || split_k < 1 || (p2_order != 0 && p2_order != 1) || t_colmajor < 0 || t_colmajor > 2)
    return fail(ctx, LCC_ERR_ARG, "invalid planner parameters");
  ctx->c.plan_params.tile_overhead = tile_overhead;
  ctx->c.plan_params.split_k = split_k;
  ctx->c.plan_params.p2_order = p2_order;
  ctx->c.plan_params.t_colmajor = t_colmajor;
  return LCC_OK;
}

lcc_status lcc_context_set_tune_cache(lcc_context ctx, const char* path) {
  if (!ctx) return fail(nullptr, LCC_ERR_ARG, "ctx is NULL");
  ctx->c.tune_cache = path ? std::string(path) : std::string();
  return LCC_OK;
}

lcc_status lcc_create_hamiltonian(lcc_context ctx, const lcc_ham_desc* d, lcc_hamiltonian* out) {
  if (!out) return fail(ctx, LCC_ERR_ARG, "out is NULL");
  *out = nullptr;
  return guarded(ctx, [&]() -> lcc_status {
    if (!d || !d->h) throw Error{LCC_ERR_ARG, "descriptor or h is NULL"};
    if (d->n_orb < 2 || d->n_orb > 64) throw Error{LCC_ERR_ARG, "n_orb must be in [2, 64]"};
    if (d->n_elec < 0 || d->n_elec > 2 * d->n_orb) throw Error{LCC_ERR_ARG, "n_elec out of range"};
    if (std::abs(d->two_sz) > d->n_elec || ((d->n_elec + d->two_sz) & 1)) throw Error{LCC_ERR_QN, "two_sz incompatible with n_elec"};
    std::unique_ptr<lcc_hamiltonian_s> h(new lcc_hamiltonian_s());
    HamDesc& hd = h->h.desc;
    const size_t K = (size_t)d->n_orb;
    hd.K = d->n_orb;
    hd.N = d->n_elec;
    hd.two_sz = d->two_sz;
    // chain position p holds orbital o[p]: every index of h, eri, u and orb_class is mapped
    std::vector<size_t> o(K);
    for (size_t p = 0; p < K; ++p) o[p] = p;
    if (d->site_order) {
      std::vector<char> seen(K, 0);
      for (size_t p = 0; p < K; ++p) {
        const int v = d->site_order[p];
        if (v < 0 || v >= (int)K || seen[v]) throw Error{LCC_ERR_ARG, "site_order must be a permutation of 0..n_orb-1"};
        seen[v] = 1;
        o[p] = (size_t)v;
      }
    }
    hd.h.resize(K * K);
    for (size_t p = 0; p < K; ++p)
      for (size_t q = 0; q < K; ++q) hd.h[p * K + q] = d->h[o[p] * K + o[q]];
    if (d->eri) {
      hd.eri.resize(K * K * K * K);
      for (size_t p = 0; p < K; ++p)
        for (size_t q = 0; q < K; ++q)
          for (size_t r = 0; r < K; ++r)
            for (size_t t = 0; t < K; ++t)
              hd.eri[((p * K + q) * K + r) * K + t] = d->eri[((o[p] * K + o[q]) * K + o[r]) * K + o[t]];
    }
    if (d->u_onsite) {
      hd.u.resize(K);
      for (size_t p = 0; p < K; ++p) hd.u[p] = d->u_onsite[o[p]];
    }
    hd.e_const = d->e_const;
    hd.switch_bond = d->switch_bond;
    if (d->part < 0 || d->part > 2) throw Error{LCC_ERR_ARG, "part must be 0 (H), 1 (H0) or 2 (U)"};
    if (d->part != 0 && !d->orb_class) throw Error{LCC_ERR_ARG, "a partition needs orb_class"};
    hd.part = d->part;
    if (d->orb_class) {
      hd.orb_class.resize(K);
      for (size_t p = 0; p < K; ++p) {
        const int c = d->orb_class[o[p]];
        if (c < 0 || c > 2) throw Error{LCC_ERR_ARG, "orb_class entries must be 0 (core), 1 (active) or 2 (virtual)"};
        hd.orb_class[p] = c;
      }
    }
    for (double v : hd.h)
      if (!std::isfinite(v)) throw Error{LCC_ERR_NAN, "non-finite h"};
    for (double v : hd.eri)
      if (!std::isfinite(v)) throw Error{LCC_ERR_NAN, "non-finite eri"};
    for (double v : hd.u)
      if (!std::isfinite(v)) throw Error{LCC_ERR_NAN, "non-finite u"};
    const std::string err = build_mpo(hd, h->h.mpo);
    if (!err.empty()) throw Error{LCC_ERR_ARG, err};
    h->h.ctx = ctx ? &ctx->c : nullptr;
    *out = h.release();
    return LCC_OK;
  });
}

void lcc_hamiltonian_destroy(lcc_hamiltonian ham) { delete ham; }

lcc_status lcc_hamiltonian_bond_dims(lcc_hamiltonian ham, int32_t* dims) {
  if (!ham || !dims) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  for (int b = 0; b <= ham->h.mpo.K; ++b) dims[b] = (int32_t)ham->h.mpo.dq[b].size();
  return LCC_OK;
}

lcc_status lcc_hamiltonian_channels(lcc_hamiltonian ham, int32_t bond, int32_t* dn, int32_t* d2sz) {
  if (!ham || !dn || !d2sz) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  if (bond < 0 || bond > ham->h.mpo.K) return fail(nullptr, LCC_ERR_ARG, "bond out of range");
  const auto& dq = ham->h.mpo.dq[bond];
  for (size_t i = 0; i < dq.size(); ++i) {
    dn[i] = dq[i].n;
    d2sz[i] = dq[i].sz;
  }
  return LCC_OK;
}

lcc_status lcc_hamiltonian_site_mpo(lcc_hamiltonian ham, int32_t site, int64_t* count, int32_t* w_in,
                                    int32_t* w_out, double* mats) {
  if (!ham || !count) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  if (site < 0 || site >= ham->h.mpo.K) return fail(nullptr, LCC_ERR_ARG, "site out of range");
  const auto& W = ham->h.mpo.W[site];
  if (!w_in) {
    *count = (int64_t)W.size();
    return LCC_OK;
  }
  if (*count < (int64_t)W.size() || !w_out || !mats) return fail(nullptr, LCC_ERR_ARG, "output arrays too small");
  for (size_t i = 0; i < W.size(); ++i) {
    w_in[i] = W[i].win;
    w_out[i] = W[i].wout;
    std::memcpy(mats + 16 * i, W[i].m, sizeof(double) * 16);
  }
  *count = (int64_t)W.size();
  return LCC_OK;
}

lcc_status lcc_build_environments(lcc_context ctx, lcc_hamiltonian ham, const lcc_mps_desc* mps, int32_t site,
                                  lcc_env* out) {
  if (!out) return fail(ctx, LCC_ERR_ARG, "out is NULL");
  *out = nullptr;
  return guarded(ctx, [&]() -> lcc_status {
    require_device(ctx);
    if (!ham || !mps) throw Error{LCC_ERR_ARG, "NULL argument"};
    std::unique_ptr<lcc_env_s> e(new lcc_env_s());
    e->e = build_env(&ctx->c, ham->h, *mps, site);
    *out = e.release();
    return LCC_OK;
  });
}

lcc_status lcc_build_environments_one_site(lcc_context ctx, lcc_hamiltonian ham, const lcc_mps_desc* mps,
                                           int32_t site, lcc_env* out) {
  if (!out) return fail(ctx, LCC_ERR_ARG, "out is NULL");
  *out = nullptr;
  return guarded(ctx, [&]() -> lcc_status {
    require_device(ctx);
    if (!ham || !mps) throw Error{LCC_ERR_ARG, "NULL argument"};
    std::unique_ptr<lcc_env_s> e(new lcc_env_s());
    e->e = build_env(&ctx->c, ham->h, *mps, site, true);
    *out = e.release();
    return LCC_OK;
  });
}

lcc_status lcc_build_transition_environments(lcc_context ctx, lcc_hamiltonian ham, const lcc_mps_desc* bra,
                                             const lcc_mps_desc* ket, int32_t site, lcc_env* out) {
  if (!out) return fail(ctx, LCC_ERR_ARG, "out is NULL");
  *out = nullptr;
  return guarded(ctx, [&]() -> lcc_status {
    require_device(ctx);
    if (!ham || !bra || !ket) throw Error{LCC_ERR_ARG, "NULL argument"};
    std::unique_ptr<lcc_env_s> e(new lcc_env_s());
    e->e = build_transition_env(&ctx->c, ham->h, *bra, *ket, site);
    *out = e.release();
    return LCC_OK;
  });
}

lcc_status lcc_build_transition_environments_one_site(lcc_context ctx, lcc_hamiltonian ham, const lcc_mps_desc* bra,
                                                      const lcc_mps_desc* ket, int32_t site, lcc_env* out) {
  if (!out) return fail(ctx, LCC_ERR_ARG, "out is NULL");
  *out = nullptr;
  return guarded(ctx, [&]() -> lcc_status {
    require_device(ctx);
    if (!ham || !bra || !ket) throw Error{LCC_ERR_ARG, "NULL argument"};
    std::unique_ptr<lcc_env_s> e(new lcc_env_s());
    e->e = build_transition_env(&ctx->c, ham->h, *bra, *ket, site, true);
    *out = e.release();
    return LCC_OK;
  });
}

// The destroy calls do not touch the context: objects may be destroyed in any order (a garbage
// collector may finalise a context before the environments made on it).  Device memory is
// released with hipFree, which waits for the device work in flight.
void lcc_env_destroy(lcc_env env) {
  if (!env || !env->owned) return;
  delete env;
}

lcc_status lcc_env_layout(lcc_env env, lcc_layout_info* info, lcc_block_entry* blocks) {
  if (!env || !info) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  const Env& e = *env->e;
  info->n_elements = e.n_elements;
  info->n_blocks = (int32_t)e.layout.size();
  info->n_sectors = (int32_t)e.sectors.size();
  info->mpo_bond_dim = e.D_mid;
  info->transition = e.transition ? 1 : 0;
  info->flops_per_apply = e.plan.flops1 + e.plan.flops2;
  if (blocks) std::memcpy(blocks, e.layout.data(), sizeof(lcc_block_entry) * e.layout.size());
  return LCC_OK;
}

lcc_status lcc_env_input_layout(lcc_env env, lcc_layout_info* info, lcc_block_entry* blocks) {
  if (!env || !info) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  const Env& e = *env->e;
  info->n_elements = e.n_in;
  info->n_blocks = (int32_t)e.layout_in.size();
  info->n_sectors = (int32_t)e.sectors_in.size();
  info->mpo_bond_dim = e.D_mid;
  info->transition = e.transition ? 1 : 0;
  info->flops_per_apply = e.plan.flops1 + e.plan.flops2;
  if (blocks) std::memcpy(blocks, e.layout_in.data(), sizeof(lcc_block_entry) * e.layout_in.size());
  return LCC_OK;
}

lcc_status lcc_env_ket_tensor(lcc_env env, double* x) {
  if (!env || !x) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  lcc_context ctx = static_cast<lcc_context>(env->e->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    if (!env->e->transition) throw Error{LCC_ERR_STATE, "not a transition environment"};
    check_hip(hipSetDevice(env->e->ctx->device), "hipSetDevice");
    hipStream_t st = env->e->ctx->stream;
    check_hip(hipMemcpyAsync(x, env->e->x0.p, sizeof(double) * env->e->n_in, hipMemcpyDeviceToDevice, st), "copy");
    check_hip(hipStreamSynchronize(st), "copy sync");
    return LCC_OK;
  });
}

lcc_status lcc_env_diagonal(lcc_env env, double* d) {
  if (!env || !d) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  lcc_context ctx = static_cast<lcc_context>(env->e->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    check_hip(hipSetDevice(env->e->ctx->device), "hipSetDevice");
    compute_diagonal(*env->e);
    hipStream_t st = env->e->ctx->stream;
    check_hip(hipMemcpyAsync(d, env->e->diag64.p, sizeof(double) * env->e->n_elements, hipMemcpyDeviceToDevice, st),
              "copy");
    check_hip(hipStreamSynchronize(st), "copy sync");
    return LCC_OK;
  });
}

lcc_status lcc_env_flops(lcc_env env, double* phase1, double* phase2) {
  if (!env || !phase1 || !phase2) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  *phase1 = env->e->plan.flops1;
  *phase2 = env->e->plan.flops2;
  return LCC_OK;
}

lcc_status lcc_apply_heff(lcc_env env, lcc_precision precision, const void* x, void* y) {
  if (!env) return fail(nullptr, LCC_ERR_ARG, "env is NULL");
  lcc_context ctx = static_cast<lcc_context>(env->e->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    if (!x || !y) throw Error{LCC_ERR_ARG, "x or y is NULL"};
    if (x == y) throw Error{LCC_ERR_ARG, "x and y must not overlap"};
    if (precision != LCC_FP64 && precision != LCC_FP32 && precision != LCC_BF16X3) throw Error{LCC_ERR_ARG, "unknown precision"};
    check_hip(hipSetDevice(env->e->ctx->device), "hipSetDevice");
    apply_heff(*env->e, precision, x, y);
    return LCC_OK;
  });
}

lcc_status lcc_env_profile_apply(lcc_env env, lcc_precision precision, const void* x, void* y, int32_t reps,
                                 float* ms1, float* ms2) {
  if (!env) return fail(nullptr, LCC_ERR_ARG, "env is NULL");
  lcc_context ctx = static_cast<lcc_context>(env->e->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    if (!x || !y || !ms1 || !ms2 || x == y) throw Error{LCC_ERR_ARG, "invalid buffers"};
    if (precision != LCC_FP64 && precision != LCC_FP32 && precision != LCC_BF16X3) throw Error{LCC_ERR_ARG, "unknown precision"};
    check_hip(hipSetDevice(env->e->ctx->device), "hipSetDevice");
    if (precision != LCC_FP64) ensure_fp32(*env->e);
    profile_apply(*env->e, precision, x, y, reps, ms1, ms2);
    return LCC_OK;
  });
}

lcc_status lcc_env_profile_launches(lcc_env env, lcc_precision precision, const void* x, void* y, int32_t reps,
                                    int32_t* count, lcc_launch_profile* out) {
  if (!env || !count) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  lcc_context ctx = static_cast<lcc_context>(env->e->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    const Plan& P = env->e->plan;
    int n = 1;
    for (const Plan::Chunk& C : P.chunks) n += (int)(C.phase1.size() + C.phase2.size());
    if (!out) {
      *count = n;
      return LCC_OK;
    }
    if (*count < n) throw Error{LCC_ERR_ARG, "output array too small"};
    if (!x || !y || x == y) throw Error{LCC_ERR_ARG, "invalid buffers"};
    if (precision != LCC_FP64 && precision != LCC_FP32 && precision != LCC_BF16X3) throw Error{LCC_ERR_ARG, "unknown precision"};
    check_hip(hipSetDevice(env->e->ctx->device), "hipSetDevice");
    std::vector<lcc_launch_profile> v = profile_launches(*env->e, precision, x, y, reps);
    for (size_t i = 0; i < v.size(); ++i) out[i] = v[i];
    *count = (int32_t)v.size();
    return LCC_OK;
  });
}

lcc_status lcc_env_autotune(lcc_env env, lcc_precision precision, int32_t reps, lcc_tune_info* info) {
  if (!env) return fail(nullptr, LCC_ERR_ARG, "env is NULL");
  lcc_context ctx = static_cast<lcc_context>(env->e->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    if (env->e->transition) throw Error{LCC_ERR_STATE, "a transition environment only supports apply"};
    if (precision != LCC_FP64 && precision != LCC_FP32 && precision != LCC_BF16X3) throw Error{LCC_ERR_ARG, "unknown precision"};
    if (reps < 1 || reps > 1000) throw Error{LCC_ERR_ARG, "reps must be in [1, 1000]"};
    check_hip(hipSetDevice(env->e->ctx->device), "hipSetDevice");
    autotune(*env->e, precision, reps, info);
    return LCC_OK;
  });
}

lcc_status lcc_lowest_eigenvalue(lcc_env env, int32_t steps, uint64_t seed, double* theta, double* residual) {
  if (!env) return fail(nullptr, LCC_ERR_ARG, "env is NULL");
  lcc_context ctx = static_cast<lcc_context>(env->e->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    if (env->e->transition) throw Error{LCC_ERR_STATE, "a transition environment only supports apply"};
    if (!theta || !residual) throw Error{LCC_ERR_ARG, "NULL output"};
    check_hip(hipSetDevice(env->e->ctx->device), "hipSetDevice");
    lowest_eigenvalue(*env->e, steps, seed, theta, residual);
    return LCC_OK;
  });
}

lcc_status lcc_lowest_eigenvalue_noalloc(lcc_env env, int32_t steps, uint64_t seed, double* theta, double* residual) {
  if (!env) return fail(nullptr, LCC_ERR_ARG, "env is NULL");
  lcc_context ctx = static_cast<lcc_context>(env->e->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    if (env->e->transition) throw Error{LCC_ERR_STATE, "a transition environment only supports apply"};
    if (!theta || !residual) throw Error{LCC_ERR_ARG, "NULL output"};
    check_hip(hipSetDevice(env->e->ctx->device), "hipSetDevice");
    lowest_eigenvalue_noalloc(*env->e, steps, seed, theta, residual);
    return LCC_OK;
  });
}

lcc_status lcc_lowest_eigenpair(lcc_env env, int32_t steps, int32_t max_restarts, double tol, uint64_t seed,
                                double* x, double* theta, double* residual) {
  if (!env) return fail(nullptr, LCC_ERR_ARG, "env is NULL");
  lcc_context ctx = static_cast<lcc_context>(env->e->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    if (env->e->transition) throw Error{LCC_ERR_STATE, "a transition environment only supports apply"};
    if (!theta || !residual || !x) throw Error{LCC_ERR_ARG, "NULL argument"};
    check_hip(hipSetDevice(env->e->ctx->device), "hipSetDevice");
    return lowest_eigenpair(*env->e, steps, max_restarts, tol, seed, x, theta, residual) ? LCC_OK : LCC_NOT_CONVERGED;
  });
}

lcc_status lcc_solve_local_lcc(lcc_env env, const lcc_solve_opts* opts, const double* b, double e0, const double* v,
                               double* x, lcc_solve_info* info) {
  if (!env) return fail(nullptr, LCC_ERR_ARG, "env is NULL");
  lcc_context ctx = static_cast<lcc_context>(env->e->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    if (env->e->transition) throw Error{LCC_ERR_STATE, "a transition environment only supports apply"};
    if (!b || !x) throw Error{LCC_ERR_ARG, "b or x is NULL"};
    check_hip(hipSetDevice(env->e->ctx->device), "hipSetDevice");
    lcc_solve_opts o{};
    if (opts) o = *opts;
    return solve_local(*env->e, o, b, e0, v, x, info);
  });
}

lcc_status lcc_batch_create(lcc_context ctx, int32_t n, const lcc_env* envs, lcc_batch* out) {
  if (!out) return fail(ctx, LCC_ERR_ARG, "out is NULL");
  *out = nullptr;
  return guarded(ctx, [&]() -> lcc_status {
    require_device(ctx);
    if (n < 1 || !envs) throw Error{LCC_ERR_ARG, "need at least one environment"};
    std::vector<Env*> v;
    for (int i = 0; i < n; ++i) {
      if (!envs[i]) throw Error{LCC_ERR_ARG, "NULL environment"};
      if (envs[i]->e->transition) throw Error{LCC_ERR_STATE, "a transition environment only supports apply"};
      v.push_back(envs[i]->e);
    }
    std::unique_ptr<lcc_batch_s> b(new lcc_batch_s());
    b->b = batch_create(&ctx->c, v);
    b->ctx = &ctx->c;
    *out = b.release();
    return LCC_OK;
  });
}

void lcc_batch_destroy(lcc_batch batch) {
  if (!batch) return;
  delete batch;
}

lcc_status lcc_batch_solve(lcc_batch batch, const lcc_solve_opts* opts, const double* const* b, const double* e0,
                           const double* const* v, double* const* x, lcc_solve_info* infos) {
  if (!batch) return fail(nullptr, LCC_ERR_ARG, "batch is NULL");
  lcc_context ctx = static_cast<lcc_context>(batch->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    if (!b || !e0 || !x) throw Error{LCC_ERR_ARG, "NULL argument"};
    check_hip(hipSetDevice(batch->ctx->device), "hipSetDevice");
    lcc_solve_opts o{};
    if (opts) o = *opts;
    if (o.preconditioner != 0) throw Error{LCC_ERR_ARG, "batched solves are not preconditioned"};
    return batch_solve(*batch->b, o, b, e0, v, x, infos);
  });
}

lcc_status lcc_solve_local_lcc_batched(int32_t n, const lcc_env* envs, const lcc_solve_opts* opts,
                                       const double* const* b, const double* e0, const double* const* v,
                                       double* const* x, lcc_solve_info* infos) {
  if (n < 1 || !envs || !envs[0]) return fail(nullptr, LCC_ERR_ARG, "need at least one environment");
  lcc_context ctx = static_cast<lcc_context>(envs[0]->e->ctx->handle);
  lcc_batch batch = nullptr;
  lcc_status st = lcc_batch_create(ctx, n, envs, &batch);
  if (st != LCC_OK) return st;
  st = lcc_batch_solve(batch, opts, b, e0, v, x, infos);
  lcc_batch_destroy(batch);
  return st;
}

lcc_status lcc_sweep_create(lcc_context ctx, lcc_hamiltonian ham, const lcc_mps_desc* mps, int32_t first_site,
                            lcc_sweep* out) {
  if (!out) return fail(ctx, LCC_ERR_ARG, "out is NULL");
  *out = nullptr;
  return guarded(ctx, [&]() -> lcc_status {
    require_device(ctx);
    if (!ham || !mps) throw Error{LCC_ERR_ARG, "NULL argument"};
    std::unique_ptr<lcc_sweep_s> s(new lcc_sweep_s());
    s->s = sweep_create(&ctx->c, ham->h, *mps, first_site);
    s->ctx = &ctx->c;
    s->view.owned = false;
    s->view.e = sweep_env(*s->s);
    *out = s.release();
    return LCC_OK;
  });
}

void lcc_sweep_destroy(lcc_sweep sweep) {
  if (!sweep) return;
  delete sweep;
}

lcc_status lcc_sweep_env(lcc_sweep sweep, lcc_env* out) {
  if (!sweep || !out) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  sweep->view.e = sweep_env(*sweep->s);
  *out = &sweep->view;
  return LCC_OK;
}

lcc_status lcc_sweep_guess(lcc_sweep sweep, double* x) {
  if (!sweep || !x) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  lcc_context ctx = static_cast<lcc_context>(sweep->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    check_hip(hipSetDevice(sweep->ctx->device), "hipSetDevice");
    sweep_copy_guess(*sweep->s, x);
    return LCC_OK;
  });
}

lcc_status lcc_sweep_advance(lcc_sweep sweep, const double* x, int32_t m_max, lcc_sweep_info* info) {
  if (!sweep || !x) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  lcc_context ctx = static_cast<lcc_context>(sweep->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    check_hip(hipSetDevice(sweep->ctx->device), "hipSetDevice");
    sweep_advance(*sweep->s, x, m_max, info);
    sweep->view.e = sweep_env(*sweep->s);
    return LCC_OK;
  });
}

lcc_status lcc_sweep_retreat(lcc_sweep sweep, const double* x, int32_t m_max, lcc_sweep_info* info) {
  if (!sweep || !x) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  lcc_context ctx = static_cast<lcc_context>(sweep->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    check_hip(hipSetDevice(sweep->ctx->device), "hipSetDevice");
    sweep_retreat(*sweep->s, x, m_max, info);
    sweep->view.e = sweep_env(*sweep->s);
    return LCC_OK;
  });
}

lcc_status lcc_sweep_position(lcc_sweep sweep, int32_t* site) {
  if (!sweep || !site) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  *site = sweep_site(*sweep->s);
  return LCC_OK;
}

lcc_status lcc_sweep_attach_reference(lcc_sweep sweep, lcc_hamiltonian op, lcc_hamiltonian u, const lcc_mps_desc* ref) {
  if (!sweep || !op || !ref) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  lcc_context ctx = static_cast<lcc_context>(sweep->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    check_hip(hipSetDevice(sweep->ctx->device), "hipSetDevice");
    sweep_attach_reference(*sweep->s, op->h, u ? &u->h : nullptr, *ref);
    return LCC_OK;
  });
}

lcc_status lcc_sweep_first_order_rhs(lcc_sweep sweep, double c, double* b, double* v, double* v_norm) {
  if (!sweep || !b || !v || !v_norm) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  if (!std::isfinite(c)) return fail(nullptr, LCC_ERR_ARG, "c must be finite");
  lcc_context ctx = static_cast<lcc_context>(sweep->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    check_hip(hipSetDevice(sweep->ctx->device), "hipSetDevice");
    sweep_first_order_rhs(*sweep->s, c, b, v, v_norm);
    return LCC_OK;
  });
}

lcc_status lcc_sweep_u_expectation(lcc_sweep sweep, const double* x, double* xux, double* xx) {
  if (!sweep || !x || !xux || !xx) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  lcc_context ctx = static_cast<lcc_context>(sweep->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    check_hip(hipSetDevice(sweep->ctx->device), "hipSetDevice");
    sweep_u_expectation(*sweep->s, x, xux, xx);
    return LCC_OK;
  });
}

lcc_status lcc_sweep_split_block(lcc_sweep sweep, const double* x, int32_t m_max, lcc_sweep_info* info) {
  if (!sweep || !x) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  lcc_context ctx = static_cast<lcc_context>(sweep->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    check_hip(hipSetDevice(sweep->ctx->device), "hipSetDevice");
    sweep_split_block(*sweep->s, x, m_max, info);
    return LCC_OK;
  });
}

lcc_status lcc_sweep_bond(lcc_sweep sweep, int32_t bond, int32_t* count, lcc_sector* sectors) {
  if (!sweep || !count) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  lcc_context ctx = static_cast<lcc_context>(sweep->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    const Bond& B = sweep_bond(*sweep->s, bond);
    if (!sectors) {
      *count = (int32_t)B.q.size();
      return LCC_OK;
    }
    if (*count < (int32_t)B.q.size()) throw Error{LCC_ERR_ARG, "sector array too small"};
    for (size_t i = 0; i < B.q.size(); ++i) sectors[i] = lcc_sector{B.q[i].n, B.q[i].sz, B.dim[i]};
    *count = (int32_t)B.q.size();
    return LCC_OK;
  });
}

lcc_status lcc_sweep_site_tensor(lcc_sweep sweep, int32_t site, int32_t* n_blocks, int64_t* n_elements,
                                 lcc_site_block* blocks, double* data_host) {
  if (!sweep || !n_blocks || !n_elements) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  lcc_context ctx = static_cast<lcc_context>(sweep->ctx->handle);
  return guarded(ctx, [&]() -> lcc_status {
    check_hip(hipSetDevice(sweep->ctx->device), "hipSetDevice");
    const DeviceMps& t = sweep_site_tensor(*sweep->s, site);
    int64_t total = 0;
    for (const SiteBlock& b : t.sites[site]) total += (int64_t)b.rows * b.cols;
    if (!blocks || !data_host) {
      *n_blocks = (int32_t)t.sites[site].size();
      *n_elements = total;
      return LCC_OK;
    }
    if (*n_blocks < (int32_t)t.sites[site].size() || *n_elements < total)
      throw Error{LCC_ERR_ARG, "output arrays too small"};
    int64_t off = 0;
    for (size_t i = 0; i < t.sites[site].size(); ++i) {
      const SiteBlock& b = t.sites[site][i];
      blocks[i] = lcc_site_block{b.l, b.s, b.r, b.rows, b.cols, off};
      check_hip(hipMemcpy(data_host + off, t.data.as<double>() + b.off, sizeof(double) * (size_t)b.rows * b.cols,
                          hipMemcpyDeviceToHost),
                "site tensor copy");
      off += (int64_t)b.rows * b.cols;
    }
    *n_blocks = (int32_t)t.sites[site].size();
    *n_elements = total;
    return LCC_OK;
  });
}

lcc_status lcc_mps_expectation(lcc_context ctx, lcc_hamiltonian ham, const lcc_mps_desc* mps, int32_t site,
                               double* value) {
  if (!ham || !mps || !value) return fail(ctx, LCC_ERR_ARG, "NULL argument");
  return guarded(ctx, [&]() -> lcc_status {
    require_device(ctx);
    // <Phi| H |Phi> as the transition operator of Phi with itself at the block (site, site + 1),
    // applied to Phi's own two-site tensor there
    std::unique_ptr<Env> e(build_transition_env(&ctx->c, ham->h, *mps, *mps, site));
    DevBuf y;
    y.alloc(sizeof(double) * std::max<int64_t>(e->n_elements, 1));
    apply_heff(*e, LCC_FP64, e->x0.p, y.p);
    Context* c = &ctx->c;
    hipStream_t st = c->stream;
    check_hip(launch_dot_f64(e->x0.as<double>(), y.as<double>(), e->n_elements, c->dot_partial.as<double>(),
                             c->dot_out.as<double>(), st), "dot");
    check_hip(hipMemcpyAsync(c->host_scalar, c->dot_out.p, sizeof(double), hipMemcpyDeviceToHost, st), "dot copy");
    check_hip(hipStreamSynchronize(st), "expectation");
    *value = c->host_scalar[0];
    return LCC_OK;
  });
}

lcc_status lcc_sweep_singular_values(lcc_sweep sweep, int32_t* count, double* out) {
  if (!sweep || !count) return fail(nullptr, LCC_ERR_ARG, "NULL argument");
  const std::vector<double>& v = sweep_singular_values(*sweep->s);
  if (!out) {
    *count = (int32_t)v.size();
    return LCC_OK;
  }
  if (*count < (int32_t)v.size()) return fail(nullptr, LCC_ERR_ARG, "output array too small");
  std::memcpy(out, v.data(), sizeof(double) * v.size());
  *count = (int32_t)v.size();
  return LCC_OK;
}

}  // extern "C"
