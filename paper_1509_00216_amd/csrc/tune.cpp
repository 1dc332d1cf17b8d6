// Autotuner of the H_eff x plan.
//
// The block-size histogram of a two-site problem (bond sectors and their dimensions, the MPO
// bond dimension) fixes the shapes of all block products.  For a histogram the tuner times,
// on the device, every candidate of the planner parameters (the per-tile cost that picks tile
// shapes, the split-K length and the group order of phase 2, the order of the two enlarged
// operators and the layout of the intermediate) and, for every launch of a plan, both GEMM kernels
// (term walk, packed k), then keeps the fastest plan and per-launch kernel choice.  The result
// is stored in a text cache keyed by a signature of the histogram, so that later environments
// with the same histogram (the same site of another sweep, another process) are planned the
// tuned way without timing anything.
#include <algorithm>
#include <cstdio>
#include <fstream>
#include <sstream>

#include "state.h"

namespace lcc {

namespace {

constexpr double kOverheads[] = {2048.0, 8192.0, 32768.0};
constexpr int64_t kSplits[] = {512, 1024, 2048};

void fnv(uint64_t& h, int64_t v) {
  for (int i = 0; i < 8; ++i) {
    h ^= (uint64_t)((v >> (8 * i)) & 0xff);
    h *= 1099511628211ull;
  }
}

// all GEMM launches of the plan, in apply order
std::vector<GemmLaunch*> launches_of(Env& env) {
  std::vector<GemmLaunch*> out;
  for (Plan::Chunk& C : env.plan.chunks) {
    for (GemmLaunch& L : C.phase1) out.push_back(&L);
    for (GemmLaunch& L : C.phase2) out.push_back(&L);
  }
  return out;
}

std::string flags_of(Env& env, int precision) {
  std::string f;
  for (GemmLaunch* L : launches_of(env)) f.push_back(L->packed[precision] ? '1' : '0');
  return f;
}

bool set_flags(Env& env, int precision, const std::string& f) {
  std::vector<GemmLaunch*> Ls = launches_of(env);
  if (f.size() != Ls.size()) return false;
  for (size_t i = 0; i < Ls.size(); ++i) Ls[i]->packed[precision] = f[i] == '1';
  return true;
}

bool same_params(const PlanParams& a, const PlanParams& b) {
  return a.tile_overhead == b.tile_overhead && a.split_k == b.split_k && a.p2_order == b.p2_order &&
         a.t_colmajor == b.t_colmajor;
}

struct Entry {
  PlanParams pp;
  std::string flags[3];
};

bool cache_find(const std::string& path, uint64_t sig, Entry& e) {
  if (path.empty()) return false;
  std::ifstream in(path);
  std::string line;
  bool found = false;
  while (std::getline(in, line)) {  // the last entry of a signature wins
    std::istringstream ls(line);
    unsigned long long s = 0;
    Entry x;
    if (!(ls >> std::hex >> s >> std::dec >> x.pp.tile_overhead >> x.pp.split_k >> x.pp.p2_order >> x.pp.t_colmajor >>
          x.flags[0] >> x.flags[1] >> x.flags[2]))
      continue;
    if (s == sig) {
      e = x;
      found = true;
    }
  }
  return found;
}

void cache_add(const std::string& path, uint64_t sig, const Entry& e) {
  if (path.empty()) return;
  std::ofstream out(path, std::ios::app);
  if (!out) throw Error{LCC_ERR_ARG, "cannot write the tuning cache " + path};
  char head[64];
  std::snprintf(head, sizeof head, "%016llx", (unsigned long long)sig);
  out << head << " " << e.pp.tile_overhead << " " << e.pp.split_k << " " << e.pp.p2_order << " " << e.pp.t_colmajor
      << " " << e.flags[0] << " " << e.flags[1] << " " << e.flags[2] << "\n";
}

// Per-launch mean times (ms) of one apply with every launch on the packed (or term-walk) kernel.
std::vector<float> time_variant(Env& env, int precision, bool packed, const void* x, void* y, int reps) {
  std::vector<GemmLaunch*> Ls = launches_of(env);
  std::vector<bool> keep(Ls.size());
  for (size_t i = 0; i < Ls.size(); ++i) {
    keep[i] = Ls[i]->packed[precision];
    Ls[i]->packed[precision] = packed;
  }
  const std::vector<lcc_launch_profile> prof = profile_launches(env, precision, x, y, reps);
  for (size_t i = 0; i < Ls.size(); ++i) Ls[i]->packed[precision] = keep[i];
  std::vector<float> out;
  for (const lcc_launch_profile& p : prof) out.push_back(p.ms);
  return out;  // GEMM launches in order, then the reduction
}

double total_ms(Env& env, int precision, const void* x, void* y, int reps) {
  double t = 0;
  for (const lcc_launch_profile& p : profile_launches(env, precision, x, y, reps)) t += p.ms;
  return t;
}

// Choose each launch's kernel for `precision` on the current plan; returns the summed time.
double choose_kernels(Env& env, int precision, const void* x, void* y, int reps) {
  const std::vector<float> tw = time_variant(env, precision, false, x, y, reps);
  const std::vector<float> tp = time_variant(env, precision, true, x, y, reps);
  std::vector<GemmLaunch*> Ls = launches_of(env);
  double t = 0;
  for (size_t i = 0; i < Ls.size(); ++i) {
    Ls[i]->packed[precision] = tp[i] < tw[i];
    t += std::min(tp[i], tw[i]);
  }
  for (size_t i = Ls.size(); i < tw.size(); ++i) t += tw[i];  // reduction
  return t;
}

}  // namespace

// Bumped whenever the planner or the kernel set changes what a cached entry means.
constexpr int64_t kPlannerVersion = 3;

uint64_t histogram_signature(const Env& env) {
  uint64_t h = 1469598103934665603ull;
  fnv(h, kPlannerVersion);
  fnv(h, env.D_mid);
  fnv(h, env.ctx->t_budget_elems);
  for (const Bond* b : {&env.bl, &env.br}) {
    fnv(h, (int64_t)b->q.size());
    for (size_t i = 0; i < b->q.size(); ++i) {
      fnv(h, b->q[i].n);
      fnv(h, b->q[i].sz);
      fnv(h, b->dim[i]);
    }
  }
  fnv(h, (int64_t)env.in.dq_mid.size());
  for (const QN& q : env.in.dq_mid) {
    fnv(h, q.n);
    fnv(h, q.sz);
  }
  return h;
}

bool apply_tuned(Env& env) {
  Entry e;
  if (!cache_find(env.ctx->tune_cache, histogram_signature(env), e)) return false;
  if (!same_params(e.pp, env.params)) plan_env(env, e.pp);
  for (int p = 0; p < 3; ++p) set_flags(env, p, e.flags[p]);
  return true;
}

void autotune(Env& env, int precision, int reps, lcc_tune_info* info) {
  if (precision < 0 || precision > 2) throw Error{LCC_ERR_ARG, "unknown precision"};
  if (reps < 1) reps = 1;
  hipStream_t st = env.ctx->stream;
  if (precision != LCC_FP64) ensure_fp32(env);
  // operands: a seeded vector (its values do not change the timings)
  DevBuf x, y, x64;
  const int64_t n = std::max<int64_t>(env.n_elements, 1);
  const size_t esz = precision == LCC_FP64 ? sizeof(double) : sizeof(float);
  x64.alloc(sizeof(double) * n);
  check_hip(launch_random_fill_f64(x64.as<double>(), n, 12345, st), "tune fill");
  x.alloc(esz * n);
  y.alloc(esz * n);
  if (precision == LCC_FP64)
    check_hip(hipMemcpyAsync(x.p, x64.p, sizeof(double) * n, hipMemcpyDeviceToDevice, st), "tune copy");
  else
    check_hip(launch_convert_f64_f32(n, x64.as<double>(), x.as<float>(), st), "tune convert");
  check_hip(hipStreamSynchronize(st), "tune inputs");

  lcc_tune_info out{};
  const uint64_t sig = histogram_signature(env);
  Entry cached;
  if (cache_find(env.ctx->tune_cache, sig, cached)) {
    out.ms_before = (float)total_ms(env, precision, x.p, y.p, reps);
    if (!same_params(cached.pp, env.params)) plan_env(env, cached.pp);
    for (int p = 0; p < 3; ++p) set_flags(env, p, cached.flags[p]);
    out.from_cache = 1;
  } else {
    (void)total_ms(env, precision, x.p, y.p, 1);  // warm-up
    out.ms_before = (float)total_ms(env, precision, x.p, y.p, reps);
    PlanParams best_pp = env.params;
    double best = 1e300;
    for (double ov : kOverheads)
      for (int64_t sk : kSplits)
      for (int order = 0; order < 2; ++order)
      for (int cm = 0; cm < 3; ++cm) {
        PlanParams pp;
        pp.tile_overhead = ov;
        pp.split_k = sk;
        pp.p2_order = order;
        pp.t_colmajor = cm;
        plan_env(env, pp);
        const double t = choose_kernels(env, precision, x.p, y.p, reps);
        ++out.candidates;
        if (t < best) {
          best = t;
          best_pp = pp;
        }
      }
    plan_env(env, best_pp);
    Entry e;
    e.pp = best_pp;
    for (int p = 0; p < 3; ++p) {
      if (p != LCC_FP64) ensure_fp32(env);
      // the other precisions' kernels are chosen on the same plan with their own operands
      if (p == precision) {
        (void)choose_kernels(env, p, x.p, y.p, reps);
      } else {
        DevBuf xp, yp;
        const size_t ez = p == LCC_FP64 ? sizeof(double) : sizeof(float);
        xp.alloc(ez * n);
        yp.alloc(ez * n);
        if (p == LCC_FP64)
          check_hip(hipMemcpyAsync(xp.p, x64.p, sizeof(double) * n, hipMemcpyDeviceToDevice, st), "tune copy");
        else
          check_hip(launch_convert_f64_f32(n, x64.as<double>(), xp.as<float>(), st), "tune convert");
        (void)choose_kernels(env, p, xp.p, yp.p, reps);
      }
      e.flags[p] = flags_of(env, p);
    }
    cache_add(env.ctx->tune_cache, sig, e);
  }
  out.tile_overhead = env.params.tile_overhead;
  out.split_k = env.params.split_k;
  out.p2_order = env.params.p2_order;
  out.t_colmajor = env.params.t_colmajor;
  out.ms_after = (float)total_ms(env, precision, x.p, y.p, reps);
  for (GemmLaunch* L : launches_of(env)) {
    ++out.launches;
    if (L->packed[precision]) ++out.packed_launches;
  }
  if (info) *info = out;
}

}  // namespace lcc
