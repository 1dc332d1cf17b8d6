// Batched local LCC solves: many independent two-site problems advanced together.
//
// Every phase of H_eff x is ONE launch per tile shape for all problems (their plans are
// merged; each group carries its problem index and the kernel takes that problem's operand
// pointers from a table).  The CG recurrences of all problems run with per-problem scalars in
// device memory and per-problem active flags, so converged problems drop out of every launch
// and no host round trip is needed inside an iteration; one iteration is captured in a HIP
// graph and replayed.  The algorithm per problem is the reliable-update CG of the single
// solve: low-precision recurrence, FP64 true residual and FP64 solution on refresh.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <set>
#include <vector>

#include "state.h"

namespace lcc {
namespace {

constexpr int kSegChunk = 8192;

enum : int { ST_RUNNING = 100 };

// ---------------------------------------------------------------------------------------
// per-problem scalar steps (one thread per problem)
// ---------------------------------------------------------------------------------------
struct Scalars {
  double *e0neg, *tol_bn, *sc, *inv_sc, *rr, *rr_new, *pAp, *alpha, *beta, *rmax, *dot, *pscale, *bn;
  int *active, *refresh, *cont, *ract, *has_v, *hv_active, *hv_refresh, *hv_ract, *status, *iters, *outer;
};

__global__ void k_start(Scalars S, int n) {  // after bn = sqrt(dot) and dot = |r|^2 of the first residual
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double rn = sqrt(S.dot[p]);
  S.sc[p] = rn > 0.0 ? rn : 1.0;
  S.inv_sc[p] = 1.0 / S.sc[p];
  S.iters[p] = 0;
  S.outer[p] = 0;
  const int go = rn > S.tol_bn[p];
  S.active[p] = go;
  S.status[p] = go ? ST_RUNNING : LCC_OK;
  S.hv_active[p] = go && S.has_v[p];
  S.refresh[p] = 0;
  S.cont[p] = 0;
}
__global__ void k_rr_init(Scalars S, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || !S.active[p]) return;
  S.rr[p] = S.dot[p];
  S.rmax[p] = sqrt(S.dot[p]);
}
__global__ void k_alpha(Scalars S, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || !S.active[p]) return;
  const double pAp = S.pAp[p];
  if (!isfinite(pAp)) {
    S.status[p] = LCC_ERR_NAN;
    S.active[p] = 0;
    S.hv_active[p] = 0;
    S.alpha[p] = 0.0;
    return;
  }
  if (pAp <= 0.0) {
    S.status[p] = LCC_ERR_NOT_SPD;
    S.active[p] = 0;
    S.hv_active[p] = 0;
    S.alpha[p] = 0.0;
    return;
  }
  S.alpha[p] = S.rr[p] / pAp;
}
__global__ void k_after_r(Scalars S, int n, double delta, int max_iter) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  S.refresh[p] = 0;
  S.cont[p] = 0;
  S.hv_refresh[p] = 0;
  if (!S.active[p]) return;
  S.iters[p] += 1;
  const double rrn = S.rr_new[p];
  if (!isfinite(rrn)) {
    S.status[p] = LCC_ERR_NAN;
    S.active[p] = 0;
    S.hv_active[p] = 0;
    return;
  }
  const double rn = sqrt(rrn) * S.sc[p];
  const int refresh = rn < delta * S.rmax[p] * S.sc[p] || rn <= S.tol_bn[p] || S.iters[p] >= max_iter;
  S.refresh[p] = refresh;
  S.hv_refresh[p] = refresh && S.has_v[p];
  S.cont[p] = !refresh;
  if (!refresh) {
    S.beta[p] = rrn / S.rr[p];
    S.rr[p] = rrn;
  }
}
__global__ void k_refresh(Scalars S, int n, int max_iter, int max_outer) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  S.ract[p] = 0;
  S.hv_ract[p] = 0;
  if (!S.refresh[p]) return;
  S.outer[p] += 1;
  const double rn2 = S.dot[p];
  const double rnorm = sqrt(rn2);
  if (!isfinite(rnorm)) {
    S.status[p] = LCC_ERR_NAN;
    S.active[p] = 0;
  } else if (rnorm <= S.tol_bn[p]) {
    S.status[p] = LCC_OK;
    S.active[p] = 0;
  } else if (S.iters[p] >= max_iter || S.outer[p] >= max_outer) {
    S.status[p] = LCC_NOT_CONVERGED;
    S.active[p] = 0;
  } else {
    const double sc = S.sc[p];
    const double beta_true = rn2 / (S.rr[p] * sc * sc);
    S.pscale[p] = beta_true * sc / rnorm;
    S.sc[p] = rnorm;
    S.inv_sc[p] = 1.0 / rnorm;
    S.ract[p] = 1;
    S.hv_ract[p] = S.has_v[p];
  }
  S.hv_active[p] = S.active[p] && S.has_v[p];
}
__global__ void k_rr_refresh(Scalars S, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || !S.ract[p]) return;
  S.rr[p] = S.dot[p];
  S.rmax[p] = sqrt(S.dot[p]);
}
__global__ void k_count_active(const int* __restrict__ active, int n, int* __restrict__ out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int c = 0;
    for (int p = 0; p < n; ++p) c += active[p];
    out[0] = c;
  }
}

struct MergedLaunch {
  bool ta = false, tb = false;
  int shape = 0, n_tiles = 0;
  DevBuf terms, slots, groups, tiles;
  bool packed[3] = {false, false, false};
  GemmDesc desc(int precision) const {
    return GemmDesc{terms.as<GemmTerm>(), slots.as<SlotRec>(), groups.as<GemmGroup>(), tiles.as<GemmTile>(),
                    n_tiles, shape, ta, tb, packed[precision]};
  }
};

template <class T>
std::vector<T> download(const DevBuf& b, size_t count, hipStream_t s) {
  std::vector<T> h(count);
  if (count) check_hip(hipMemcpyAsync(h.data(), b.p, count * sizeof(T), hipMemcpyDeviceToHost, s), "download");
  check_hip(hipStreamSynchronize(s), "download sync");
  return h;
}

}  // namespace

struct Batch {
  Context* ctx = nullptr;
  std::vector<Env*> envs;
  int n = 0;
  std::vector<int64_t> off;  // arena offset per problem
  int64_t total = 0;
  std::vector<SegBlock> hblocks;
  std::vector<int32_t> hfirst;
  DevBuf blocks, first, partial;
  std::vector<std::vector<MergedLaunch>> phase1, phase2;  // per chunk index
  DevBuf reduce_groups, reduce_tiles;
  int n_reduce_tiles = 0;
  DevBuf table64, table32;
  // arena vectors
  DevBuf x64, bq, t64, v64, r32, p32, Ap32, d32, v32;
  // scalars
  DevBuf sd, si;
  Scalars S{};
  DevBuf count;
  int* host_count = nullptr;
  hipStream_t stream = nullptr;
  // concurrent launches of one GEMM phase (the context's overlap setting): side streams of
  // default priority joined by events, also inside the captured iteration graph
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev_join;
  hipEvent_t ev_fork = nullptr;
  ~Batch() {
    for (hipStream_t t : side) {
      (void)hipStreamSynchronize(t);
      (void)hipStreamDestroy(t);
    }
    for (hipEvent_t e : ev_join) (void)hipEventDestroy(e);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (stream) (void)hipStreamDestroy(stream);
    if (host_count) (void)hipHostFree(host_count);
  }
};

namespace {

// One merged launch per tile shape and operand layout: members planned with different
// layouts (e.g. one with the column-major intermediate) keep separate launches.
void merge_phase(const std::vector<Env*>& envs, int chunk, int phase, hipStream_t st, std::vector<MergedLaunch>& out) {
  for (int key = 0; key < 4 * kNumTileShapes; ++key) {
    const int shape = key / 4;
    const bool ta = (key & 1) != 0, tb = (key & 2) != 0;
    std::vector<GemmTerm> terms;
    std::vector<SlotRec> slots;
    std::vector<GemmGroup> groups;
    std::vector<GemmTile> tiles;
    bool first = true;
    bool packed[3] = {false, false, false};
    for (size_t p = 0; p < envs.size(); ++p) {
      if (chunk >= (int)envs[p]->plan.chunks.size()) continue;
      const Plan::Chunk& C = envs[p]->plan.chunks[chunk];
      const std::vector<GemmLaunch>& Ls = phase == 1 ? C.phase1 : C.phase2;
      for (const GemmLaunch& L : Ls) {
        if (L.shape != shape || L.ta != ta || L.tb != tb) continue;
        const size_t ng = L.groups.bytes / sizeof(GemmGroup);
        auto hs = download<SlotRec>(L.slots, (size_t)L.n_slots, st);
        auto hg = download<GemmGroup>(L.groups, ng, st);
        auto hl = download<GemmTile>(L.tiles, (size_t)L.n_tiles, st);
        const int32_t sb0 = (int32_t)slots.size(), tb0 = (int32_t)terms.size(), gb0 = (int32_t)groups.size();
        // only the real groups (buffers are padded): the ones the tiles reference
        int32_t max_group = -1;
        for (const GemmTile& t : hl) max_group = std::max(max_group, t.group);
        int32_t n_terms = 0;
        for (int32_t gi = 0; gi <= max_group; ++gi) n_terms = std::max(n_terms, hg[gi].term_end);
        auto ht = download<GemmTerm>(L.terms, (size_t)n_terms, st);
        terms.insert(terms.end(), ht.begin(), ht.end());
        slots.insert(slots.end(), hs.begin(), hs.end());
        for (int32_t gi = 0; gi <= max_group; ++gi) {
          GemmGroup g = hg[gi];
          g.slot_begin += sb0;
          g.slot_end += sb0;
          g.term_begin += tb0;
          g.term_end += tb0;
          g.problem = (int32_t)p;
          groups.push_back(g);
        }
        if (first)
          for (int q = 0; q < 3; ++q) packed[q] = L.packed[q];
        first = false;
        for (const GemmTile& t : hl) tiles.push_back(GemmTile{t.group + gb0, t.tile});
      }
    }
    if (tiles.empty()) continue;
    if (slots.size() > (size_t)INT32_MAX) throw Error{LCC_ERR_ARG, "batched plan too large"};
    MergedLaunch M;
    M.ta = ta;
    M.tb = tb;
    M.shape = shape;
    M.n_tiles = (int)tiles.size();
    for (int q = 0; q < 3; ++q) M.packed[q] = packed[q];
    upload(M.terms, terms, st);
    upload(M.slots, slots, st);
    upload(M.groups, groups, st);
    upload(M.tiles, tiles, st);
    out.push_back(std::move(M));
  }
}

}  // namespace

Batch* batch_create(Context* ctx, const std::vector<Env*>& envs) {
  hipStream_t st = ctx->stream;
  std::unique_ptr<Batch> B(new Batch());
  B->ctx = ctx;
  B->envs = envs;
  B->n = (int)envs.size();
  std::set<const Env*> seen;
  for (Env* e : envs) {
    if (e->ctx != ctx) throw Error{LCC_ERR_ARG, "all environments of a batch must belong to one context"};
    // an environment's intermediate and split-K buffers serve one problem at a time
    if (!seen.insert(e).second) throw Error{LCC_ERR_ARG, "an environment appears twice in a batch"};
    ensure_fp32(*e);
  }
  // arena layout and segment blocks
  for (int p = 0; p < B->n; ++p) {
    B->off.push_back(B->total);
    const int64_t n = envs[p]->n_elements;
    B->hfirst.push_back((int32_t)B->hblocks.size());
    for (int64_t b = 0; b < n; b += kSegChunk)
      B->hblocks.push_back(SegBlock{p, 0, B->total + b, B->total + std::min<int64_t>(n, b + kSegChunk)});
    B->total += (n + 63) / 64 * 64;
  }
  B->hfirst.push_back((int32_t)B->hblocks.size());
  upload(B->blocks, B->hblocks, st);
  upload(B->first, B->hfirst, st);
  B->partial.alloc(sizeof(double) * std::max<size_t>(1, B->hblocks.size()));
  // merged plans
  size_t nchunks = 0;
  for (Env* e : envs) nchunks = std::max(nchunks, e->plan.chunks.size());
  B->phase1.resize(nchunks);
  B->phase2.resize(nchunks);
  for (size_t c = 0; c < nchunks; ++c) {
    merge_phase(envs, (int)c, 1, st, B->phase1[c]);
    merge_phase(envs, (int)c, 2, st, B->phase2[c]);
  }
  {
    std::vector<ReduceGroup> rg;
    std::vector<ReduceTile> rt;
    for (int p = 0; p < B->n; ++p) {
      const Plan& P = envs[p]->plan;
      const size_t ng = P.reduce_groups.bytes / sizeof(ReduceGroup);
      auto hg = download<ReduceGroup>(P.reduce_groups, ng, st);
      auto ht = download<ReduceTile>(P.reduce_tiles, (size_t)P.n_reduce_tiles, st);
      const int32_t g0 = (int32_t)rg.size();
      int32_t max_group = -1;
      for (const ReduceTile& t : ht) max_group = std::max(max_group, t.group);
      for (int32_t gi = 0; gi <= max_group; ++gi) {
        ReduceGroup g = hg[gi];
        g.problem = p;
        rg.push_back(g);
      }
      for (const ReduceTile& t : ht) rt.push_back(ReduceTile{t.group + g0, t.chunk});
    }
    upload(B->reduce_groups, rg, st);
    upload(B->reduce_tiles, rt, st);
    B->n_reduce_tiles = (int)rt.size();
  }
  // arena vectors
  const size_t N = (size_t)std::max<int64_t>(B->total, 1);
  for (DevBuf* d : {&B->x64, &B->bq, &B->t64, &B->v64}) d->alloc(sizeof(double) * N);
  for (DevBuf* d : {&B->r32, &B->p32, &B->Ap32, &B->d32, &B->v32}) d->alloc(sizeof(float) * N);
  // operand tables: FP64 products map x64 -> t64, low-precision products p32 -> Ap32
  std::vector<Bases<double>> t64(B->n);
  std::vector<Bases<float>> t32(B->n);
  for (int p = 0; p < B->n; ++p) {
    Env& e = *envs[p];
    Bases<double>& a = t64[p];
    std::memset(&a, 0, sizeof(a));
    a.p[BASE_ENV] = e.env64.as<double>();
    a.p[BASE_MERGED] = e.merged64.as<double>();
    a.p[BASE_X] = B->x64.as<double>() + B->off[p];
    a.p[BASE_T] = e.tbuf.as<double>();
    a.p[BASE_Y] = B->t64.as<double>() + B->off[p];
    a.p[BASE_WORK] = e.work.as<double>();
    Bases<float>& b = t32[p];
    std::memset(&b, 0, sizeof(b));
    b.p[BASE_ENV] = e.env32.as<float>();
    b.p[BASE_MERGED] = e.merged32.as<float>();
    b.p[BASE_X] = B->p32.as<float>() + B->off[p];
    b.p[BASE_T] = e.tbuf.as<float>();
    b.p[BASE_Y] = B->Ap32.as<float>() + B->off[p];
    b.p[BASE_WORK] = e.work.as<float>();
  }
  upload(B->table64, t64, st);
  upload(B->table32, t32, st);
  // scalars: 13 double arrays, 11 int arrays
  B->sd.alloc(sizeof(double) * 13 * B->n);
  B->si.alloc(sizeof(int) * 11 * B->n);
  double* d = B->sd.as<double>();
  int* i = B->si.as<int>();
  Scalars& S = B->S;
  double** dp[] = {&S.e0neg, &S.tol_bn, &S.sc, &S.inv_sc, &S.rr, &S.rr_new, &S.pAp, &S.alpha, &S.beta, &S.rmax, &S.dot, &S.pscale, &S.bn};
  for (int k = 0; k < 13; ++k) *dp[k] = d + (size_t)k * B->n;
  int** ip[] = {&S.active, &S.refresh, &S.cont, &S.ract, &S.has_v, &S.hv_active, &S.hv_refresh, &S.hv_ract, &S.status, &S.iters, &S.outer};
  for (int k = 0; k < 11; ++k) *ip[k] = i + (size_t)k * B->n;
  B->count.alloc(sizeof(int) * 4);
  check_hip(hipHostMalloc(reinterpret_cast<void**>(&B->host_count), sizeof(int) * 4, hipHostMallocDefault), "hipHostMalloc");
  check_hip(hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking), "batch stream");
  if (ctx->overlap > 0) {
    check_hip(hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming), "batch event");
    for (int k = 0; k < ctx->overlap; ++k) {
      hipStream_t t = nullptr;
      hipEvent_t e = nullptr;
      check_hip(hipStreamCreateWithFlags(&t, hipStreamNonBlocking), "batch side stream");
      B->side.push_back(t);
      check_hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "batch event");
      B->ev_join.push_back(e);
    }
  }
  check_hip(hipStreamSynchronize(st), "batch create");
  return B.release();
}

void batch_destroy(Batch* b) { delete b; }

namespace {

struct Runner {
  Batch& B;
  hipStream_t s;
  int prec;
  int nb() const { return (int)B.hblocks.size(); }
  const SegBlock* blk() const { return B.blocks.as<SegBlock>(); }
  void dot64(const double* a, const double* b, double* out, const int* mask) {
    check_hip(launch_seg_dot<double>(a, b, blk(), nb(), B.first.as<int32_t>(), B.n, B.partial.as<double>(), out, mask, s),
              "seg dot");
  }
  void dot32(const float* a, const float* b, double* out, const int* mask) {
    check_hip(launch_seg_dot<float>(a, b, blk(), nb(), B.first.as<int32_t>(), B.n, B.partial.as<double>(), out, mask, s),
              "seg dot");
  }
  template <class TX, class TY>
  void axpby(const double* ca, double ka, const TX* x, const double* cb, double kb, TY* y, const int* mask) {
    check_hip(launch_seg_axpby<TX, TY>(blk(), nb(), ca, ka, x, cb, kb, y, mask, s), "seg axpby");
  }
  dim3 sg() const { return dim3((B.n + 63) / 64); }
  // y = H_eff x for all problems under `mask`, FP64 (x64 -> t64) or low precision (p32 -> Ap32)
  void heff(bool fp64, const int* mask) {
    Bases<double> d64{};
    Bases<float> d32{};
    for (size_t c = 0; c < B.phase1.size(); ++c)
      for (int ph = 1; ph <= 2; ++ph) {
        const std::vector<MergedLaunch>& Ls = ph == 1 ? B.phase1[c] : B.phase2[c];
        // the launches of one phase are independent: the first on s, the others on side streams
        const int nside = std::min<int>((int)B.side.size(), (int)Ls.size() - 1);
        if (nside > 0) {
          check_hip(hipEventRecord(B.ev_fork, s), "fork");
          for (int k = 0; k < nside; ++k) check_hip(hipStreamWaitEvent(B.side[k], B.ev_fork, 0), "fork wait");
        }
        for (size_t i = 0; i < Ls.size(); ++i) {
          const MergedLaunch& L = Ls[i];
          hipStream_t q = (i == 0 || nside == 0) ? s : B.side[(i - 1) % nside];
          hipError_t e;
          if (fp64)
            e = launch_gemm_f64(L.desc(LCC_FP64), d64, q, B.table64.as<Bases<double>>(), mask);
          else if (prec == LCC_FP32)
            e = launch_gemm_f32(L.desc(LCC_FP32), d32, q, B.table32.as<Bases<float>>(), mask);
          else
            e = launch_gemm_bf16x3(L.desc(LCC_BF16X3), d32, q, B.table32.as<Bases<float>>(), mask);
          check_hip(e, "batched gemm");
        }
        for (int k = 0; k < nside; ++k) {
          check_hip(hipEventRecord(B.ev_join[k], B.side[k]), "join");
          check_hip(hipStreamWaitEvent(s, B.ev_join[k], 0), "join wait");
        }
      }
    hipError_t e = fp64 ? launch_reduce_f64(B.reduce_groups.as<ReduceGroup>(), B.reduce_tiles.as<ReduceTile>(),
                                            B.n_reduce_tiles, d64, s, B.table64.as<Bases<double>>(), mask)
                        : launch_reduce_f32(B.reduce_groups.as<ReduceGroup>(), B.reduce_tiles.as<ReduceTile>(),
                                            B.n_reduce_tiles, d32, s, B.table32.as<Bases<float>>(), mask);
    check_hip(e, "batched reduce");
  }
  // t64 = Q (H - e0) Q x64 under mask (x64 already in range(Q))
  void A64(const int* mask, const int* hv_mask) {
    heff(true, mask);
    axpby<double, double>(B.S.e0neg, 1.0, B.x64.as<double>(), nullptr, 1.0, B.t64.as<double>(), mask);
    dot64(B.v64.as<double>(), B.t64.as<double>(), B.S.dot, hv_mask);
    axpby<double, double>(B.S.dot, -1.0, B.v64.as<double>(), nullptr, 1.0, B.t64.as<double>(), hv_mask);
  }
  void A32(const int* mask, const int* hv_mask) {
    heff(false, mask);
    axpby<float, float>(B.S.e0neg, 1.0, B.p32.as<float>(), nullptr, 1.0, B.Ap32.as<float>(), mask);
    dot32(B.v32.as<float>(), B.Ap32.as<float>(), B.S.dot, hv_mask);
    axpby<float, float>(B.S.dot, -1.0, B.v32.as<float>(), nullptr, 1.0, B.Ap32.as<float>(), hv_mask);
  }
  // one reliable-update CG iteration of every active problem (graph-capturable: kernels only)
  void iteration(double delta, int max_iter, int max_outer) {
    Scalars& S = B.S;
    float* p32 = B.p32.as<float>();
    float* Ap32 = B.Ap32.as<float>();
    float* r32 = B.r32.as<float>();
    float* d32 = B.d32.as<float>();
    A32(S.active, S.hv_active);
    dot32(p32, Ap32, S.pAp, S.active);
    hipLaunchKernelGGL(k_alpha, sg(), dim3(64), 0, s, S, B.n);
    axpby<float, float>(S.alpha, 1.0, p32, nullptr, 1.0, d32, S.active);
    axpby<float, float>(S.alpha, -1.0, Ap32, nullptr, 1.0, r32, S.active);
    dot32(r32, r32, S.rr_new, S.active);
    hipLaunchKernelGGL(k_after_r, sg(), dim3(64), 0, s, S, B.n, delta, max_iter);
    // continuing problems: p = r + beta p
    axpby<float, float>(nullptr, 1.0, r32, S.beta, 1.0, p32, S.cont);
    // refreshing problems: x += sc d, d = 0, true residual in FP64, new units
    double* x64 = B.x64.as<double>();
    axpby<float, double>(S.sc, 1.0, d32, nullptr, 1.0, x64, S.refresh);
    dot64(B.v64.as<double>(), x64, S.dot, S.hv_refresh);
    axpby<double, double>(S.dot, -1.0, B.v64.as<double>(), nullptr, 1.0, x64, S.hv_refresh);
    axpby<float, float>(nullptr, 0.0, d32, nullptr, 0.0, d32, S.refresh);
    A64(S.refresh, S.hv_refresh);
    axpby<double, double>(nullptr, 1.0, B.bq.as<double>(), nullptr, -1.0, B.t64.as<double>(), S.refresh);  // t = bq - A x
    dot64(B.t64.as<double>(), B.t64.as<double>(), S.dot, S.refresh);
    hipLaunchKernelGGL(k_refresh, sg(), dim3(64), 0, s, S, B.n, max_iter, max_outer);
    axpby<double, float>(S.inv_sc, 1.0, B.t64.as<double>(), nullptr, 0.0, r32, S.ract);
    axpby<float, float>(nullptr, 1.0, r32, S.pscale, 1.0, p32, S.ract);
    dot32(r32, r32, S.dot, S.ract);
    hipLaunchKernelGGL(k_rr_refresh, sg(), dim3(64), 0, s, S, B.n);
  }
};

}  // namespace

lcc_status batch_solve(Batch& B, const lcc_solve_opts& o, const double* const* b, const double* e0,
                       const double* const* v, double* const* x, lcc_solve_info* infos) {
  const auto t0 = std::chrono::steady_clock::now();
  const int prec = o.precision;
  if (prec != LCC_FP32 && prec != LCC_BF16X3)
    throw Error{LCC_ERR_ARG, "batched solves run the mixed-precision method (LCC_FP32 or LCC_BF16X3)"};
  const int max_iter = o.max_iter > 0 ? o.max_iter : 1000;
  const double tol = o.tol > 0 ? o.tol : 1e-10;
  const double delta = o.inner_tol > 0 ? o.inner_tol : 0.1;
  const int max_outer = o.max_outer > 0 ? o.max_outer : 200;
  hipStream_t s = B.stream;
  // order after the caller's work on the context stream
  hipEvent_t ev;
  check_hip(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
  check_hip(hipEventRecord(ev, B.ctx->stream), "record");
  check_hip(hipStreamWaitEvent(s, ev, 0), "wait");
  Runner R{B, s, prec};
  Scalars& S = B.S;
  // inputs into the arena
  std::vector<double> e0neg(B.n), zero(B.n, 0.0);
  std::vector<int> hv(B.n);
  for (int p = 0; p < B.n; ++p) {
    const size_t bytes = sizeof(double) * B.envs[p]->n_elements;
    if (!b[p] || !x[p]) throw Error{LCC_ERR_ARG, "b and x must be given for every problem"};
    if (!std::isfinite(e0[p])) throw Error{LCC_ERR_NAN, "e0 is not finite"};
    check_hip(hipMemcpyAsync(B.bq.as<double>() + B.off[p], b[p], bytes, hipMemcpyDeviceToDevice, s), "copy b");
    check_hip(hipMemcpyAsync(B.x64.as<double>() + B.off[p], x[p], bytes, hipMemcpyDeviceToDevice, s), "copy x");
    if (v && v[p]) check_hip(hipMemcpyAsync(B.v64.as<double>() + B.off[p], v[p], bytes, hipMemcpyDeviceToDevice, s), "copy v");
    e0neg[p] = -e0[p];
    hv[p] = (v && v[p]) ? 1 : 0;
  }
  check_hip(hipMemcpyAsync(S.e0neg, e0neg.data(), sizeof(double) * B.n, hipMemcpyHostToDevice, s), "e0");
  check_hip(hipMemcpyAsync(S.has_v, hv.data(), sizeof(int) * B.n, hipMemcpyHostToDevice, s), "has_v");
  check_hip(hipStreamSynchronize(s), "inputs");
  // projections of b and x, v in FP32, ||Q b||
  R.dot64(B.v64.as<double>(), B.bq.as<double>(), S.dot, S.has_v);
  R.axpby<double, double>(S.dot, -1.0, B.v64.as<double>(), nullptr, 1.0, B.bq.as<double>(), S.has_v);
  R.dot64(B.v64.as<double>(), B.x64.as<double>(), S.dot, S.has_v);
  R.axpby<double, double>(S.dot, -1.0, B.v64.as<double>(), nullptr, 1.0, B.x64.as<double>(), S.has_v);
  R.axpby<double, float>(nullptr, 1.0, B.v64.as<double>(), nullptr, 0.0, B.v32.as<float>(), S.has_v);
  R.dot64(B.bq.as<double>(), B.bq.as<double>(), S.bn, nullptr);
  {
    std::vector<double> bn(B.n), tolbn(B.n);
    check_hip(hipMemcpyAsync(bn.data(), S.bn, sizeof(double) * B.n, hipMemcpyDeviceToHost, s), "bn");
    check_hip(hipStreamSynchronize(s), "bn");
    for (int p = 0; p < B.n; ++p) tolbn[p] = tol * std::sqrt(bn[p]);
    check_hip(hipMemcpyAsync(S.tol_bn, tolbn.data(), sizeof(double) * B.n, hipMemcpyHostToDevice, s), "tol");
  }
  // first FP64 residual for every problem: t = bq - A x
  std::vector<int> ones(B.n, 1);
  check_hip(hipMemcpyAsync(S.refresh, ones.data(), sizeof(int) * B.n, hipMemcpyHostToDevice, s), "mask");
  check_hip(hipMemcpyAsync(S.hv_refresh, hv.data(), sizeof(int) * B.n, hipMemcpyHostToDevice, s), "mask");
  R.A64(S.refresh, S.hv_refresh);
  R.axpby<double, double>(nullptr, 1.0, B.bq.as<double>(), nullptr, -1.0, B.t64.as<double>(), S.refresh);
  R.dot64(B.t64.as<double>(), B.t64.as<double>(), S.dot, nullptr);
  hipLaunchKernelGGL(k_start, R.sg(), dim3(64), 0, s, S, B.n);
  R.axpby<double, float>(S.inv_sc, 1.0, B.t64.as<double>(), nullptr, 0.0, B.r32.as<float>(), S.active);
  R.axpby<float, float>(nullptr, 1.0, B.r32.as<float>(), nullptr, 0.0, B.p32.as<float>(), S.active);
  R.axpby<float, float>(nullptr, 0.0, B.d32.as<float>(), nullptr, 0.0, B.d32.as<float>(), nullptr);
  R.dot32(B.r32.as<float>(), B.r32.as<float>(), S.dot, S.active);
  hipLaunchKernelGGL(k_rr_init, R.sg(), dim3(64), 0, s, S, B.n);
  check_hip(hipGetLastError(), "start");
  // capture one iteration and replay it until every problem has stopped
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  check_hip(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
  R.iteration(delta, max_iter, max_outer);
  check_hip(hipStreamEndCapture(s, &graph), "end capture");
  check_hip(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "instantiate");
  constexpr int kCheckEvery = 4;
  int replays = 0;
  for (;;) {
    for (int k = 0; k < kCheckEvery; ++k) check_hip(hipGraphLaunch(exec, s), "graph launch");
    replays += kCheckEvery;
    hipLaunchKernelGGL(k_count_active, dim3(1), dim3(64), 0, s, S.active, B.n, B.count.as<int>());
    check_hip(hipMemcpyAsync(B.host_count, B.count.p, sizeof(int), hipMemcpyDeviceToHost, s), "count");
    check_hip(hipStreamSynchronize(s), "count sync");
    if (B.host_count[0] == 0 || replays > max_iter + kCheckEvery) break;
  }
  (void)hipGraphExecDestroy(exec);
  (void)hipGraphDestroy(graph);
  // final FP64 residual and energy per problem
  check_hip(hipMemcpyAsync(S.refresh, ones.data(), sizeof(int) * B.n, hipMemcpyHostToDevice, s), "mask");
  check_hip(hipMemcpyAsync(S.hv_refresh, hv.data(), sizeof(int) * B.n, hipMemcpyHostToDevice, s), "mask");
  R.A64(S.refresh, S.hv_refresh);
  R.axpby<double, double>(nullptr, 1.0, B.bq.as<double>(), nullptr, -1.0, B.t64.as<double>(), S.refresh);
  std::vector<double> rr(B.n), xr(B.n), bx(B.n), bn(B.n);
  std::vector<int> status(B.n), iters(B.n), outer(B.n);
  R.dot64(B.t64.as<double>(), B.t64.as<double>(), S.dot, nullptr);
  check_hip(hipMemcpyAsync(rr.data(), S.dot, sizeof(double) * B.n, hipMemcpyDeviceToHost, s), "rr");
  check_hip(hipStreamSynchronize(s), "rr");
  R.dot64(B.x64.as<double>(), B.t64.as<double>(), S.dot, nullptr);
  check_hip(hipMemcpyAsync(xr.data(), S.dot, sizeof(double) * B.n, hipMemcpyDeviceToHost, s), "xr");
  check_hip(hipStreamSynchronize(s), "xr");
  R.dot64(B.bq.as<double>(), B.x64.as<double>(), S.dot, nullptr);
  check_hip(hipMemcpyAsync(bx.data(), S.dot, sizeof(double) * B.n, hipMemcpyDeviceToHost, s), "bx");
  check_hip(hipMemcpyAsync(bn.data(), S.bn, sizeof(double) * B.n, hipMemcpyDeviceToHost, s), "bn");
  check_hip(hipMemcpyAsync(status.data(), S.status, sizeof(int) * B.n, hipMemcpyDeviceToHost, s), "status");
  check_hip(hipMemcpyAsync(iters.data(), S.iters, sizeof(int) * B.n, hipMemcpyDeviceToHost, s), "iters");
  check_hip(hipMemcpyAsync(outer.data(), S.outer, sizeof(int) * B.n, hipMemcpyDeviceToHost, s), "outer");
  for (int p = 0; p < B.n; ++p)
    check_hip(hipMemcpyAsync(x[p], B.x64.as<double>() + B.off[p], sizeof(double) * B.envs[p]->n_elements,
                             hipMemcpyDeviceToDevice, s), "copy x back");
  check_hip(hipStreamSynchronize(s), "results");
  (void)hipEventDestroy(ev);
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  lcc_status worst = LCC_OK;
  for (int p = 0; p < B.n; ++p) {
    int st = status[p] == ST_RUNNING ? LCC_NOT_CONVERGED : status[p];
    if (st < 0 && (worst >= 0 || st < worst)) worst = st;
    if (st == LCC_NOT_CONVERGED && worst == LCC_OK) worst = LCC_NOT_CONVERGED;
    if (infos) {
      lcc_solve_info& I = infos[p];
      I = lcc_solve_info{};
      I.iterations = iters[p];
      I.outer = outer[p];
      I.applies_low = iters[p];
      I.applies_fp64 = outer[p] + 2;
      const double nb = std::sqrt(bn[p]);
      I.rel_residual = nb > 0 ? std::sqrt(rr[p]) / nb : 0.0;
      I.hylleraas = -xr[p] - bx[p];
      I.e2 = -bx[p];
      I.ms_total = ms;
    }
  }
  return worst;
}

}  // namespace lcc
