// Environments, the enlarged two-site operators and the H_eff contraction plan.
//
// Transition-element figure (Implementation section): <Psi|H|Psi> is contracted site by
// site; cutting out the two-site tensor at (l, l+1) leaves
//     H_eff = sum_{w1} Lt^{w1} (x) Rt^{w1},          w1 = channels of MPO bond l+1,
//     Lt^{w1}[(a',s1'),(a,s1)] = sum_w W_l^{w,w1}[s1',s1] L^w[a',a]      (left block + site l)
//     Rt^{w1}[(s2',b'),(s2,b)] = sum_w2 W_{l+1}^{w1,w2}[s2',s2] R^w2[b',b] (site l+1 + right block)
// so that, with the two-site vector stored as one matrix X_q per middle-bond sector q
// (rows (a,s1), columns (s2,b)),
//     phase 1:  T_{w1,q} = Lt^{w1} X_q            (grouped GEMM over L blocks)
//     phase 2:  Y_{q'}  += T_{w1,q} Rt^{w1 T}     (grouped GEMM over R blocks),  q' = q + dq(w1).
// The MPO sums over w and w2 (the "W mixing") are folded in once per environment: a
// single contributing block is referenced with its coefficient as the GEMM alpha, several
// are pre-summed into a merged block.  Environments themselves are built on the device by
// the same grouped GEMM:  L_{j+1}^{w'} = sum W_j^{w,w'}[s',s] A^{s' T} L_j^w A^s.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <unordered_map>

#include "state.h"

namespace lcc {

void check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error{LCC_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e)};
}

void DevBuf::alloc(size_t n) {
  release();
  if (n == 0) n = 16;
  n = (n + 255) & ~(size_t)255;
  hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    throw Error{e == hipErrorOutOfMemory ? LCC_ERR_OOM : LCC_ERR_HIP,
                "device allocation of " + std::to_string(n) + " bytes failed: " + hipGetErrorString(e)};
  }
  bytes = n;
}


// ---------------------------------------------------------------------------------------
// Grouped GEMM launch construction
// ---------------------------------------------------------------------------------------
void GemmBuilder::group(int8_t c_base, int64_t c_off, int ldc, int m, int n, bool accumulate) {
  GemmGroup g{};
  g.c_off = c_off;
  g.ldc = ldc;
  g.m = m;
  g.n = n;
  g.c_base = c_base;
  g.accumulate = accumulate ? 1 : 0;
  g.term_begin = g.term_end = (int32_t)terms.size();
  groups.push_back(g);
}

void GemmBuilder::term(int8_t a_base, int64_t a_off, int lda, int8_t b_base, int64_t b_off, int ldb, int k,
                       double alpha) {
  GemmTerm t{};
  t.a_base = a_base;
  t.a_off = a_off;
  t.lda = lda;
  t.b_base = b_base;
  t.b_off = b_off;
  t.ldb = ldb;
  t.k = k;
  t.alpha = alpha;
  terms.push_back(t);
  GemmGroup& g = groups.back();
  g.term_end = (int32_t)terms.size();
  flops += 2.0 * g.m * (double)g.n * k;
}

namespace {

// Tile shape of a group: the one with the least padded output area plus a fixed per-tile
// cost (staging, descriptor loads, epilogue), so tiny blocks get small tiles and large
// blocks get large ones.
int shape_for(int m, int n, double tile_overhead) {
  int best = TILE_64x64;
  double best_cost = 1e300;
  for (int s = 0; s < kNumTileShapes; ++s) {
    const int bm = kTileShapes[s][0], bn = kTileShapes[s][1];
    const double tiles = (double)((m + bm - 1) / bm) * ((n + bn - 1) / bn);
    const double cost = tiles * (bm * (double)bn + tile_overhead);
    if (cost < best_cost) { best_cost = cost; best = s; }
  }
  return best;
}

}  // namespace

// One launch per tile shape.  Each term is cut into k-quads (SlotRec) whose A / B offsets
// point at the quad's first k, so the kernel walks a group's terms as one packed k stream.
std::vector<GemmLaunch> finalize(const GemmBuilder& b, bool ta, bool tb, hipStream_t s, double tile_overhead,
                                 bool longest_first) {
  std::vector<GemmLaunch> out;
  for (int shape = 0; shape < kNumTileShapes; ++shape) {
    const int bm = kTileShapes[shape][0], bn = kTileShapes[shape][1];
    std::vector<GemmTerm> terms;
    std::vector<SlotRec> slots;
    std::vector<GemmGroup> groups;
    std::vector<GemmTile> tiles;
    GemmLaunch L;
    std::set<std::pair<int, int64_t>> seen;
    // longest_first: groups in order of decreasing accumulation length, so that the long tiles
    // start first and the short ones fill the tail of the launch; else in the builder's order
    std::vector<int64_t> gcost(b.groups.size(), 0);
    for (size_t i = 0; i < b.groups.size(); ++i)
      for (int t = b.groups[i].term_begin; t < b.groups[i].term_end; ++t) gcost[i] += (b.terms[t].k + 3) / 4 * 4;
    std::vector<int> order(b.groups.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    if (longest_first)
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return gcost[x] > gcost[y]; });
    for (int oi : order) {
      const GemmGroup& g0 = b.groups[oi];
      if (g0.m <= 0 || g0.n <= 0) continue;
      if (shape_for(g0.m, g0.n, tile_overhead) != shape) continue;
      GemmGroup g = g0;
      g.slot_begin = (int32_t)slots.size();
      g.term_begin = (int32_t)terms.size();
      for (int t = g0.term_begin; t < g0.term_end; ++t) {
        const GemmTerm& tm = b.terms[t];
        if (tm.k <= 0) continue;
        // the kernels address an operand block with 32-bit byte offsets from its first element
        const int64_t ea = ta ? (int64_t)(tm.k - 1) * tm.lda + g.m : (int64_t)(g.m - 1) * tm.lda + tm.k;
        const int64_t eb = tb ? (int64_t)(g.n - 1) * tm.ldb + tm.k : (int64_t)(tm.k - 1) * tm.ldb + g.n;
        if (std::max(ea, eb) > (int64_t)INT32_MAX / (int64_t)sizeof(double))
          throw Error{LCC_ERR_ARG, "an operand block exceeds the 2 GiB reach of 32-bit offsets"};
        terms.push_back(tm);
        for (int k0 = 0; k0 < tm.k; k0 += 4) {
          SlotRec r{};
          r.a_off = tm.a_off + (ta ? (int64_t)k0 * tm.lda : k0);
          r.b_off = tm.b_off + (tb ? k0 : (int64_t)k0 * tm.ldb);
          r.lda = tm.lda;
          r.ldb = tm.ldb;
          r.alpha = tm.alpha;
          r.a_base = tm.a_base;
          r.b_base = tm.b_base;
          r.kv = (int8_t)std::min(4, tm.k - k0);
          slots.push_back(r);
        }
        L.flops += 2.0 * g.m * (double)g.n * tm.k;
        if (seen.insert({tm.a_base, tm.a_off}).second) L.elems_read += (double)g.m * tm.k;
        if (seen.insert({tm.b_base, tm.b_off}).second) L.elems_read += (double)tm.k * g.n;
      }
      if (slots.size() > (size_t)INT32_MAX) throw Error{LCC_ERR_ARG, "plan too large"};
      g.slot_end = (int32_t)slots.size();
      g.term_end = (int32_t)terms.size();
      g.tiles_n = (g.n + bn - 1) / bn;
      const int tiles_m = (g.m + bm - 1) / bm;
      const int gi = (int)groups.size();
      groups.push_back(g);
      for (int t = 0; t < tiles_m * g.tiles_n; ++t) tiles.push_back(GemmTile{gi, t});
      // MFMA work issued.  The term-walk kernels skip the 16 x 16 sub-tiles outside the block
      // (m, n padded to 16) and pad k to 4 (FP64 / FP32) or 32 (BF16x3) per term; the packed
      // kernels pad k to 16 per group of quads (FP64 / FP32, same sub-tile skip) or run whole
      // tiles with k padded to 32 (BF16x3).
      const int64_t nk = (int64_t)(g.slot_end - g.slot_begin) * 4;
      int64_t k4 = 0, k32 = 0;
      for (int t = g0.term_begin; t < g0.term_end; ++t) {
        k4 += (b.terms[t].k + 3) / 4 * 4;
        k32 += (b.terms[t].k + 31) / 32 * 32;
      }
      const double live = 2.0 * ((g.m + 15) / 16 * 16) * (double)((g.n + 15) / 16 * 16);
      const double whole = 2.0 * tiles_m * g.tiles_n * (double)bm * bn;
      for (int p = LCC_FP64; p <= LCC_FP32; ++p) {
        L.exec_flops[p][0] += live * k4;
        L.exec_flops[p][1] += live * ((nk + 15) / 16 * 16);
      }
      L.exec_flops[LCC_BF16X3][0] += live * k32;
      L.exec_flops[LCC_BF16X3][1] += whole * ((nk + 31) / 32 * 32);
      L.elems_written += (double)g.m * g.n;
    }
    if (tiles.empty()) continue;
    if (tiles.size() > (size_t)INT32_MAX) throw Error{LCC_ERR_ARG, "plan too large"};
    L.ta = ta;
    L.tb = tb;
    L.shape = shape;
    L.n_tiles = (int)tiles.size();
    L.n_slots = (int64_t)slots.size();
    // small tiles stage little per chunk: packing short terms into shared chunks pays there
    const bool small = bm * bn <= 1024;
    for (int p = 0; p < 3; ++p) L.packed[p] = small;
    upload(L.terms, terms, s);
    upload(L.slots, slots, s);
    upload(L.groups, groups, s);
    upload(L.tiles, tiles, s);
    out.push_back(std::move(L));
  }
  return out;
}

void run_gemm64(const std::vector<GemmLaunch>& Ls, const Bases<double>& b, hipStream_t s) {
  for (const GemmLaunch& L : Ls)
    check_hip(launch_gemm_f64(L.desc(LCC_FP64), b, s), "gemm f64 launch");
}

namespace {

struct MixBuilder {
  std::vector<MixTerm> terms;
  std::vector<MixGroup> groups;
  void group(int8_t dst_base, int64_t dst_off, int count, int8_t src_base) {
    MixGroup g{};
    g.dst_off = dst_off;
    g.count = count;
    g.dst_base = dst_base;
    g.src_base = src_base;
    g.term_begin = g.term_end = (int32_t)terms.size();
    groups.push_back(g);
  }
  void term(int64_t src_off, double alpha) {
    terms.push_back(MixTerm{src_off, alpha});
    groups.back().term_end = (int32_t)terms.size();
  }
};

void run_mix(const MixBuilder& mb, const Bases<double>& b, hipStream_t s) {
  std::vector<MixTile> tiles;
  for (size_t g = 0; g < mb.groups.size(); ++g) {
    const int chunks = (mb.groups[g].count + 1023) / 1024;
    for (int c = 0; c < chunks; ++c) tiles.push_back(MixTile{(int32_t)g, c});
  }
  if (tiles.empty()) return;
  DevBuf dt, dg, dtl;
  upload(dt, mb.terms, s);
  upload(dg, mb.groups, s);
  upload(dtl, tiles, s);
  check_hip(launch_mix_f64(dt.as<MixTerm>(), dg.as<MixGroup>(), dtl.as<MixTile>(), (int)tiles.size(), b, s),
            "mix launch");
  check_hip(hipStreamSynchronize(s), "mix sync");
}

// ---------------------------------------------------------------------------------------
// MPS on the device
// ---------------------------------------------------------------------------------------

}  // namespace

void load_mps(const lcc_mps_desc& d, int N, int two_sz, hipStream_t s, DeviceMps& out) {
  if (d.n_sites < 2 || !d.bond_offsets || !d.sectors || !d.block_offsets || !d.blocks)
    throw Error{LCC_ERR_ARG, "incomplete MPS descriptor"};
  const int K = d.n_sites;
  out.K = K;
  out.bonds.resize(K + 1);
  for (int j = 0; j <= K; ++j) {
    const int b0 = d.bond_offsets[j], b1 = d.bond_offsets[j + 1];
    if (b1 < b0) throw Error{LCC_ERR_ARG, "bond offsets must be non-decreasing"};
    Bond& B = out.bonds[j];
    for (int i = b0; i < b1; ++i) {
      const lcc_sector& sc = d.sectors[i];
      if (sc.dim <= 0) throw Error{LCC_ERR_ARG, "sector dimensions must be positive"};
      QN q(sc.n, sc.two_sz);
      if (!B.q.empty() && !(B.q.back() < q)) throw Error{LCC_ERR_ARG, "bond sectors must be strictly increasing"};
      B.index[q] = (int)B.q.size();
      B.q.push_back(q);
      B.dim.push_back(sc.dim);
    }
  }
  if (out.bonds[0].q.size() != 1 || out.bonds[0].q[0] != QN(0, 0) || out.bonds[0].dim[0] != 1)
    throw Error{LCC_ERR_QN, "bond 0 must hold the single sector (0, 0) of dimension 1"};
  if (out.bonds[K].q.size() != 1 || out.bonds[K].q[0] != QN(N, two_sz) || out.bonds[K].dim[0] != 1)
    throw Error{LCC_ERR_QN, "bond K must hold the single sector (N, 2Sz) of dimension 1"};
  out.sites.resize(K);
  int64_t total = 0;
  for (int j = 0; j < K; ++j) {
    std::set<std::pair<int, int>> seen;
    for (int64_t i = d.block_offsets[j]; i < d.block_offsets[j + 1]; ++i) {
      const lcc_mps_block& b = d.blocks[i];
      const Bond &L = out.bonds[j], &R = out.bonds[j + 1];
      if (b.left < 0 || b.left >= (int)L.q.size() || b.right < 0 || b.right >= (int)R.q.size() || b.s < 0 ||
          b.s > 3 || !b.data)
        throw Error{LCC_ERR_ARG, "MPS block index out of range at site " + std::to_string(j)};
      if (L.q[b.left] + local_qn(b.s) != R.q[b.right])
        throw Error{LCC_ERR_QN, "MPS block violates the (N, 2Sz) rule at site " + std::to_string(j)};
      if (!seen.insert({b.left, b.s}).second) throw Error{LCC_ERR_ARG, "duplicate MPS block"};
      SiteBlock sb{b.left, b.s, b.right, total, L.dim[b.left], R.dim[b.right]};
      total += (int64_t)sb.rows * sb.cols;
      out.sites[j].push_back(sb);
    }
  }
  std::vector<double> host(total);
  for (int j = 0; j < K; ++j) {
    int64_t i = d.block_offsets[j];
    for (const SiteBlock& sb : out.sites[j]) {
      std::memcpy(host.data() + sb.off, d.blocks[i].data, sizeof(double) * sb.rows * sb.cols);
      ++i;
    }
  }
  for (double v : host)
    if (!std::isfinite(v)) throw Error{LCC_ERR_NAN, "non-finite MPS entry"};
  upload(out.data, host, s);
}

// ---------------------------------------------------------------------------------------
// Environment steps
// ---------------------------------------------------------------------------------------
static inline double wcoef(const MpoEntry& e, int sp, int s) { return e.m[sp * 4 + s]; }

// L_{j+1}^{w'}[a', a] = sum_{w,s',s} W_j^{w,w'}[s',s] (A'^{s'T} L_j^w A^s)[a', a], with A' the bra's
// tensor (rows of L) and A the ket's (columns of L); the same MPS on both sides for H_eff.
Environment left_step(const Environment& L, const DeviceMps& mps, int j, const Mpo& mpo, hipStream_t st) {
  return left_step(L, mps, mps, j, mpo, st);
}

Environment left_step(const Environment& L, const DeviceMps& bra, const DeviceMps& ket, int j, const Mpo& mpo,
                      hipStream_t st) {
  const Bond& bn = bra.bonds[j + 1];
  const Bond& bn0 = ket.bonds[j + 1];
  std::map<std::pair<int, int>, int> A, Ab;  // (left sector, s) -> block of the ket / the bra
  for (size_t i = 0; i < ket.sites[j].size(); ++i) A[{ket.sites[j][i].l, ket.sites[j][i].s}] = (int)i;
  for (size_t i = 0; i < bra.sites[j].size(); ++i) Ab[{bra.sites[j][i].l, bra.sites[j][i].s}] = (int)i;
  auto Ablk = [&](int l, int s) -> const SiteBlock* {
    auto it = A.find({l, s});
    return it == A.end() ? nullptr : &ket.sites[j][it->second];
  };
  auto Abra = [&](int l, int s) -> const SiteBlock* {
    auto it = Ab.find({l, s});
    return it == Ab.end() ? nullptr : &bra.sites[j][it->second];
  };
  // enumerate sandwiches S(w, s', s, c) and their destinations
  struct SKey { int w, sp, s, c; bool operator<(const SKey& o) const { return std::tie(w, sp, s, c) < std::tie(o.w, o.sp, o.s, o.c); } };
  std::map<SKey, int64_t> s_off;      // sandwich -> offset in S buffer
  std::map<std::tuple<int, int, int>, int64_t> u_off;  // (w, s, c) -> offset in U buffer
  struct Dest { int wp, ap, a; };
  std::map<std::tuple<int, int, int>, std::vector<std::pair<SKey, double>>> dest;  // (w', a, a') -> terms
  std::vector<std::vector<int>> L_by_w(mpo.dq[j].size());
  for (size_t i = 0; i < L.blocks.size(); ++i) L_by_w[L.blocks[i].w].push_back((int)i);
  int64_t u_total = 0, s_total = 0;
  for (const MpoEntry& e : mpo.W[j]) {
    for (int bi : L_by_w[e.win]) {
      const EnvBlock& lb = L.blocks[bi];
      for (int sp = 0; sp < 4; ++sp)
        for (int s = 0; s < 4; ++s) {
          const double c = wcoef(e, sp, s);
          if (c == 0.0) continue;
          const SiteBlock* as = Ablk(lb.c, s);
          const SiteBlock* ap = Abra(lb.r, sp);
          if (!as || !ap) continue;
          auto uk = std::make_tuple(lb.w, s, lb.c);
          if (!u_off.count(uk)) { u_off[uk] = u_total; u_total += (int64_t)lb.rows * as->cols; }
          SKey sk{lb.w, sp, s, lb.c};
          if (!s_off.count(sk)) { s_off[sk] = s_total; s_total += (int64_t)ap->cols * as->cols; }
          dest[std::make_tuple(e.wout, as->r, ap->r)].push_back({sk, c});
        }
    }
  }
  Environment out;
  out.nsec = (int)bn0.q.size();
  // output blocks in (w', a) order
  for (const auto& kv : dest) {
    EnvBlock b;
    b.w = std::get<0>(kv.first);
    b.c = std::get<1>(kv.first);
    b.r = std::get<2>(kv.first);
    if (bn.q[b.r] != bn0.q[b.c] + mpo.dq[j + 1][b.w]) throw Error{LCC_ERR_QN, "internal: environment charge mismatch"};
    b.rows = bn.dim[b.r];
    b.cols = bn0.dim[b.c];
    b.off = out.size;
    out.size += (int64_t)b.rows * b.cols;
    out.lookup[(int64_t)b.w * out.nsec + b.c] = (int)out.blocks.size();
    out.blocks.push_back(b);
  }
  out.data.alloc(sizeof(double) * std::max<int64_t>(out.size, 1));
  if (out.blocks.empty()) return out;
  DevBuf U, S;
  U.alloc(sizeof(double) * std::max<int64_t>(u_total, 1));
  S.alloc(sizeof(double) * std::max<int64_t>(s_total, 1));
  // step 1: U(w, s, c) = L^w[r<-c] A^s[c -> a]
  GemmBuilder g1;
  for (const auto& kv : u_off) {
    const int w = std::get<0>(kv.first), s = std::get<1>(kv.first), c = std::get<2>(kv.first);
    const EnvBlock& lb = L.blocks[L.find(w, c)];
    const SiteBlock* as = Ablk(c, s);
    g1.group(BASE_T, kv.second, as->cols, lb.rows, as->cols, false);
    g1.term(BASE_ENV, lb.off, lb.cols, BASE_MPS, as->off, as->cols, lb.cols, 1.0);
  }
  // step 2: S(w, s', s, c) = A'^{s'}[r -> a']^T U(w, s, c)
  GemmBuilder g2;
  for (const auto& kv : s_off) {
    const SKey& k = kv.first;
    const EnvBlock& lb = L.blocks[L.find(k.w, k.c)];
    const SiteBlock* as = Ablk(k.c, k.s);
    const SiteBlock* ap = Abra(lb.r, k.sp);
    g2.group(BASE_Y, kv.second, as->cols, ap->cols, as->cols, false);
    g2.term(BASE_MPS, ap->off, ap->cols, BASE_T, u_off[std::make_tuple(k.w, k.s, k.c)], as->cols, ap->rows, 1.0);
  }
  Bases<double> b{};
  b.p[BASE_ENV] = L.data.as<double>();
  b.p[BASE_MPS] = ket.data.as<double>();
  b.p[BASE_T] = U.as<double>();
  b.p[BASE_Y] = S.as<double>();
  b.p[BASE_X] = out.data.as<double>();
  {
    auto l1 = finalize(g1, false, false, st);
    run_gemm64(l1, b, st);
    Bases<double> b2 = b;
    b2.p[BASE_MPS] = bra.data.as<double>();
    auto l2 = finalize(g2, true, false, st);
    run_gemm64(l2, b2, st);
    check_hip(hipStreamSynchronize(st), "left step gemm");
  }
  // step 3: mix
  MixBuilder mb;
  for (const EnvBlock& ob : out.blocks) {
    mb.group(BASE_X, ob.off, ob.rows * ob.cols, BASE_Y);
    for (const auto& t : dest[std::make_tuple(ob.w, ob.c, ob.r)]) mb.term(s_off[t.first], t.second);
  }
  run_mix(mb, b, st);
  return out;
}

// R_j^{w}[b', b] = sum_{w',s',s} W_j^{w,w'}[s',s] (B'^{s'} R_{j+1}^{w'} B^{s T})[b', b], with B' the
// bra's tensor (rows of R) and B the ket's (columns of R).
Environment right_step(const Environment& R, const DeviceMps& mps, int j, const Mpo& mpo, hipStream_t st) {
  return right_step(R, mps, mps, j, mpo, st);
}

Environment right_step(const Environment& R, const DeviceMps& bra, const DeviceMps& ket, int j, const Mpo& mpo,
                       hipStream_t st) {
  const Bond& bj = bra.bonds[j];
  const Bond& bj0 = ket.bonds[j];
  std::map<std::pair<int, int>, int> B, Bb;  // (right sector, s) -> block of the ket / the bra
  for (size_t i = 0; i < ket.sites[j].size(); ++i) B[{ket.sites[j][i].r, ket.sites[j][i].s}] = (int)i;
  for (size_t i = 0; i < bra.sites[j].size(); ++i) Bb[{bra.sites[j][i].r, bra.sites[j][i].s}] = (int)i;
  auto Bblk = [&](int r, int s) -> const SiteBlock* {
    auto it = B.find({r, s});
    return it == B.end() ? nullptr : &ket.sites[j][it->second];
  };
  auto Bbra = [&](int r, int s) -> const SiteBlock* {
    auto it = Bb.find({r, s});
    return it == Bb.end() ? nullptr : &bra.sites[j][it->second];
  };
  struct SKey { int w, sp, s, c; bool operator<(const SKey& o) const { return std::tie(w, sp, s, c) < std::tie(o.w, o.sp, o.s, o.c); } };
  std::map<SKey, int64_t> s_off;
  std::map<std::tuple<int, int, int>, int64_t> u_off;  // (w', s, c)
  std::map<std::tuple<int, int, int>, std::vector<std::pair<SKey, double>>> dest;  // (w, b, b') -> terms
  std::vector<std::vector<int>> R_by_w(mpo.dq[j + 1].size());
  for (size_t i = 0; i < R.blocks.size(); ++i) R_by_w[R.blocks[i].w].push_back((int)i);
  int64_t u_total = 0, s_total = 0;
  for (const MpoEntry& e : mpo.W[j]) {
    for (int bi : R_by_w[e.wout]) {
      const EnvBlock& rb = R.blocks[bi];
      for (int sp = 0; sp < 4; ++sp)
        for (int s = 0; s < 4; ++s) {
          const double c = wcoef(e, sp, s);
          if (c == 0.0) continue;
          const SiteBlock* bs = Bblk(rb.c, s);
          const SiteBlock* bp = Bbra(rb.r, sp);
          if (!bs || !bp) continue;
          auto uk = std::make_tuple(rb.w, s, rb.c);
          if (!u_off.count(uk)) { u_off[uk] = u_total; u_total += (int64_t)rb.rows * bs->rows; }
          SKey sk{rb.w, sp, s, rb.c};
          if (!s_off.count(sk)) { s_off[sk] = s_total; s_total += (int64_t)bp->rows * bs->rows; }
          dest[std::make_tuple(e.win, bs->l, bp->l)].push_back({sk, c});
        }
    }
  }
  Environment out;
  out.nsec = (int)bj0.q.size();
  for (const auto& kv : dest) {
    EnvBlock b;
    b.w = std::get<0>(kv.first);
    b.c = std::get<1>(kv.first);
    b.r = std::get<2>(kv.first);
    if (bj.q[b.r] != bj0.q[b.c] + mpo.dq[j][b.w]) throw Error{LCC_ERR_QN, "internal: environment charge mismatch"};
    b.rows = bj.dim[b.r];
    b.cols = bj0.dim[b.c];
    b.off = out.size;
    out.size += (int64_t)b.rows * b.cols;
    out.lookup[(int64_t)b.w * out.nsec + b.c] = (int)out.blocks.size();
    out.blocks.push_back(b);
  }
  out.data.alloc(sizeof(double) * std::max<int64_t>(out.size, 1));
  if (out.blocks.empty()) return out;
  DevBuf U, S;
  U.alloc(sizeof(double) * std::max<int64_t>(u_total, 1));
  S.alloc(sizeof(double) * std::max<int64_t>(s_total, 1));
  // step 1: U(w', s, c) = R^{w'}[r <- c] B^s[b -> c]^T     (rows M_r, cols M_b)
  GemmBuilder g1;
  for (const auto& kv : u_off) {
    const int w = std::get<0>(kv.first), s = std::get<1>(kv.first), c = std::get<2>(kv.first);
    const EnvBlock& rb = R.blocks[R.find(w, c)];
    const SiteBlock* bs = Bblk(c, s);
    g1.group(BASE_T, kv.second, bs->rows, rb.rows, bs->rows, false);
    g1.term(BASE_ENV, rb.off, rb.cols, BASE_MPS, bs->off, bs->cols, rb.cols, 1.0);
  }
  // step 2: S(w', s', s, c) = B^{s'}[b' -> r] U(w', s, c)  (rows M_b', cols M_b)
  GemmBuilder g2;
  for (const auto& kv : s_off) {
    const SKey& k = kv.first;
    const EnvBlock& rb = R.blocks[R.find(k.w, k.c)];
    const SiteBlock* bs = Bblk(k.c, k.s);
    const SiteBlock* bp = Bbra(rb.r, k.sp);
    g2.group(BASE_Y, kv.second, bs->rows, bp->rows, bs->rows, false);
    g2.term(BASE_MPS, bp->off, bp->cols, BASE_T, u_off[std::make_tuple(k.w, k.s, k.c)], bs->rows, bp->cols, 1.0);
  }
  Bases<double> b{};
  b.p[BASE_ENV] = R.data.as<double>();
  b.p[BASE_MPS] = ket.data.as<double>();
  b.p[BASE_T] = U.as<double>();
  b.p[BASE_Y] = S.as<double>();
  b.p[BASE_X] = out.data.as<double>();
  {
    auto l1 = finalize(g1, false, true, st);
    run_gemm64(l1, b, st);
    Bases<double> b2 = b;
    b2.p[BASE_MPS] = bra.data.as<double>();
    auto l2 = finalize(g2, false, false, st);
    run_gemm64(l2, b2, st);
    check_hip(hipStreamSynchronize(st), "right step gemm");
  }
  MixBuilder mb;
  for (const EnvBlock& ob : out.blocks) {
    mb.group(BASE_X, ob.off, ob.rows * ob.cols, BASE_Y);
    for (const auto& t : dest[std::make_tuple(ob.w, ob.c, ob.r)]) mb.term(s_off[t.first], t.second);
  }
  run_mix(mb, b, st);
  return out;
}

Environment unit_env(hipStream_t st) {
  Environment e;
  e.nsec = 1;
  e.blocks.push_back(EnvBlock{0, 0, 0, 0, 1, 1});
  e.lookup[0] = 0;
  e.size = 1;
  std::vector<double> one{1.0};
  upload(e.data, one, st);
  return e;
}

// The identity channel of a canonical environment must be the identity matrix.
void check_identity(const Environment& E, int w_id, const Bond& bond, hipStream_t st, const char* which) {
  for (size_t q = 0; q < bond.q.size(); ++q) {
    const int bi = E.find(w_id, (int)q);
    if (bi < 0) throw Error{LCC_ERR_ARG, std::string(which) + " environment lacks its identity channel"};
    const EnvBlock& b = E.blocks[bi];
    std::vector<double> h((size_t)b.rows * b.cols);
    check_hip(hipMemcpyAsync(h.data(), E.data.as<double>() + b.off, h.size() * sizeof(double), hipMemcpyDeviceToHost, st),
              "identity check copy");
    check_hip(hipStreamSynchronize(st), "identity check sync");
    double worst = 0;
    for (int r = 0; r < b.rows; ++r)
      for (int c = 0; c < b.cols; ++c) worst = std::max(worst, std::fabs(h[(size_t)r * b.cols + c] - (r == c ? 1.0 : 0.0)));
    if (!(worst <= 1e-10))
      throw Error{LCC_ERR_ARG, std::string("MPS is not ") + which + "-canonical (deviation " + std::to_string(worst) + ")"};
  }
}

int channel_of_kind(const Mpo& mpo, int bond, int kind) {
  for (size_t i = 0; i < mpo.kind[bond].size(); ++i)
    if (mpo.kind[bond][i] == kind) return (int)i;
  return -1;
}

// ---------------------------------------------------------------------------------------
// build_env: environments, enlarged operators, vector layout, and the apply plan
// ---------------------------------------------------------------------------------------
Env* build_env(Context* ctx, const Hamiltonian& ham, const lcc_mps_desc& md, int site, bool one_site) {
  hipStream_t st = ctx->stream;
  const Mpo& mpo = ham.mpo;
  const int K = mpo.K;
  if (md.n_sites != K) throw Error{LCC_ERR_ARG, "MPS length differs from the Hamiltonian's orbital count"};
  if (one_site) {
    if (site < 0 || site >= K) throw Error{LCC_ERR_ARG, "one-site problem must satisfy 0 <= site < K"};
  } else if (site < 0 || site + 1 >= K) {
    throw Error{LCC_ERR_ARG, "two-site block must satisfy 0 <= site < K-1"};
  }
  DeviceMps mps;
  load_mps(md, ham.desc.N, ham.desc.two_sz, st, mps);

  // left environment at MPS bond `site`, right environment at MPS bond `site + 2` (two sites) or
  // `site + 1` (one site)
  const int rb = one_site ? site + 1 : site + 2;
  Environment L = unit_env(st);
  for (int j = 0; j < site; ++j) L = left_step(L, mps, j, mpo, st);
  Environment R = unit_env(st);
  for (int j = K - 1; j >= rb; --j) R = right_step(R, mps, j, mpo, st);
  // the identity channel of each environment certifies the canonical form of its sites
  const int w_left_id = channel_of_kind(mpo, site, 0), w_right_id = channel_of_kind(mpo, rb, 1);
  if (site > 0 && w_left_id >= 0) check_identity(L, w_left_id, mps.bonds[site], st, "left");
  if (rb < K && w_right_id >= 0) check_identity(R, w_right_id, mps.bonds[rb], st, "right");
  return make_env(ctx, mpo, site, mps.bonds[site], mps.bonds[rb], mps.bonds[site], mps.bonds[rb], L, R, false,
                  one_site);
}

// The MPO of the identity operator: one channel on every bond, the identity on every site.
Mpo identity_mpo(int K) {
  Mpo m;
  m.K = K;
  m.dq.assign(K + 1, std::vector<QN>{QN(0, 0)});
  m.kind.assign(K + 1, std::vector<int8_t>{0});
  m.W.assign(K, {});
  for (int j = 0; j < K; ++j) {
    MpoEntry e;
    e.win = 0;
    e.wout = 0;
    for (int q = 0; q < 16; ++q) e.m[q] = (q % 5 == 0) ? 1.0 : 0.0;
    m.W[j].push_back(e);
  }
  return m;
}

// Transition operator <bra| H |ket> with the bra's two-site block (site, site+1) cut out: left
// and right environments between the two MPS (transition-element figure), then the same
// enlarged operators and plan as an effective Hamiltonian, mapping the ket's two-site space onto
// the bra's.  The bra must be canonical around the block (its two-site space is the one of the
// local problem); the ket may be in any gauge.
Env* build_transition_env(Context* ctx, const Hamiltonian& ham, const lcc_mps_desc& bra_d, const lcc_mps_desc& ket_d,
                          int site, bool one_site) {
  hipStream_t st = ctx->stream;
  const Mpo& mpo = ham.mpo;
  const int K = mpo.K;
  if (bra_d.n_sites != K || ket_d.n_sites != K)
    throw Error{LCC_ERR_ARG, "MPS length differs from the Hamiltonian's orbital count"};
  if (one_site) {
    if (site < 0 || site >= K) throw Error{LCC_ERR_ARG, "one-site problem must satisfy 0 <= site < K"};
  } else if (site < 0 || site + 1 >= K) {
    throw Error{LCC_ERR_ARG, "two-site block must satisfy 0 <= site < K-1"};
  }
  const int rb = one_site ? site + 1 : site + 2;  // bond of the right environment
  DeviceMps bra, ket;
  load_mps(bra_d, ham.desc.N, ham.desc.two_sz, st, bra);
  load_mps(ket_d, ham.desc.N, ham.desc.two_sz, st, ket);
  {
    const Mpo id = identity_mpo(K);
    Environment L = unit_env(st);
    for (int j = 0; j < site; ++j) L = left_step(L, bra, j, id, st);
    if (site > 0) check_identity(L, 0, bra.bonds[site], st, "left");
    Environment R = unit_env(st);
    for (int j = K - 1; j >= rb; --j) R = right_step(R, bra, j, id, st);
    if (rb < K) check_identity(R, 0, bra.bonds[rb], st, "right");
  }
  Environment L = unit_env(st);
  for (int j = 0; j < site; ++j) L = left_step(L, bra, ket, j, mpo, st);
  Environment R = unit_env(st);
  for (int j = K - 1; j >= rb; --j) R = right_step(R, bra, ket, j, mpo, st);
  std::unique_ptr<Env> env(make_env(ctx, mpo, site, bra.bonds[site], bra.bonds[rb], ket.bonds[site], ket.bonds[rb],
                                    L, R, true, one_site));
  if (one_site)
    build_ket_site_tensor(*env, ket, st);
  else
    build_ket_tensor(*env, ket, ket, st);
  return env.release();
}

// The ket's own one-site tensor at the site of a one-site transition operator (input layout):
// its site tensor's blocks, copied into the (a, s, 0, b) blocks of the layout.
void build_ket_site_tensor(Env& E, const DeviceMps& ket, hipStream_t st) {
  std::map<std::pair<int, int>, const SiteBlock*> A;
  for (const SiteBlock& b : ket.sites[E.site]) A[{b.l, b.s}] = &b;
  E.x0.alloc(sizeof(double) * std::max<int64_t>(E.n_in, 1));
  check_hip(launch_fill_f64(E.x0.as<double>(), E.n_in, 0.0, st), "zero ket tensor");
  for (const lcc_block_entry& blk : E.layout_in) {
    auto it = A.find({blk.left, blk.s1});
    if (it == A.end() || it->second->r != blk.right) continue;
    const SiteBlock& sb = *it->second;
    check_hip(hipMemcpy2DAsync(E.x0.as<double>() + blk.offset, sizeof(double) * blk.ld,
                               ket.data.as<double>() + sb.off, sizeof(double) * sb.cols, sizeof(double) * sb.cols,
                               sb.rows, hipMemcpyDeviceToDevice, st),
              "ket site tensor");
  }
  check_hip(hipStreamSynchronize(st), "ket tensor");
}

// The ket's own two-site tensor at the block of a transition operator (input layout):
// x0[a,s1,s2,b] = sum_c A_site^{s1}[a,c] A_{site+1}^{s2}[c,b], with the two site tensors taken from
// t1 (site) and t2 (site + 1).
void build_ket_tensor(Env& E, const DeviceMps& t1, const DeviceMps& t2, hipStream_t st) {
  const int site = E.site;
  std::map<std::pair<int, int>, const SiteBlock*> A1, A2;
  for (const SiteBlock& b : t1.sites[site]) A1[{b.l, b.s}] = &b;
  for (const SiteBlock& b : t2.sites[site + 1]) A2[{b.l, b.s}] = &b;
  GemmBuilder g;
  for (const lcc_block_entry& blk : E.layout_in) {
    auto i1 = A1.find({blk.left, blk.s1});
    if (i1 == A1.end()) continue;
    auto i2 = A2.find({i1->second->r, blk.s2});
    if (i2 == A2.end() || i2->second->r != blk.right) continue;
    g.group(BASE_X, blk.offset, blk.ld, blk.rows, blk.cols, false);
    g.term(BASE_MPS, i1->second->off, i1->second->cols, BASE_ENV, i2->second->off, i2->second->cols,
           i1->second->cols, 1.0);
  }
  E.x0.alloc(sizeof(double) * std::max<int64_t>(E.n_in, 1));
  check_hip(launch_fill_f64(E.x0.as<double>(), E.n_in, 0.0, st), "zero ket tensor");
  Bases<double> b{};
  b.p[BASE_MPS] = t1.data.as<double>();
  b.p[BASE_ENV] = t2.data.as<double>();
  b.p[BASE_X] = E.x0.as<double>();
  run_gemm64(finalize(g, false, false, st), b, st);
  check_hip(hipStreamSynchronize(st), "ket tensor");
}

// The contraction plan of an environment for given planner parameters: channel chunks and
// the intermediate layout, the phase-1 and phase-2 grouped GEMMs, the split-K reduction and
// the workspaces.  Replaces any previous plan.
void plan_env(Env& E, const PlanParams& pp) {
  ++E.plan_epoch;
  Env* env = &E;
  Context* ctx = E.ctx;
  hipStream_t st = ctx->stream;
  const Bond& bl = E.bl;      // output (bra) rows and columns
  const Bond& br = E.br;
  const Bond& bl0 = E.bl_in;  // input (ket) rows and columns
  const Bond& br0 = E.br_in;
  auto& sec_index = E.in.sec_index;        // output sectors by (N, 2Sz)
  auto& sec_index_in = E.in.sec_index_in;  // input sectors
  auto& row_at_in = E.in.row_at_in;
  auto& col_at_in = E.in.col_at_in;
  auto& lt = E.in.lt;
  auto& rt = E.in.rt;
  const std::vector<QN>& dq_mid = E.in.dq_mid;
  E.params = pp;
  E.plan = Plan();
  // ---- active (w1, source sector) pairs and the intermediate layout
  const int D = env->D_mid;
  const int nsec = (int)env->sectors_in.size();  // source (input) sectors
  std::vector<char> lact((size_t)D * nsec, 0), ract((size_t)D * nsec, 0);
  for (const auto& kv : lt) {
    const int w1 = std::get<0>(kv.first);
    for (const auto& src : kv.second) lact[(size_t)w1 * nsec + row_at_in[{std::get<0>(src), std::get<1>(src)}].first] = 1;
  }
  for (const auto& kv : rt) {
    const int w1 = std::get<0>(kv.first);
    for (const auto& src : kv.second) ract[(size_t)w1 * nsec + col_at_in[{std::get<0>(src), std::get<1>(src)}].first] = 1;
  }
  // Two orders of the factorised product.  Left first (t_colmajor 0 or 1): T_{w1,m} = Lt^{w1} X_m
  // (nrows(m') x ncols(m), stored row- or column-major), then Y_{m'} += T Rt^{w1 T} with chains
  // over (w1, column blocks of m).  Right first (t_colmajor 2): T_{w1,m} = X_m Rt^{w1 T}
  // (nrows(m) x ncols(m'), row-major), then Y_{m'} += Lt^{w1} T with chains over (w1, row blocks
  // of m).  The flops are the same; the left enlarged operator has about one source block per
  // output row block, so left first gives short independent phase-1 products and right first
  // puts those short products in the accumulation chains.
  const bool right_first = pp.t_colmajor == 2;
  auto t_size = [&](int m, int mp) -> int64_t {
    return right_first ? (int64_t)env->sectors_in[m].nrows * env->sectors[mp].ncols
                       : (int64_t)env->sectors[mp].nrows * env->sectors_in[m].ncols;
  };
  // Channels are taken in order and cut into chunks whose intermediates fit the workspace
  // budget; each chunk reuses the same intermediate buffer (and, when small, stays in the
  // last-level cache between its two phases).
  const int64_t budget = std::max<int64_t>(ctx->t_budget_elems, 1);
  std::vector<int64_t> t_off((size_t)D * nsec, -1);
  std::vector<int> chunk_of(D, 0);
  int nchunks = 1;
  int64_t used = 0, t_max = 0;
  for (int w1 = 0; w1 < D; ++w1) {
    int64_t need = 0;
    for (int m = 0; m < nsec; ++m) {
      if (!lact[(size_t)w1 * nsec + m] || !ract[(size_t)w1 * nsec + m]) continue;
      auto it = sec_index.find(env->sectors_in[m].q + dq_mid[w1]);
      if (it == sec_index.end()) continue;
      need += t_size(m, it->second);
    }
    if (used > 0 && used + need > budget) {
      ++nchunks;
      used = 0;
    }
    chunk_of[w1] = nchunks - 1;
    for (int m = 0; m < nsec; ++m) {
      if (!lact[(size_t)w1 * nsec + m] || !ract[(size_t)w1 * nsec + m]) continue;
      auto it = sec_index.find(env->sectors_in[m].q + dq_mid[w1]);
      if (it == sec_index.end()) continue;
      t_off[(size_t)w1 * nsec + m] = used;
      used += t_size(m, it->second);
    }
    t_max = std::max(t_max, used);
  }
  env->t_elems = t_max;
  env->tbuf.alloc(sizeof(double) * std::max<int64_t>(t_max, 1));

  std::vector<GemmBuilder> p1(nchunks);
  if (!right_first) {
    // ---- phase 1: T_{w1,m}[(a',s1') rows] = sum Lt^{w1}[(a',s1'),(a,s1)] X_m[(a,s1) rows]
    for (int w1 = 0; w1 < D; ++w1)
      for (int m = 0; m < nsec; ++m) {
        const int64_t to = t_off[(size_t)w1 * nsec + m];
        if (to < 0) continue;
        GemmBuilder& B1 = p1[chunk_of[w1]];
        const MiddleSector& S = env->sectors_in[m];
        const MiddleSector& Sp = env->sectors[sec_index[S.q + dq_mid[w1]]];
        for (size_t i = 0; i < Sp.rows.size(); ++i) {
          const int ap = Sp.rows[i].first, sp = Sp.rows[i].second;
          // row-major T: the block of rows (a',s1') is Lt X;  column-major T: its transpose,
          // X^T Lt^T, is a row-major (ncols x dim a') block with leading dimension nrows(q')
          if (pp.t_colmajor)
            B1.group(BASE_T, to + Sp.row_off[i], Sp.nrows, S.ncols, bl.dim[ap], false);
          else
            B1.group(BASE_T, to + (int64_t)Sp.row_off[i] * S.ncols, S.ncols, bl.dim[ap], S.ncols, false);
          auto it = lt.find(std::make_tuple(w1, ap, sp));
          if (it == lt.end()) continue;
          for (const auto& src : it->second) {
            const auto ra = row_at_in[{std::get<0>(src), std::get<1>(src)}];
            if (ra.first != m) continue;
            const OperandRef& ref = std::get<2>(src);
            const int ka = bl0.dim[std::get<0>(src)];
            const int64_t x_off = S.off + (int64_t)S.row_off[ra.second] * S.ncols;
            if (pp.t_colmajor)
              B1.term(BASE_X, x_off, S.ncols, ref.base, ref.off, ka, ka, ref.alpha);
            else
              B1.term(ref.base, ref.off, ka, BASE_X, x_off, S.ncols, ka, ref.alpha);
          }
        }
      }
  } else {
    // ---- phase 1: T_{w1,m}[:, (s2',b')] = sum X_m[:, (s2,b)] Rt^{w1}[(s2',b'),(s2,b)]^T
    for (int w1 = 0; w1 < D; ++w1)
      for (int m = 0; m < nsec; ++m) {
        const int64_t to = t_off[(size_t)w1 * nsec + m];
        if (to < 0) continue;
        GemmBuilder& B1 = p1[chunk_of[w1]];
        const MiddleSector& S = env->sectors_in[m];
        const MiddleSector& Sp = env->sectors[sec_index[S.q + dq_mid[w1]]];
        for (size_t jx = 0; jx < Sp.cols.size(); ++jx) {
          const int s2p = Sp.cols[jx].first, bp = Sp.cols[jx].second;
          B1.group(BASE_T, to + Sp.col_off[jx], Sp.ncols, S.nrows, br.dim[bp], false);
          auto it = rt.find(std::make_tuple(w1, s2p, bp));
          if (it == rt.end()) continue;
          for (const auto& src : it->second) {
            const auto ca = col_at_in[{std::get<0>(src), std::get<1>(src)}];
            if (ca.first != m) continue;
            const OperandRef& ref = std::get<2>(src);
            const int kb = br0.dim[std::get<1>(src)];
            B1.term(BASE_X, S.off + S.col_off[ca.second], S.ncols, ref.base, ref.off, kb, kb, ref.alpha);
          }
        }
      }
  }
  // ---- phase 2: each output block's chain is cut at chunk boundaries and, inside a chunk, into
  // parts of about pp.split_k; parts write partial tiles that one ordered reduction adds into y.
  std::vector<GemmBuilder> p2(nchunks);
  std::vector<ReduceGroup> red;
  int64_t work = 0;
  double flops2 = 0;
  // A phase-2 group (one output block, or one split-K part of it) before emission.
  struct Emit {
    int chunk = 0, first_w1 = -1, jx = 0;
    int8_t c_base = BASE_Y;
    int64_t c_off = 0;
    int ldc = 0, m = 0, n = 0;
    std::vector<GemmTerm> terms;
  };
  // the parts of one output block (gm x gn at y_off, leading dimension ldc) from its chain
  auto emit_block = [&](std::vector<Emit>& emits, const std::vector<std::vector<GemmTerm>>& per,
                        const std::vector<std::vector<int>>& per_w1, int jx, int64_t y_off, int ldc, int gm, int gn) {
    struct Part { int chunk; size_t b, e; };
    std::vector<Part> parts;
    for (int c = 0; c < nchunks; ++c) {
      const auto& T = per[c];
      if (T.empty()) continue;
      int64_t ksum = 0;
      for (const GemmTerm& t : T) ksum += t.k;
      int np = (int)std::min<int64_t>(std::max<int64_t>(1, (ksum + pp.split_k - 1) / pp.split_k), 64);
      np = std::min<int>(np, (int)T.size());
      size_t i = 0;
      int64_t acc = 0;
      for (int p = 0; p < np; ++p) {
        const size_t b0 = i;
        const int64_t goal = (ksum * (p + 1)) / np;
        const size_t left = (size_t)(np - p - 1);
        do {
          acc += T[i].k;
          ++i;
        } while (i < T.size() && acc < goal && (T.size() - i) > left);
        if (p == np - 1) i = T.size();
        parts.push_back(Part{c, b0, i});
      }
    }
    if (parts.size() <= 1) {
      Emit em;
      em.chunk = parts.empty() ? 0 : parts[0].chunk;
      em.first_w1 = parts.empty() || parts[0].b == parts[0].e ? -1 : per_w1[em.chunk][parts[0].b];
      em.jx = jx;
      em.c_base = BASE_Y;
      em.c_off = y_off;
      em.ldc = ldc;
      em.m = gm;
      em.n = gn;
      if (!parts.empty()) em.terms.assign(per[em.chunk].begin() + parts[0].b, per[em.chunk].begin() + parts[0].e);
      emits.push_back(std::move(em));
      return;
    }
    const int64_t mn = (int64_t)gm * gn;
    const int64_t woff = work;
    for (size_t p = 0; p < parts.size(); ++p) {
      Emit em;
      em.chunk = parts[p].chunk;
      em.first_w1 = per_w1[em.chunk][parts[p].b];
      em.jx = jx;
      em.c_base = BASE_WORK;
      em.c_off = woff + (int64_t)p * mn;
      em.ldc = gn;
      em.m = gm;
      em.n = gn;
      em.terms.assign(per[em.chunk].begin() + parts[p].b, per[em.chunk].begin() + parts[p].e);
      emits.push_back(std::move(em));
    }
    work += (int64_t)parts.size() * mn;
    ReduceGroup rg{};
    rg.dst_off = y_off;
    rg.src_off = woff;
    rg.ldc = ldc;
    rg.m = gm;
    rg.n = gn;
    rg.parts = (int32_t)parts.size();
    red.push_back(rg);
  };
  for (int mp = 0; mp < (int)env->sectors.size(); ++mp) {
    const MiddleSector& Sp = env->sectors[mp];
    std::vector<Emit> emits;
    if (!right_first) {
      // Y_{m'}[:, (s2',b')] = sum_{w1,(s2,b)} T_{w1,m}[:, (s2,b)] Rt^{w1}[(s2',b'),(s2,b)]^T
      for (size_t jx = 0; jx < Sp.cols.size(); ++jx) {
        const int s2p = Sp.cols[jx].first, bp = Sp.cols[jx].second;
        const int gm = Sp.nrows, gn = br.dim[bp];
        std::vector<std::vector<GemmTerm>> per(nchunks);
        std::vector<std::vector<int>> per_w1(nchunks);
        for (int w1 = 0; w1 < D; ++w1) {
          auto si = sec_index_in.find(Sp.q - dq_mid[w1]);
          if (si == sec_index_in.end()) continue;
          const int m = si->second;
          const int64_t to = t_off[(size_t)w1 * nsec + m];
          if (to < 0) continue;
          auto it = rt.find(std::make_tuple(w1, s2p, bp));
          if (it == rt.end()) continue;
          const MiddleSector& S = env->sectors_in[m];
          for (const auto& src : it->second) {
            const auto ca = col_at_in[{std::get<0>(src), std::get<1>(src)}];
            if (ca.first != m) continue;
            const OperandRef& ref = std::get<2>(src);
            const int kb = br0.dim[std::get<1>(src)];
            GemmTerm t{};
            t.a_base = BASE_T;
            if (pp.t_colmajor) {  // columns (s2,b) of a column-major block: stored k x m
              t.a_off = to + (int64_t)S.col_off[ca.second] * gm;
              t.lda = gm;
            } else {
              t.a_off = to + S.col_off[ca.second];
              t.lda = S.ncols;
            }
            t.b_base = ref.base;
            t.b_off = ref.off;
            t.ldb = kb;
            t.k = kb;
            t.alpha = ref.alpha;
            per[chunk_of[w1]].push_back(t);
            per_w1[chunk_of[w1]].push_back(w1);
            flops2 += 2.0 * gm * (double)gn * kb;
          }
        }
        emit_block(emits, per, per_w1, (int)jx, Sp.off + Sp.col_off[jx], Sp.ncols, gm, gn);
      }
    } else {
      // Y_{m'}[(a',s1') rows, :] = sum_{w1,(a,s1)} Lt^{w1}[(a',s1'),(a,s1)] T_{w1,m}[(a,s1) rows, :]
      for (size_t ix = 0; ix < Sp.rows.size(); ++ix) {
        const int ap = Sp.rows[ix].first, sp = Sp.rows[ix].second;
        const int gm = bl.dim[ap], gn = Sp.ncols;
        std::vector<std::vector<GemmTerm>> per(nchunks);
        std::vector<std::vector<int>> per_w1(nchunks);
        for (int w1 = 0; w1 < D; ++w1) {
          auto si = sec_index_in.find(Sp.q - dq_mid[w1]);
          if (si == sec_index_in.end()) continue;
          const int m = si->second;
          const int64_t to = t_off[(size_t)w1 * nsec + m];
          if (to < 0) continue;
          auto it = lt.find(std::make_tuple(w1, ap, sp));
          if (it == lt.end()) continue;
          const MiddleSector& S = env->sectors_in[m];
          for (const auto& src : it->second) {
            const auto ra = row_at_in[{std::get<0>(src), std::get<1>(src)}];
            if (ra.first != m) continue;
            const OperandRef& ref = std::get<2>(src);
            const int ka = bl0.dim[std::get<0>(src)];
            GemmTerm t{};
            t.a_base = ref.base;
            t.a_off = ref.off;
            t.lda = ka;
            t.b_base = BASE_T;
            t.b_off = to + (int64_t)S.row_off[ra.second] * Sp.ncols;
            t.ldb = Sp.ncols;
            t.k = ka;
            t.alpha = ref.alpha;
            per[chunk_of[w1]].push_back(t);
            per_w1[chunk_of[w1]].push_back(w1);
            flops2 += 2.0 * gm * (double)gn * ka;
          }
        }
        emit_block(emits, per, per_w1, (int)ix, Sp.off + (int64_t)Sp.row_off[ix] * Sp.ncols, Sp.ncols, gm, gn);
      }
    }
    // Emission order of the sector's groups.  Output-major (0): block by block, each block's
    // parts in channel order.  Channel-major (1): by the first channel of each part, so that
    // the parts of different output blocks that read the same intermediate columns are
    // neighbours in the tile list (and in one XCD's L2).
    if (pp.p2_order == 1)
      std::stable_sort(emits.begin(), emits.end(), [](const Emit& a, const Emit& b) {
        if (a.chunk != b.chunk) return a.chunk < b.chunk;
        return a.first_w1 != b.first_w1 ? a.first_w1 < b.first_w1 : a.jx < b.jx;
      });
    for (Emit& em : emits) {
      GemmBuilder& B2 = p2[em.chunk];
      B2.group(em.c_base, em.c_off, em.ldc, em.m, em.n, false);
      for (const GemmTerm& t : em.terms) B2.terms.push_back(t);
      B2.groups.back().term_end = (int32_t)B2.terms.size();
    }
  }
  double flops1 = 0;
  for (const GemmBuilder& B1 : p1) flops1 += B1.flops;
  // reported as (enlarged left operator products, enlarged right operator products)
  env->plan.flops1 = right_first ? flops2 : flops1;
  env->plan.flops2 = right_first ? flops1 : flops2;
  env->plan.chunks.resize(nchunks);
  for (int c = 0; c < nchunks; ++c) {
    if (right_first) {
      // phase 1: A = X (row-major), B = Rt (stored n-major); phase 2: A = Lt, B = T (row-major)
      env->plan.chunks[c].phase1 = finalize(p1[c], false, true, st, pp.tile_overhead);
      env->plan.chunks[c].phase2 = finalize(p2[c], false, false, st, pp.tile_overhead, pp.p2_order == 0);
    } else {
      env->plan.chunks[c].phase1 = finalize(p1[c], pp.t_colmajor != 0, pp.t_colmajor != 0, st, pp.tile_overhead);
      env->plan.chunks[c].phase2 = finalize(p2[c], pp.t_colmajor != 0, true, st, pp.tile_overhead, pp.p2_order == 0);
    }
  }
  {
    std::vector<ReduceTile> rtl;
    for (size_t g = 0; g < red.size(); ++g) {
      const int64_t mn = (int64_t)red[g].m * red[g].n;
      for (int64_t c = 0; c * kReduceChunk < mn; ++c) rtl.push_back(ReduceTile{(int32_t)g, (int32_t)c});
    }
    upload(env->plan.reduce_groups, red, st);
    upload(env->plan.reduce_tiles, rtl, st);
    env->plan.n_reduce_tiles = (int)rtl.size();
    env->work_elems = work;
    env->work.alloc(sizeof(double) * std::max<int64_t>(work, 1));
  }
  check_hip(hipStreamSynchronize(st), "plan");
}

namespace {

// Middle-bond sectors of a two-site block (rows (a, s1) over bond bl, columns (s2, b) over bond
// br), their vector layout and the row / column lookup (a, s1) -> (sector, row index),
// (s2, b) -> (sector, col index).  Returns the vector length.
int64_t middle_sectors(const Bond& bl, const Bond& br, std::vector<MiddleSector>& sectors, std::map<QN, int>& sec_index,
                       std::vector<lcc_block_entry>& layout,
                       std::map<std::pair<int, int>, std::pair<int, int>>& row_at,
                       std::map<std::pair<int, int>, std::pair<int, int>>& col_at, bool one_site) {
  std::map<QN, MiddleSector> secs;
  for (size_t a = 0; a < bl.q.size(); ++a)
    for (int s1 = 0; s1 < 4; ++s1) secs[bl.q[a] + local_qn(s1)].rows.push_back({(int)a, s1});
  // one site: the columns are the right bond alone (one trivial local state, s2 = 0, no charge)
  for (int s2 = 0; s2 < (one_site ? 1 : 4); ++s2)
    for (size_t b = 0; b < br.q.size(); ++b) {
      auto it = secs.find(br.q[b] - local_qn(s2));
      if (it != secs.end()) it->second.cols.push_back({s2, (int)b});
    }
  int64_t total = 0;
  for (auto& kv : secs) {
    MiddleSector& m = kv.second;
    if (m.rows.empty() || m.cols.empty()) continue;
    m.q = kv.first;
    for (auto& r : m.rows) { m.row_off.push_back(m.nrows); m.nrows += bl.dim[r.first]; }
    for (auto& c : m.cols) { m.col_off.push_back(m.ncols); m.ncols += br.dim[c.second]; }
    m.off = total;
    total += (int64_t)m.nrows * m.ncols;
    sec_index[m.q] = (int)sectors.size();
    sectors.push_back(m);
  }
  for (const MiddleSector& m : sectors)
    for (size_t i = 0; i < m.rows.size(); ++i)
      for (size_t jx = 0; jx < m.cols.size(); ++jx) {
        lcc_block_entry e;
        e.left = m.rows[i].first;
        e.s1 = m.rows[i].second;
        e.s2 = m.cols[jx].first;
        e.right = m.cols[jx].second;
        e.offset = m.off + (int64_t)m.row_off[i] * m.ncols + m.col_off[jx];
        e.ld = m.ncols;
        e.rows = bl.dim[e.left];
        e.cols = br.dim[e.right];
        layout.push_back(e);
      }
  for (size_t m = 0; m < sectors.size(); ++m) {
    for (size_t i = 0; i < sectors[m].rows.size(); ++i) row_at[sectors[m].rows[i]] = {(int)m, (int)i};
    for (size_t i = 0; i < sectors[m].cols.size(); ++i) col_at[sectors[m].cols[i]] = {(int)m, (int)i};
  }
  return total;
}

}  // namespace

Env* make_env(Context* ctx, const Mpo& mpo, int site, const Bond& bond_l, const Bond& bond_r,
              const Environment& L, const Environment& R) {
  return make_env(ctx, mpo, site, bond_l, bond_r, bond_l, bond_r, L, R, false);
}

Env* make_env(Context* ctx, const Mpo& mpo, int site, const Bond& bond_l, const Bond& bond_r, const Bond& ket_l,
              const Bond& ket_r, const Environment& L, const Environment& R, bool transition, bool one_site) {
  hipStream_t st = ctx->stream;
  const int K = mpo.K;
  std::unique_ptr<Env> env(new Env());
  env->ctx = ctx;
  env->site = site;
  env->K = K;
  env->bl = bond_l;
  env->br = bond_r;
  env->bl_in = ket_l;
  env->br_in = ket_r;
  env->transition = transition;
  env->one_site = one_site;
  const int mid = site + 1;  // MPO bond between the two sites (one site: between the site and R)
  env->D_mid = (int)mpo.dq[mid].size();

  // ---- middle-bond sectors and the vector layouts (output: bra; input: ket)
  auto& row_at = env->in.row_at;
  auto& col_at = env->in.col_at;
  auto& row_at_in = env->in.row_at_in;
  auto& col_at_in = env->in.col_at_in;
  env->n_elements =
      middle_sectors(env->bl, env->br, env->sectors, env->in.sec_index, env->layout, row_at, col_at, one_site);
  env->n_in = middle_sectors(env->bl_in, env->br_in, env->sectors_in, env->in.sec_index_in, env->layout_in, row_at_in,
                             col_at_in, one_site);

  // ---- environment data on the device: [L | R]
  env->env_elems = L.size + R.size;
  env->env64.alloc(sizeof(double) * std::max<int64_t>(env->env_elems, 1));
  check_hip(hipMemcpyAsync(env->env64.p, L.data.p, sizeof(double) * L.size, hipMemcpyDeviceToDevice, st), "env copy");
  check_hip(hipMemcpyAsync(env->env64.as<double>() + L.size, R.data.p, sizeof(double) * R.size, hipMemcpyDeviceToDevice, st),
            "env copy");
  const int64_t r_base = L.size;

  // ---- enlarged operators.  A reference is (base, offset, coefficient).
  // Lt: key (w1, row (a',s1'), src row (a,s1)) -> contributions (L block, coef)
  std::map<std::tuple<int, int, int, int, int>, std::vector<std::pair<int, double>>> lt_terms;
  std::vector<std::vector<int>> L_by_w(mpo.dq[site].size());
  for (size_t i = 0; i < L.blocks.size(); ++i) L_by_w[L.blocks[i].w].push_back((int)i);
  for (const MpoEntry& e : mpo.W[site])
    for (int bi : L_by_w[e.win]) {
      const EnvBlock& lb = L.blocks[bi];
      for (int sp = 0; sp < 4; ++sp)
        for (int s = 0; s < 4; ++s) {
          const double c = e.m[sp * 4 + s];
          if (c == 0.0) continue;
          if (!row_at.count({lb.r, sp}) || !row_at_in.count({lb.c, s})) continue;
          lt_terms[std::make_tuple(e.wout, lb.r, sp, lb.c, s)].push_back({bi, c});
        }
    }
  std::map<std::tuple<int, int, int, int, int>, std::vector<std::pair<int, double>>> rt_terms;
  if (one_site) {  // Rt^{w1} = R^{w1}: the right environment itself, on the trivial local state
    for (size_t bi = 0; bi < R.blocks.size(); ++bi) {
      const EnvBlock& rb = R.blocks[bi];
      if (!col_at.count({0, rb.r}) || !col_at_in.count({0, rb.c})) continue;
      rt_terms[std::make_tuple(rb.w, 0, rb.r, 0, rb.c)].push_back({(int)bi, 1.0});
    }
  } else {
    std::vector<std::vector<int>> R_by_w(mpo.dq[site + 2].size());
    for (size_t i = 0; i < R.blocks.size(); ++i) R_by_w[R.blocks[i].w].push_back((int)i);
    for (const MpoEntry& e : mpo.W[site + 1])
      for (int bi : R_by_w[e.wout]) {
        const EnvBlock& rb = R.blocks[bi];
        for (int sp = 0; sp < 4; ++sp)
          for (int s = 0; s < 4; ++s) {
            const double c = e.m[sp * 4 + s];
            if (c == 0.0) continue;
            if (!col_at.count({sp, rb.r}) || !col_at_in.count({s, rb.c})) continue;
            rt_terms[std::make_tuple(e.win, sp, rb.r, s, rb.c)].push_back({bi, c});
          }
      }
  }
  // references, merging multi-term entries
  MixBuilder merge;
  int64_t merged = 0;
  // Lt index: (w1, a', s1') -> list of (a, s1, ref)
  auto& lt = env->in.lt;
  for (const auto& kv : lt_terms) {
    int w1, ap, sp, a, s;
    std::tie(w1, ap, sp, a, s) = kv.first;
    OperandRef ref;
    if (kv.second.size() == 1) {
      ref = OperandRef{BASE_ENV, L.blocks[kv.second[0].first].off, kv.second[0].second};
    } else {
      const EnvBlock& b0 = L.blocks[kv.second[0].first];
      merge.group(BASE_MERGED, merged, b0.rows * b0.cols, BASE_ENV);
      for (const auto& c : kv.second) merge.term(L.blocks[c.first].off, c.second);
      ref = OperandRef{BASE_MERGED, merged, 1.0};
      merged += (int64_t)b0.rows * b0.cols;
    }
    lt[std::make_tuple(w1, ap, sp)].push_back(std::make_tuple(a, s, ref));
  }
  auto& rt = env->in.rt;  // (w1, s2', b') -> (s2, b, ref)
  for (const auto& kv : rt_terms) {
    int w1, sp, bp, s, b;
    std::tie(w1, sp, bp, s, b) = kv.first;
    OperandRef ref;
    if (kv.second.size() == 1) {
      ref = OperandRef{BASE_ENV, r_base + R.blocks[kv.second[0].first].off, kv.second[0].second};
    } else {
      const EnvBlock& b0 = R.blocks[kv.second[0].first];
      merge.group(BASE_MERGED, merged, b0.rows * b0.cols, BASE_ENV);
      for (const auto& c : kv.second) merge.term(r_base + R.blocks[c.first].off, c.second);
      ref = OperandRef{BASE_MERGED, merged, 1.0};
      merged += (int64_t)b0.rows * b0.cols;
    }
    rt[std::make_tuple(w1, sp, bp)].push_back(std::make_tuple(s, b, ref));
  }
  env->merged_elems = merged;
  env->merged64.alloc(sizeof(double) * std::max<int64_t>(merged, 1));
  {
    Bases<double> b{};
    b.p[BASE_ENV] = env->env64.as<double>();
    b.p[BASE_MERGED] = env->merged64.as<double>();
    run_mix(merge, b, st);
  }

  env->in.dq_mid = mpo.dq[mid];
  plan_env(*env, ctx->plan_params);
  if (!transition) {
    // CG workspace (FP64)
    for (auto& w : env->w64) w.alloc(sizeof(double) * std::max<int64_t>(env->n_elements, 1));
    env->flag.alloc(sizeof(int) * 4);
    apply_tuned(*env);
  }
  check_hip(hipStreamSynchronize(st), "build_env");
  return env.release();
}

void ensure_fp32(Env& env) {
  if (env.have32) return;
  hipStream_t st = env.ctx->stream;
  env.env32.alloc(sizeof(float) * std::max<int64_t>(env.env_elems, 1));
  env.merged32.alloc(sizeof(float) * std::max<int64_t>(env.merged_elems, 1));
  check_hip(launch_convert_f64_f32(env.env_elems, env.env64.as<double>(), env.env32.as<float>(), st), "convert env");
  if (env.merged_elems)
    check_hip(launch_convert_f64_f32(env.merged_elems, env.merged64.as<double>(), env.merged32.as<float>(), st), "convert merged");
  for (auto& w : env.w32) w.alloc(sizeof(float) * std::max<int64_t>(env.n_elements, 1));
  check_hip(hipStreamSynchronize(st), "ensure_fp32");
  env.have32 = true;
}

// diag(H_eff)[(a,s1,i),(s2,b,j)] = sum_{w1} Lt^{w1}[(a,s1,i),(a,s1,i)] Rt^{w1}[(s2,b,j),(s2,b,j)] over the
// middle channels that keep the sector (dq = 0): per sector q the diagonals of the enlarged
// operators' diagonal blocks are gathered into DL_q (channels x rows) and DR_q (channels x
// columns), and D_q = DL_q^T DR_q is one GEMM.
void compute_diagonal(Env& E) {
  if (E.have_diag) return;
  if (E.transition) throw Error{LCC_ERR_STATE, "a transition environment has no diagonal"};
  hipStream_t st = E.ctx->stream;
  const int nsec = (int)E.sectors.size();
  struct Ref { int w1, m, off, dim; OperandRef ref; };
  std::vector<Ref> lrefs, rrefs;
  std::set<std::pair<int, int>> lhas, rhas;  // (sector, w1)
  for (const auto& kv : E.in.lt) {
    int w1, ap, sp;
    std::tie(w1, ap, sp) = kv.first;
    if (E.in.dq_mid[w1] != QN(0, 0)) continue;
    for (const auto& src : kv.second) {
      if (std::get<0>(src) != ap || std::get<1>(src) != sp) continue;
      const auto ra = E.in.row_at.at({ap, sp});
      lrefs.push_back(Ref{w1, ra.first, E.sectors[ra.first].row_off[ra.second], E.bl.dim[ap], std::get<2>(src)});
      lhas.insert({ra.first, w1});
    }
  }
  for (const auto& kv : E.in.rt) {
    int w1, s2p, bp;
    std::tie(w1, s2p, bp) = kv.first;
    if (E.in.dq_mid[w1] != QN(0, 0)) continue;
    for (const auto& src : kv.second) {
      if (std::get<0>(src) != s2p || std::get<1>(src) != bp) continue;
      const auto ca = E.in.col_at.at({s2p, bp});
      rrefs.push_back(Ref{w1, ca.first, E.sectors[ca.first].col_off[ca.second], E.br.dim[bp], std::get<2>(src)});
      rhas.insert({ca.first, w1});
    }
  }
  std::vector<std::map<int, int>> chan(nsec);  // sector -> w1 -> row of DL / DR
  std::vector<int64_t> dl_off(nsec, 0), dr_off(nsec, 0);
  int64_t dl_total = 0, dr_total = 0;
  for (const auto& mw : lhas)
    if (rhas.count(mw)) chan[mw.first].emplace(mw.second, (int)chan[mw.first].size());
  for (int m = 0; m < nsec; ++m) {
    dl_off[m] = dl_total;
    dr_off[m] = dr_total;
    dl_total += (int64_t)chan[m].size() * E.sectors[m].nrows;
    dr_total += (int64_t)chan[m].size() * E.sectors[m].ncols;
  }
  std::vector<DiagItem> items;
  auto add = [&](const Ref& r, int64_t base_off, int width, double* /*unused*/) {
    DiagItem it{};
    it.src_off = r.ref.off;
    it.dst_off = base_off + (int64_t)chan[r.m].at(r.w1) * width + r.off;
    it.alpha = r.ref.alpha;
    it.ld = r.dim;
    it.count = r.dim;
    it.src_base = r.ref.base;
    items.push_back(it);
  };
  for (const Ref& r : lrefs)
    if (chan[r.m].count(r.w1)) add(r, dl_off[r.m], E.sectors[r.m].nrows, nullptr);
  const size_t n_left = items.size();
  for (const Ref& r : rrefs)
    if (chan[r.m].count(r.w1)) add(r, dr_off[r.m], E.sectors[r.m].ncols, nullptr);
  DevBuf dl, dr, dli, dri;
  dl.alloc(sizeof(double) * std::max<int64_t>(dl_total, 1));
  dr.alloc(sizeof(double) * std::max<int64_t>(dr_total, 1));
  check_hip(launch_fill_f64(dl.as<double>(), std::max<int64_t>(dl_total, 1), 0.0, st), "zero DL");
  check_hip(launch_fill_f64(dr.as<double>(), std::max<int64_t>(dr_total, 1), 0.0, st), "zero DR");
  std::vector<DiagItem> li(items.begin(), items.begin() + n_left), ri(items.begin() + n_left, items.end());
  upload(dli, li, st);
  upload(dri, ri, st);
  Bases<double> b{};
  b.p[BASE_ENV] = E.env64.as<double>();
  b.p[BASE_MERGED] = E.merged64.as<double>();
  check_hip(launch_diag_gather(dli.as<DiagItem>(), (int)li.size(), b, dl.as<double>(), st), "diag gather");
  check_hip(launch_diag_gather(dri.as<DiagItem>(), (int)ri.size(), b, dr.as<double>(), st), "diag gather");
  // D_q = DL_q^T DR_q: A stored k-major (channel c, row r at c * nrows + r), B row-major
  GemmBuilder g;
  for (int m = 0; m < nsec; ++m) {
    const MiddleSector& S = E.sectors[m];
    g.group(BASE_Y, S.off, S.ncols, S.nrows, S.ncols, false);
    if (!chan[m].empty()) g.term(BASE_T, dl_off[m], S.nrows, BASE_WORK, dr_off[m], S.ncols, (int)chan[m].size(), 1.0);
  }
  E.diag64.alloc(sizeof(double) * std::max<int64_t>(E.n_elements, 1));
  Bases<double> gb{};
  gb.p[BASE_T] = dl.as<double>();
  gb.p[BASE_WORK] = dr.as<double>();
  gb.p[BASE_Y] = E.diag64.as<double>();
  run_gemm64(finalize(g, true, false, st), gb, st);
  check_hip(hipStreamSynchronize(st), "diagonal");
  E.have_diag = true;
}

namespace {
void no_callback(void*, const LaunchRef&) {}
}  // namespace

namespace {

void bases_of(Env& env, int precision, const void* x, void* y, Bases<double>& b64, Bases<float>& b32) {
  b64 = Bases<double>{};
  b32 = Bases<float>{};
  if (precision == LCC_FP64) {
    b64.p[BASE_ENV] = env.env64.as<double>();
    b64.p[BASE_MERGED] = env.merged64.as<double>();
    b64.p[BASE_X] = const_cast<double*>(static_cast<const double*>(x));
    b64.p[BASE_T] = env.tbuf.as<double>();
    b64.p[BASE_Y] = static_cast<double*>(y);
    b64.p[BASE_WORK] = env.work.as<double>();
  } else {
    b32.p[BASE_ENV] = env.env32.as<float>();
    b32.p[BASE_MERGED] = env.merged32.as<float>();
    b32.p[BASE_X] = const_cast<float*>(static_cast<const float*>(x));
    b32.p[BASE_T] = env.tbuf.as<float>();
    b32.p[BASE_Y] = static_cast<float*>(y);
    b32.p[BASE_WORK] = env.work.as<float>();
  }
}

void launch_one(const GemmLaunch& L, int precision, const Bases<double>& b64, const Bases<float>& b32,
                hipStream_t st, const int* active = nullptr) {
  hipError_t e;
  if (precision == LCC_FP64)
    e = launch_gemm_f64(L.desc(LCC_FP64), b64, st, nullptr, active);
  else if (precision == LCC_FP32)
    e = launch_gemm_f32(L.desc(LCC_FP32), b32, st, nullptr, active);
  else
    e = launch_gemm_bf16x3(L.desc(LCC_BF16X3), b32, st, nullptr, active);
  check_hip(e, "gemm launch");
}

void launch_reduce(const Plan& P, int precision, const Bases<double>& b64, const Bases<float>& b32, hipStream_t st,
                   const int* active = nullptr) {
  hipError_t e = precision == LCC_FP64
                     ? launch_reduce_f64(P.reduce_groups.as<ReduceGroup>(), P.reduce_tiles.as<ReduceTile>(),
                                         P.n_reduce_tiles, b64, st, nullptr, active)
                     : launch_reduce_f32(P.reduce_groups.as<ReduceGroup>(), P.reduce_tiles.as<ReduceTile>(),
                                         P.n_reduce_tiles, b32, st, nullptr, active);
  check_hip(e, "reduce launch");
}

// Side streams of a context (default priority), created on first use.
void ensure_side_streams(Context& C) {
  if ((int)C.side.size() >= C.overlap) return;
  if (!C.ev_fork) check_hip(hipEventCreateWithFlags(&C.ev_fork, hipEventDisableTiming), "event");
  while ((int)C.side.size() < C.overlap) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    check_hip(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "side stream");
    C.side.push_back(s);
    check_hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
    C.ev_join.push_back(e);
  }
}

}  // namespace

// H_eff x.  The launches of one phase (one per tile shape) are independent: with side streams
// enabled on the context they run concurrently (the longest on the context stream, the others
// spread over the side streams), so that short launches fill the tail of long ones; the
// phases, chunks and the reduction stay ordered on the context stream.  With `active` given
// (a device word), every workgroup returns at once while it reads 0.
void apply_heff(Env& env, int precision, const void* x, void* y, const int* active) {
  Context& C = *env.ctx;
  if (C.overlap <= 0 && !active) {
    apply_heff_each(env, precision, x, y, no_callback, nullptr);
    return;
  }
  hipStream_t st = C.stream;
  const Plan& P = env.plan;
  if (precision != LCC_FP64) ensure_fp32(env);
  ensure_side_streams(C);
  Bases<double> b64;
  Bases<float> b32;
  bases_of(env, precision, x, y, b64, b32);
  for (const Plan::Chunk& Ch : P.chunks)
    for (int ph = 1; ph <= 2; ++ph) {
      const std::vector<GemmLaunch>& Ls = ph == 1 ? Ch.phase1 : Ch.phase2;
      if (Ls.size() <= 1 || C.overlap <= 0) {
        for (const GemmLaunch& L : Ls) launch_one(L, precision, b64, b32, st, active);
        continue;
      }
      std::vector<int> order(Ls.size());
      for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return Ls[a].flops > Ls[b].flops; });
      const int nside = std::min<int>(C.overlap, (int)Ls.size() - 1);
      check_hip(hipEventRecord(C.ev_fork, st), "fork");
      for (int k = 0; k < nside; ++k) check_hip(hipStreamWaitEvent(C.side[k], C.ev_fork, 0), "fork wait");
      for (size_t i = 0; i < order.size(); ++i)
        launch_one(Ls[order[i]], precision, b64, b32, i == 0 ? st : C.side[(i - 1) % nside], active);
      for (int k = 0; k < nside; ++k) {
        check_hip(hipEventRecord(C.ev_join[k], C.side[k]), "join");
        check_hip(hipStreamWaitEvent(st, C.ev_join[k], 0), "join wait");
      }
    }
  launch_reduce(P, precision, b64, b32, st, active);
}

// Every launch of one H_eff x in order on the context stream: for each channel chunk its
// phase-1 launches (one per tile shape) then its phase-2 launches, and finally the split-K
// reduction into y (the order the per-launch profile and the batched graph use).
void apply_heff_each(Env& env, int precision, const void* x, void* y,
                     void (*after_each)(void*, const LaunchRef&), void* user) {
  hipStream_t st = env.ctx->stream;
  const Plan& P = env.plan;
  if (precision != LCC_FP64) ensure_fp32(env);
  Bases<double> b64;
  Bases<float> b32;
  bases_of(env, precision, x, y, b64, b32);
  for (const Plan::Chunk& C : P.chunks)
    for (int ph = 1; ph <= 2; ++ph)
      for (const GemmLaunch& L : ph == 1 ? C.phase1 : C.phase2) {
        launch_one(L, precision, b64, b32, st);
        after_each(user, LaunchRef{ph, 0, &L});
      }
  launch_reduce(P, precision, b64, b32, st);
  after_each(user, LaunchRef{2, 1, nullptr});
}

}  // namespace lcc
