// gfx950 kernels: grouped block GEMM on MFMA (FP64, FP32, BF16x3), block mixing, and the
// FP64-accumulating vector operations of conjugate gradients.
//
// The grouped GEMM computes, for every output block ("group") g,
//     C_g  (=|+=)  sum_{t in terms(g)} alpha_t * op(A_t) * op(B_t)
// with uneven m, n, k.  A workgroup owns one BM x BN output tile of one group and walks the
// group's whole term list, so every output element is produced by exactly one workgroup in
// a fixed order: results are deterministic and no atomics are used.  The per-term alpha is
// applied while A is staged into LDS: this is where the MPO coefficients of the two sites
// (the W-mixing of the effective Hamiltonian) enter without an extra pass over memory.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace lcc {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Operand and output pointers live in a by-value struct (Bases); read through them as is, they
// are generic (flat) pointers, whose loads also count against the LDS wait counter and so hold
// up the LDS reads that follow a prefetch.  The kernels address device memory through these
// global-address-space views instead.
template <class T>
using gptr = const __attribute__((address_space(1))) T*;
template <class T>
using gmut = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> global_view(const T* p) { return (gptr<T>)p; }
template <class T>
__device__ __forceinline__ gmut<T> global_mut(T* p) { return (gmut<T>)p; }

constexpr int kThreads = 256;

// Workgroups are dispatched round-robin over the 8 XCDs.  Tiles are handed out in runs of
// kTileRun consecutive tiles per XCD (run r goes to XCD r mod 8): consecutive tiles belong to
// the same output block and share operand panels, which then meet in one XCD's L2, while the
// interleaving of runs keeps the work of every XCD a uniform sample of the launch (a
// contiguous slice per XCD leaves XCDs idle when block sizes vary along the tile list).  The
// tail of the grid that does not fill whole rounds keeps the plain order.
constexpr int kTileRun = 16;
__device__ __forceinline__ int xcd_remap(int bid, int n) {
  const int full = n / (8 * kTileRun) * (8 * kTileRun);
  if (bid >= full) return bid;
  const int xcd = bid & 7, local = bid >> 3;
  return ((local / kTileRun) * 8 + xcd) * kTileRun + (local % kTileRun);
}

// Number of a wave's 16-row (or 16-column) sub-tiles, starting at `first`, that intersect a
// block of `extent` rows (columns); at most T16.  Wave-uniform: the sub-tiles of an edge tile
// that lie wholly outside the block issue no MFMA and read no LDS.
template <int T16>
__device__ __forceinline__ int live_subtiles(int first, int extent) {
  const int n = (extent - first + 15) >> 4;
  return __builtin_amdgcn_readfirstlane(n < 0 ? 0 : (n > T16 ? T16 : n));
}

template <int MODE>
struct Mfma;
template <>
struct Mfma<0> {
  typedef double T;
  typedef d4 Acc;
  static __device__ __forceinline__ Acc step(T a, T b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<1> {
  typedef float T;
  typedef f4 Acc;
  static __device__ __forceinline__ Acc step(T a, T b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
// MODE 2: FP32 operands staged as for MODE 1, split into bf16 hi + lo as they are read from LDS
// and multiplied on v_mfma_f32_16x16x32_bf16 (hi*hi + hi*lo + lo*hi, FP32 accumulation);
// accumulator layout as MODE 1.
template <>
struct Mfma<2> {
  typedef float T;
  typedef f4 Acc;
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// ------------------------------------------------------------------------------------------
// Packed-k operand staging.  A workgroup consumes its group's k-quads (SlotRec, four
// consecutive k of one term) in chunks of BK/4 quads, so that terms with short k share a
// chunk.  Before a chunk is loaded, BK/4 threads resolve its quads (pointers, leading
// dimensions, valid count, alpha) into LDS, where every thread finds the quads of the elements
// it stages.  An operand stored k-contiguous (KC: element (r, k) at p[r*ld + k]) is staged by
// quads along k, otherwise (p[k*ld + r]) by quads along r; either way one 16-byte global load
// (two for double) per full quad, element-aligned.  Elements outside the matrix or past a
// quad's valid count are zeros.
// ------------------------------------------------------------------------------------------
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));

template <class T>
struct QuadRef {
  const T* a;
  const T* b;
  int lda, ldb, kv;
  T alpha;
};

// A pointer that is the same in every lane, moved to scalar registers.
template <class T>
__device__ __forceinline__ T* uniform(T* p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (T*)(((unsigned long long)hi << 32) | lo);
}

// The launch's operand base pointers (or, in a batched launch, the problem's row of the
// table), staged in LDS: a term's base is then one LDS read with its base index, where
// indexing the by-value argument struct would copy it to private memory.
template <class T>
struct BaseTable {
  T* p[NUM_BASES];
  // threads < NUM_BASES write; the caller synchronises before use
  __device__ __forceinline__ void stage(const Bases<T>& bs, const Bases<T>* row) {
    const int tid = threadIdx.x;
    if (tid < NUM_BASES) {
      T* v = bs.p[0];
#pragma unroll
      for (int j = 1; j < NUM_BASES; ++j)
        if (tid == j) v = bs.p[j];
      if (row) v = row->p[tid];
      p[tid] = v;
    }
  }
  // base i, for an index that is the same in every lane
  __device__ __forceinline__ T* get(int i) const { return uniform(p[i]); }
};

template <class T>
__device__ __forceinline__ void resolve_quad(QuadRef<T>& Q, const SlotRec& s, bool valid, const BaseTable<T>& bt) {
  if (valid) {
    Q.a = bt.p[s.a_base] + s.a_off;
    Q.b = bt.p[s.b_base] + s.b_off;
    Q.lda = s.lda;
    Q.ldb = s.ldb;
    Q.kv = s.kv;
    Q.alpha = (T)s.alpha;
  } else {
    Q.a = nullptr;
    Q.b = nullptr;
    Q.lda = Q.ldb = Q.kv = 0;
    Q.alpha = (T)0;
  }
}

__device__ __forceinline__ void load_quad(float* v, gptr<float> p) {
  const f4u w = *(const __attribute__((address_space(1))) f4u*)p;
  v[0] = w[0]; v[1] = w[1]; v[2] = w[2]; v[3] = w[3];
}
__device__ __forceinline__ void load_quad(double* v, gptr<double> p) {
  const d2u w0 = *(const __attribute__((address_space(1))) d2u*)p;
  const d2u w1 = *(const __attribute__((address_space(1))) d2u*)(p + 2);
  v[0] = w0[0]; v[1] = w0[1]; v[2] = w1[0]; v[3] = w1[1];
}
// 16-byte-aligned LDS quads (two 16-byte accesses for double).
__device__ __forceinline__ f4 lds_read_quad(const float* p) { return *reinterpret_cast<const f4*>(p); }
__device__ __forceinline__ d4 lds_read_quad(const double* p) {
  const d2 w0 = *reinterpret_cast<const d2*>(p);
  const d2 w1 = *reinterpret_cast<const d2*>(p + 2);
  return d4{w0[0], w0[1], w1[0], w1[1]};
}
__device__ __forceinline__ void lds_write_quad(float* p, float a, float b, float c, float d) {
  *reinterpret_cast<f4*>(p) = f4{a, b, c, d};
}
__device__ __forceinline__ void lds_write_quad(double* p, double a, double b, double c, double d) {
  *reinterpret_cast<d2*>(p) = d2{a, b};
  *reinterpret_cast<d2*>(p + 2) = d2{c, d};
}

// OP 0: operand A (rows = output rows, scaled by the quad's alpha); OP 1: operand B.
template <class T, bool KC, int R, int BK, int OP, int NT>
struct Stager {
  static constexpr int QUADS = R * BK / 4;
  static constexpr int NQ = (QUADS + NT - 1) / NT;
  static constexpr int SPC = BK / 4;
  static constexpr int PAD = 16 / (int)sizeof(T);
  // LDS tile of the FP64/FP32 kernel mirrors the stored layout: [R][BK] if KC, else [BK][R]
  static constexpr int D0 = KC ? R : BK;
  static constexpr int D1 = KC ? BK + PAD : R + PAD;
  T v[NQ][4];
  T scale[NQ];

  static __device__ __forceinline__ bool live(int q) { return QUADS % NT == 0 || q < QUADS; }
  // quad q -> (first row r, packed k kk): KC quads run along k, the others along r
  static __device__ __forceinline__ void coords(int q, int& r, int& kk) {
    if (KC) {
      r = q / SPC;
      kk = 4 * (q % SPC);
    } else {
      kk = q / (R / 4);
      r = 4 * (q % (R / 4));
    }
  }
  __device__ __forceinline__ void load(const QuadRef<T>* refs, int r0, int rmax) {
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
#pragma unroll
      for (int j = 0; j < 4; ++j) v[i][j] = (T)0;
      scale[i] = (T)1;
      const int q = threadIdx.x + i * NT;
      if (!live(q)) continue;
      int r, kk;
      coords(q, r, kk);
      const QuadRef<T>& Q = refs[kk >> 2];
      if (OP == 0) scale[i] = Q.alpha;
      const T* P = OP == 0 ? Q.a : Q.b;
      const int ld = OP == 0 ? Q.lda : Q.ldb;
      const int gr = r0 + r;
      if (KC) {
        if (gr >= rmax || Q.kv == 0) continue;
        const gptr<T> p = global_view(P) + (int64_t)gr * ld;
        if (Q.kv == 4) {
          load_quad(v[i], p);
        } else {
#pragma unroll
          for (int j = 0; j < 3; ++j)
            if (j < Q.kv) v[i][j] = p[j];
        }
      } else {
        const int jj = kk & 3;
        if (jj >= Q.kv) continue;
        const gptr<T> p = global_view(P) + (int64_t)jj * ld + gr;
        if (gr + 3 < rmax) {
          load_quad(v[i], p);
        } else {
#pragma unroll
          for (int j = 0; j < 3; ++j)
            if (gr + j < rmax) v[i][j] = p[j];
        }
      }
    }
  }
  // FP64 / FP32 kernel: into the mirrored LDS tile
  __device__ __forceinline__ void store(T (*S)[D1]) const {
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int q = threadIdx.x + i * NT;
      if (!live(q)) continue;
      int r, kk;
      coords(q, r, kk);
      const T s = scale[i];
      lds_write_quad(KC ? &S[r][kk] : &S[kk][r], v[i][0] * s, v[i][1] * s, v[i][2] * s, v[i][3] * s);
    }
  }
  // BF16x3 kernel: into k-contiguous hi / lo tiles [R][KP]
  template <int KP>
  __device__ __forceinline__ void store_split(__bf16 (*H)[KP], __bf16 (*L)[KP]) const {
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int q = threadIdx.x + i * NT;
      if (!live(q)) continue;
      int r, kk;
      coords(q, r, kk);
      bf4 h, l;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float x = (float)(v[i][j] * scale[i]);
        h[j] = (__bf16)x;
        l[j] = (__bf16)(x - (float)h[j]);
      }
      if (KC) {
        *reinterpret_cast<bf4*>(&H[r][kk]) = h;
        *reinterpret_cast<bf4*>(&L[r][kk]) = l;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          H[r + j][kk] = h[j];
          L[r + j][kk] = l[j];
        }
      }
    }
  }
};

// The chunk walk of the kernels: resolve the quads of chunk 0, load it, prefetch the raw
// records of chunk 1; then for each chunk c: store the staged chunk c to LDS, resolve chunk
// c+1, load chunk c+1 into registers and prefetch the records of chunk c+2 while chunk c is
// multiplied.

// ------------------------------------------------------------------------------------------
// FP64 / FP32 MFMA 16x16x4 grouped GEMM.
//   MODE 0: double operands, v_mfma_f64_16x16x4_f64: lane l holds A[l%16][k(l/16)], B[k(l/16)][l%16],
//           accumulator element r at row l/16 + 4r, column l%16.
//   MODE 1: float operands, v_mfma_f32_16x16x4_f32: same inputs, accumulator element r at
//           row 4(l/16) + r, column l%16.
// The four MFMAs of a 16-wide k group take k(l/16) = 4(l/16) + s in step s (s = 0..3): the sum
// over k is the same for any assignment that A and B share, and with it a lane fetches the
// four k values of its row of a k-contiguous LDS tile with one 16-byte read (two for double);
// from an r-contiguous tile it reads them one by one.
// Waves are arranged WM x WN; each wave owns (BM/WM) x (BN/WN) = (16 TM) x (16 TN).
// ------------------------------------------------------------------------------------------
// MFMAs of one staged chunk of the packed-k kernel.  The wave's sub-tiles i >= ni or j >= nj
// lie outside the block and are skipped (their LDS reads stay: unconditional reads pair up).
// arow / bcol: the lane's row (column) in the LDS tile for sub-tile 0.
template <int MODE, bool TA, bool TB, int BK, int TM, int TN, class TA_, class TB_>
__device__ __forceinline__ void packed_chunk(const TA_& As, const TB_& Bs, int arow, int bcol, int kmax, int ni,
                                             int nj, typename Mfma<MODE>::Acc (&acc)[TM][TN]) {
  typedef typename Mfma<MODE>::T T;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int kg = 0; kg < BK; kg += 16) {
    if (kg < kmax) {
      const int kq = kg + 4 * (lane >> 4);
      T a[TM][4], b[TN][4];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int r = arow + i * 16;
        if (!TA) {
          const auto q = lds_read_quad(&As[r][kq]);
#pragma unroll
          for (int s = 0; s < 4; ++s) a[i][s] = q[s];
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s) a[i][s] = As[kq + s][r];
        }
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int cc = bcol + j * 16;
        if (TB) {
          const auto q = lds_read_quad(&Bs[cc][kq]);
#pragma unroll
          for (int s = 0; s < 4; ++s) b[j][s] = q[s];
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s) b[j][s] = Bs[kq + s][cc];
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            if (i < ni && j < nj) acc[i][j] = Mfma<MODE>::step(a[i][s], b[j][s], acc[i][j]);
    }
  }
}

template <int MODE, bool TA, bool TB, int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN)
gemm_packed_kernel(const SlotRec* __restrict__ slots, const GemmGroup* __restrict__ groups,
                 const GemmTile* __restrict__ tiles, int n_tiles,
                 Bases<typename Mfma<MODE>::T> bases, const Bases<typename Mfma<MODE>::T>* __restrict__ table,
                 const int* __restrict__ active) {
  typedef typename Mfma<MODE>::T T;
  typedef typename Mfma<MODE>::Acc Acc;
  constexpr int BK = 128 / (int)sizeof(T);  // one 128-byte line of a row per chunk
  constexpr int SPC = BK / 4;
  constexpr int TM = BM / WM / 16;
  constexpr int TN = BN / WN / 16;
  constexpr int NT = 64 * WM * WN;
  typedef Stager<T, !TA, BM, BK, 0, NT> SA;
  typedef Stager<T, TB, BN, BK, 1, NT> SB;
  __shared__ __attribute__((aligned(16))) T As[SA::D0][SA::D1];
  __shared__ __attribute__((aligned(16))) T Bs[SB::D0][SB::D1];
  __shared__ QuadRef<T> refs[SPC];

  __shared__ BaseTable<T> bt;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;

  const GemmTile tile = tiles[xcd_remap(blockIdx.x, n_tiles)];
  const GemmGroup g = groups[tile.group];
  // a problem whose active flag is 0 is skipped (batched: converged; single: halted solve)
  if (active && !active[table ? g.problem : 0]) return;
  const Bases<T>* row = table ? table + g.problem : nullptr;  // batched: per-problem operands
  bt.stage(bases, row);
  __syncthreads();
  const int tm = tile.tile / g.tiles_n, tn = tile.tile % g.tiles_n;
  const int row0 = tm * BM, col0 = tn * BN;
  const int arow = wm * (BM / WM) + (lane & 15), bcol = wn * (BN / WN) + (lane & 15);
  const int ni = live_subtiles<TM>(row0 + wm * (BM / WM), g.m);
  const int nj = live_subtiles<TN>(col0 + wn * (BN / WN), g.n);

  Acc acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

  SA sa;
  SB sb;
  const int nslots = g.slot_end - g.slot_begin;
  const int nch = (nslots + SPC - 1) / SPC;
  const SlotRec* __restrict__ gs = slots + g.slot_begin;
  SlotRec pending{};
  if (nch > 0) {
    if (tid < SPC) {
      const bool ok = tid < nslots;
      if (ok) pending = gs[tid];
      resolve_quad(refs[tid], pending, ok, bt);
    }
    __syncthreads();
    sa.load(refs, row0, g.m);
    sb.load(refs, col0, g.n);
    if (tid < SPC && SPC + tid < nslots) pending = gs[SPC + tid];
  }
  for (int c = 0; c < nch; ++c) {
    const int kmax = min(BK, 4 * (nslots - c * SPC));
    __syncthreads();
    sa.store(As);
    sb.store(Bs);
    if (tid < SPC) resolve_quad(refs[tid], pending, (c + 1) * SPC + tid < nslots, bt);
    __syncthreads();
    if (c + 1 < nch) {
      sa.load(refs, row0, g.m);
      sb.load(refs, col0, g.n);
      if (tid < SPC && (c + 2) * SPC + tid < nslots) pending = gs[(c + 2) * SPC + tid];
    }
    packed_chunk<MODE, TA, TB, BK, TM, TN>(As, Bs, arow, bcol, kmax, ni, nj, acc);
  }

  const gmut<T> C = global_mut(bt.get(g.c_base) + g.c_off);
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wm * (BM / WM) + i * 16 + Mfma<MODE>::row(lane, r);
        const int gc = col0 + wn * (BN / WN) + j * 16 + (lane & 15);
        if (gr < g.m && gc < g.n) {
          const gmut<T> p = C + (int64_t)gr * g.ldc + gc;
          *p = g.accumulate ? *p + acc[i][j][r] : acc[i][j][r];
        }
      }
}

// ------------------------------------------------------------------------------------------
// BF16x3 split-product GEMM on v_mfma_f32_16x16x32_bf16.  FP32 operands are split while
// staged: hi = bf16(x), lo = bf16(x - hi); the product is hi*hi + hi*lo + lo*hi with FP32
// accumulation (the lo*lo term is below the representation error of the split).
// Lane l holds A[l%16][8(l/16) + i], B[8(l/16) + i][l%16] (i = 0..7); accumulator element r
// at row 4(l/16) + r, column l%16.  LDS holds A as [m][k] and B as [n][k] so that each
// lane's eight k values are contiguous.
// ------------------------------------------------------------------------------------------
// Split-product MFMAs of one staged 32-k chunk (LDS hi / lo tiles [r][k]); arow, bcol as for
// packed_chunk.  Every sub-tile runs: skipping those outside the block (as the FP64 / FP32
// kernels do) raises the register count of these kernels past an occupancy step.
template <int TM, int TN, class TA_, class TB_>
__device__ __forceinline__ void bf16x3_chunk(const TA_& Ah, const TA_& Al, const TB_& Bh, const TB_& Bl, int arow,
                                             int bcol, f4 (&acc)[TM][TN]) {
  const int lane = threadIdx.x & 63;
  bf8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    ah[i] = *reinterpret_cast<const bf8*>(&Ah[arow + i * 16][8 * (lane >> 4)]);
    al[i] = *reinterpret_cast<const bf8*>(&Al[arow + i * 16][8 * (lane >> 4)]);
  }
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    bh[j] = *reinterpret_cast<const bf8*>(&Bh[bcol + j * 16][8 * (lane >> 4)]);
    bl[j] = *reinterpret_cast<const bf8*>(&Bl[bcol + j * 16][8 * (lane >> 4)]);
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
    }
}

// bf16x3_chunk with the sub-tiles outside the block (i >= ni, j >= nj) issuing no MFMA
template <int TM, int TN, class TA_, class TB_>
__device__ __forceinline__ void bf16x3_chunk_live(const TA_& Ah, const TA_& Al, const TB_& Bh, const TB_& Bl, int arow,
                                                  int bcol, int ni, int nj, f4 (&acc)[TM][TN]) {
  const int lane = threadIdx.x & 63;
  bf8 ah[TM], al[TM];
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    ah[i] = *reinterpret_cast<const bf8*>(&Ah[arow + i * 16][8 * (lane >> 4)]);
    al[i] = *reinterpret_cast<const bf8*>(&Al[arow + i * 16][8 * (lane >> 4)]);
  }
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    if (j < nj) {
      const bf8 bh = *reinterpret_cast<const bf8*>(&Bh[bcol + j * 16][8 * (lane >> 4)]);
      const bf8 bl = *reinterpret_cast<const bf8*>(&Bl[bcol + j * 16][8 * (lane >> 4)]);
#pragma unroll
      for (int i = 0; i < TM; ++i)
        if (i < ni) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, acc[i][j], 0, 0, 0);
        }
    }
  }
}

template <bool TA, bool TB, int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN)
gemm_bf16x3_packed_kernel(const SlotRec* __restrict__ slots, const GemmGroup* __restrict__ groups,
                   const GemmTile* __restrict__ tiles, int n_tiles, Bases<float> bases,
                   const Bases<float>* __restrict__ table, const int* __restrict__ active) {
  constexpr int BK = 32;
  constexpr int SPC = BK / 4;
  constexpr int KP = BK + 8;  // row pitch in bf16 elements (16-byte aligned rows)
  constexpr int TM = BM / WM / 16;
  constexpr int TN = BN / WN / 16;
  constexpr int NT = 64 * WM * WN;
  typedef Stager<float, !TA, BM, BK, 0, NT> SA;
  typedef Stager<float, TB, BN, BK, 1, NT> SB;
  __shared__ __attribute__((aligned(16))) __bf16 Ah[BM][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Al[BM][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[BN][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[BN][KP];
  __shared__ QuadRef<float> refs[SPC];

  __shared__ BaseTable<float> bt;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;

  const GemmTile tile = tiles[xcd_remap(blockIdx.x, n_tiles)];
  const GemmGroup g = groups[tile.group];
  // a problem whose active flag is 0 is skipped (batched: converged; single: halted solve)
  if (active && !active[table ? g.problem : 0]) return;
  const Bases<float>* row = table ? table + g.problem : nullptr;  // batched: per-problem operands
  bt.stage(bases, row);
  __syncthreads();
  const int tm = tile.tile / g.tiles_n, tn = tile.tile % g.tiles_n;
  const int row0 = tm * BM, col0 = tn * BN;
  const int arow = wm * (BM / WM) + (lane & 15), bcol = wn * (BN / WN) + (lane & 15);

  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  SA sa;
  SB sb;
  const int nslots = g.slot_end - g.slot_begin;
  const int nch = (nslots + SPC - 1) / SPC;
  const SlotRec* __restrict__ gs = slots + g.slot_begin;
  SlotRec pending{};
  if (nch > 0) {
    if (tid < SPC) {
      const bool ok = tid < nslots;
      if (ok) pending = gs[tid];
      resolve_quad(refs[tid], pending, ok, bt);
    }
    __syncthreads();
    sa.load(refs, row0, g.m);
    sb.load(refs, col0, g.n);
    if (tid < SPC && SPC + tid < nslots) pending = gs[SPC + tid];
  }
  for (int c = 0; c < nch; ++c) {
    const int kmax = min(BK, 4 * (nslots - c * SPC));
    __syncthreads();
    sa.template store_split<KP>(Ah, Al);
    sb.template store_split<KP>(Bh, Bl);
    if (tid < SPC) resolve_quad(refs[tid], pending, (c + 1) * SPC + tid < nslots, bt);
    __syncthreads();
    if (c + 1 < nch) {
      sa.load(refs, row0, g.m);
      sb.load(refs, col0, g.n);
      if (tid < SPC && (c + 2) * SPC + tid < nslots) pending = gs[(c + 2) * SPC + tid];
    }
    (void)kmax;
    bf16x3_chunk<TM, TN>(Ah, Al, Bh, Bl, arow, bcol, acc);
  }

  const gmut<float> C = global_mut(bt.get(g.c_base) + g.c_off);
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wm * (BM / WM) + i * 16 + 4 * (lane >> 4) + r;
        const int gc = col0 + wn * (BN / WN) + j * 16 + (lane & 15);
        if (gr < g.m && gc < g.n) {
          const gmut<float> p = C + (int64_t)gr * g.ldc + gc;
          *p = g.accumulate ? *p + acc[i][j][r] : acc[i][j][r];
        }
      }
}

// ------------------------------------------------------------------------------------------
// Term-walk FP64 / FP32 grouped GEMM: a workgroup walks its group's terms one by one, each in
// chunks of BK k (a term's last chunk is partial).  Lane layouts of the MFMAs as below; the LDS
// tiles are [k][m] and [k][n] and every MFMA operand is one LDS read.
// ------------------------------------------------------------------------------------------
// Operand staging of the term-walk kernels: each thread holds N elements of the next A chunk
// and N of the next B chunk in registers, so the global loads of chunk i+1 are in flight while
// the MFMAs of chunk i run.
//
// A block is read through a buffer resource whose base is the block's first element: element
// (slow, fast), with `fast` the contiguous coordinate, is at byte (slow * ld + fast) *
// sizeof(T).  Byte offsets within a block fit 31 bits (checked by the planner); an element
// outside the block gets the offset 2^31, which the buffer's range check turns into a zero
// load.  Thread t holds fast = t % FAST and slow = t / FAST + i * STEP (i = 0..N-1), so
// consecutive threads read consecutive addresses and the offsets of a thread's elements differ
// by a uniform stride.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, 0x7fffffff, 0x00020000);
}
constexpr unsigned kOutside = 0x80000000u;
__device__ __forceinline__ void buffer_load(float& v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ __forceinline__ void buffer_load(double& v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

template <class T, int FAST, int SLOW, int NT>
struct Strip {
  static constexpr int STEP = NT / FAST;
  static constexpr int N = SLOW / STEP;
  static_assert(NT % FAST == 0 && SLOW % STEP == 0, "strip does not tile the chunk");
  static __device__ __forceinline__ int fast() { return threadIdx.x % FAST; }
  static __device__ __forceinline__ int slow(int i) { return (int)threadIdx.x / FAST + i * STEP; }
  // elements [slow0, slow_lim) x [fast0, fast_lim) of the block at P are in range
  static __device__ __forceinline__ void load(T (&r)[N], const T* P, int ld, int slow0, int slow_lim, int fast0,
                                              int fast_lim) {
    const __amdgpu_buffer_rsrc_t rs = block_rsrc(P);
    const int f = fast(), s = slow(0);
    const bool fok = fast0 + f < fast_lim;
    const int left = slow_lim - slow0 - s;  // element i is in range while i * STEP < left
    const unsigned base = ((unsigned)(slow0 + s) * (unsigned)ld + (unsigned)(fast0 + f)) * (unsigned)sizeof(T);
    const unsigned step = (unsigned)STEP * (unsigned)ld * (unsigned)sizeof(T);
#pragma unroll
    for (int i = 0; i < N; ++i) buffer_load(r[i], rs, (fok && i * STEP < left) ? base + i * step : kOutside);
  }
};

// A chunk: BM rows x BK k of A (TA: stored k-major, element (k, r) at k * lda + r).
template <class T, bool TA, int BM, int BK, int NT>
struct ALoader {
  typedef Strip<T, TA ? BM : BK, TA ? BK : BM, NT> S;
  static constexpr int N = S::N;
  static __device__ __forceinline__ void coords(int i, int& mm, int& kk) {
    if (TA) { mm = S::fast(); kk = S::slow(i); } else { kk = S::fast(); mm = S::slow(i); }
  }
  static __device__ __forceinline__ void load(T (&r)[N], const T* A, int lda, int row0, int m, int k0, int K) {
    if (TA) S::load(r, A, lda, k0, K, row0, m);
    else S::load(r, A, lda, row0, m, k0, K);
  }
};
// B chunk: BK k x BN columns of B (TB: stored n-major, element (k, c) at c * ldb + k).
template <class T, bool TB, int BN, int BK, int NT>
struct BLoader {
  typedef Strip<T, TB ? BK : BN, TB ? BN : BK, NT> S;
  static constexpr int N = S::N;
  static __device__ __forceinline__ void coords(int i, int& nn, int& kk) {
    if (TB) { kk = S::fast(); nn = S::slow(i); } else { nn = S::fast(); kk = S::slow(i); }
  }
  static __device__ __forceinline__ void load(T (&r)[N], const T* B, int ldb, int col0, int n, int k0, int K) {
    if (TB) S::load(r, B, ldb, col0, n, k0, K);
    else S::load(r, B, ldb, k0, K, col0, n);
  }
};

// LDS tiles [k][r] of the term-walk kernel: row pitch r + 1 words for the FP32 kernel, r + 2
// words for the BF16x3 kernel (whose lanes read eight consecutive k rows), r + 1 doubles for
// FP64.  The bank-conflict counter behaves as if the LDS served a wave in halves of 32 lanes
// over 32 four-byte banks; in that model, with pitch r + 1
// the 32 k of a staging store (32 lanes, one row r) fall on 32 banks, and the operand reads of
// full chunks below are spread so that the two lane groups of a half read rows 16 apart
// (16 pitches = 16 banks apart).  The FP32 kernel's bank-conflict cycles are a third of those
// of pitch r + 2, whose stores put the 32 k on 16 banks.
template <class T>
struct KPitch {
  static constexpr int of(int r) { return r + (sizeof(T) == 8 ? 1 : 2); }
};

// MFMAs of one staged chunk of the term-walk kernel (LDS tiles [k][m], [k][n]); ni, nj, arow,
// bcol as for packed_chunk.  A full FP32 chunk is walked in BK/4 steps where step s gives lane
// group g = lane/16 the k index s + (BK/2)(g & 1) + (BK/4)(g >> 1): groups 0 and 1 (one half of
// the wave) read rows BK/2 = 16 apart, as do groups 2 and 3, which the row pitch r + 1 puts 16
// banks apart.  A partial chunk (the last chunk of a short term) takes k = 4 s + g instead, so
// that steps wholly past the term's end are skipped.  The sum over k is the same for any
// assignment that A and B share.
template <int MODE, int BK, int TM, int TN, class TA_, class TB_>
__device__ __forceinline__ void terms_chunk(const TA_& As, const TB_& Bs, int arow, int bcol, int kmax, int ni,
                                            int nj, typename Mfma<MODE>::Acc (&acc)[TM][TN]) {
  typedef typename Mfma<MODE>::T T;
  const int lane = threadIdx.x & 63;
  // FP32 full chunk: row of step st = st + (BK/4) g; otherwise 4 st + g
  const bool spread = MODE == 1 && kmax >= BK;
  const int g = lane >> 4;
  const int r0 = spread ? (BK / 2) * (g & 1) + (BK / 4) * (g >> 1) : g;
  const int rs = spread ? 1 : 4;
#pragma unroll
  for (int st = 0; st < BK / 4; ++st) {
    if (spread || 4 * st < kmax) {
      const int row = r0 + rs * st;
      T a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[row][arow + i * 16];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = Bs[row][bcol + j * 16];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          if (i < ni && j < nj) acc[i][j] = Mfma<MODE>::step(a[i], b[j], acc[i][j]);
    }
  }
}

// LDS of the term-walk kernel: FP64 / FP32 operands as [k][r] tiles (pitches in KPitch); the
// BF16x3 kernel splits each operand once, as it is staged, into bf16 hi and lo tiles [r][k] whose
// rows are 40 elements (80 bytes) apart, so that a lane reads its eight k values of a row with one
// 16-byte access and eight consecutive rows fall on eight different 16-byte bank groups.
template <int MODE, class T, int BM, int BN, int BK>
struct TermsLds {
  static constexpr int PA = MODE == 1 ? BM + 1 : KPitch<T>::of(BM);  // see KPitch
  static constexpr int PB = MODE == 1 ? BN + 1 : KPitch<T>::of(BN);
  T As[BK][PA];
  T Bs[BK][PB];
};
template <class T, int BM, int BN, int BK>
struct TermsLds<2, T, BM, BN, BK> {
  static constexpr int KP = BK + 8;
  __attribute__((aligned(16))) __bf16 Ah[BM][KP];
  __attribute__((aligned(16))) __bf16 Al[BM][KP];
  __attribute__((aligned(16))) __bf16 Bh[BN][KP];
  __attribute__((aligned(16))) __bf16 Bl[BN][KP];
};

template <int MODE, bool TA, bool TB, int BM, int BN, int WM, int WN>
__device__ __forceinline__ void gemm_terms_body(const GemmTerm* __restrict__ terms, const GemmGroup* __restrict__ groups,
                                                const GemmTile* __restrict__ tiles, int n_tiles,
                                                Bases<typename Mfma<MODE>::T> bases,
                                                const Bases<typename Mfma<MODE>::T>* __restrict__ table,
                                                const int* __restrict__ active) {
  typedef typename Mfma<MODE>::T T;
  typedef typename Mfma<MODE>::Acc Acc;
  constexpr int BK = 128 / (int)sizeof(T);  // one 128-byte line of a row per chunk
  constexpr int TM = BM / WM / 16;
  constexpr int TN = BN / WN / 16;
  constexpr int NT = 64 * WM * WN;
  typedef ALoader<T, TA, BM, BK, NT> LA;
  typedef BLoader<T, TB, BN, BK, NT> LB;
  __shared__ TermsLds<MODE, T, BM, BN, BK> lds;

  __shared__ BaseTable<T> bt;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;

  const GemmTile tile = tiles[xcd_remap(blockIdx.x, n_tiles)];
  const GemmGroup g = groups[tile.group];
  // a problem whose active flag is 0 is skipped (batched: converged; single: halted solve)
  if (active && !active[table ? g.problem : 0]) return;
  const Bases<T>* row = table ? table + g.problem : nullptr;  // batched: per-problem operands
  bt.stage(bases, row);
  __syncthreads();
  const int tm = tile.tile / g.tiles_n, tn = tile.tile % g.tiles_n;
  const int row0 = tm * BM, col0 = tn * BN;
  const int arow = wm * (BM / WM) + (lane & 15), bcol = wn * (BN / WN) + (lane & 15);
  const int ni = live_subtiles<TM>(row0 + wm * (BM / WM), g.m);
  const int nj = live_subtiles<TN>(col0 + wn * (BN / WN), g.n);

  Acc acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

  // chunk iterator over (term, k0); registers hold the chunk that is staged next
  T ra[LA::N], rb[LB::N];
  int t = g.term_begin, k0 = 0;
  GemmTerm term;
  if (t < g.term_end) {
    term = terms[t];
    LA::load(ra, bt.get(term.a_base) + term.a_off, term.lda, row0, g.m, 0, term.k);
    LB::load(rb, bt.get(term.b_base) + term.b_off, term.ldb, col0, g.n, 0, term.k);
  }
  while (t < g.term_end) {
    const T alpha = (T)term.alpha;
    const int kmax = min(BK, term.k - k0);
    __syncthreads();
    if constexpr (MODE == 2) {
#pragma unroll
      for (int i = 0; i < LA::N; ++i) {
        int mm, kk;
        LA::coords(i, mm, kk);
        const float x = alpha * ra[i];
        const __bf16 h = (__bf16)x;
        lds.Ah[mm][kk] = h;
        lds.Al[mm][kk] = (__bf16)(x - (float)h);
      }
#pragma unroll
      for (int i = 0; i < LB::N; ++i) {
        int nn, kk;
        LB::coords(i, nn, kk);
        const float x = rb[i];
        const __bf16 h = (__bf16)x;
        lds.Bh[nn][kk] = h;
        lds.Bl[nn][kk] = (__bf16)(x - (float)h);
      }
    } else {
#pragma unroll
      for (int i = 0; i < LA::N; ++i) {
        int mm, kk;
        LA::coords(i, mm, kk);
        lds.As[kk][mm] = alpha * ra[i];
      }
#pragma unroll
      for (int i = 0; i < LB::N; ++i) {
        int nn, kk;
        LB::coords(i, nn, kk);
        lds.Bs[kk][nn] = rb[i];
      }
    }
    __syncthreads();
    k0 += BK;
    if (k0 >= term.k) {
      ++t;
      k0 = 0;
      if (t < g.term_end) term = terms[t];
    }
    if (t < g.term_end) {
      LA::load(ra, bt.get(term.a_base) + term.a_off, term.lda, row0, g.m, k0, term.k);
      LB::load(rb, bt.get(term.b_base) + term.b_off, term.ldb, col0, g.n, k0, term.k);
    }
    if constexpr (MODE == 2) {
      bf16x3_chunk_live<TM, TN>(lds.Ah, lds.Al, lds.Bh, lds.Bl, arow, bcol, ni, nj, acc);
    } else {
      // waves issuing a chunk's MFMAs go ahead of waves staging the next chunk, so that the
      // matrix pipe stays fed while others store and wait at the barrier (1.6% on the
      // dominant FP32 launch)
      __builtin_amdgcn_s_setprio(1);
      terms_chunk<MODE, BK, TM, TN>(lds.As, lds.Bs, arow, bcol, kmax, ni, nj, acc);
      __builtin_amdgcn_s_setprio(0);
    }
  }

  const gmut<T> C = global_mut(bt.get(g.c_base) + g.c_off);
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wm * (BM / WM) + i * 16 + Mfma<MODE>::row(lane, r);
        const int gc = col0 + wn * (BN / WN) + j * 16 + (lane & 15);
        if (gr < g.m && gc < g.n) {
          const gmut<T> p = C + (int64_t)gr * g.ldc + gc;
          *p = g.accumulate ? *p + acc[i][j][r] : acc[i][j][r];
        }
      }
}

template <int MODE, bool TA, bool TB, int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN)
gemm_terms_kernel(const GemmTerm* __restrict__ terms, const GemmGroup* __restrict__ groups,
                  const GemmTile* __restrict__ tiles, int n_tiles, Bases<typename Mfma<MODE>::T> bases,
                  const Bases<typename Mfma<MODE>::T>* __restrict__ table, const int* __restrict__ active) {
  gemm_terms_body<MODE, TA, TB, BM, BN, WM, WN>(terms, groups, tiles, n_tiles, bases, table, active);
}

// The BF16x3 term walk: each operand element is split into bf16 hi and lo once, as it is staged
// (TermsLds), and the chunk runs bf16x3_chunk_live.  Its chunks are bound by LDS reads (per 32 k,
// a wave reads hi and lo of all its rows and columns for three MFMAs per 16x16 sub-tile), so the
// 128x128 tile runs four waves of 64x64 (the launcher maps it), whose reads per MFMA are two
// thirds of those of eight waves of 32x64, at three waves per SIMD (about 155 registers); the
// other shapes keep four waves per SIMD.
template <int BM, int BN, int WM, int WN>
struct Bf16x3Waves {
  static constexpr int value = (BM == 128 && BN == 128 && WM * WN == 4) ? 3 : 4;
};
template <bool TA, bool TB, int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN) __attribute__((amdgpu_waves_per_eu(Bf16x3Waves<BM, BN, WM, WN>::value)))
gemm_bf16x3_terms_kernel(const GemmTerm* __restrict__ terms, const GemmGroup* __restrict__ groups,
                         const GemmTile* __restrict__ tiles, int n_tiles, Bases<float> bases,
                         const Bases<float>* __restrict__ table, const int* __restrict__ active) {
  gemm_terms_body<2, TA, TB, BM, BN, WM, WN>(terms, groups, tiles, n_tiles, bases, table, active);
}

// ------------------------------------------------------------------------------------------
// Launchers.  The tile shape (rows x cols per workgroup, wave grid) is chosen per group by the
// planner from the block sizes; see kTileShapes in internal.h.
// ------------------------------------------------------------------------------------------
template <int MODE, bool TA, bool TB, int BM, int BN, int WM, int WN>
static void fire_mfma(const GemmDesc& d, const Bases<typename Mfma<MODE>::T>& b, hipStream_t s,
                      const Bases<typename Mfma<MODE>::T>* table, const int* active) {
  if (d.packed)
    hipLaunchKernelGGL((gemm_packed_kernel<MODE, TA, TB, BM, BN, WM, WN>), dim3(d.n_tiles), dim3(64 * WM * WN), 0, s,
                       d.slots, d.groups, d.tiles, d.n_tiles, b, table, active);
  else
    hipLaunchKernelGGL((gemm_terms_kernel<MODE, TA, TB, BM, BN, WM, WN>), dim3(d.n_tiles), dim3(64 * WM * WN), 0, s,
                       d.terms, d.groups, d.tiles, d.n_tiles, b, table, active);
}
template <int MODE, int BM, int BN, int WM, int WN>
static hipError_t launch_mfma_shape(const GemmDesc& d, const Bases<typename Mfma<MODE>::T>& b, hipStream_t s,
                                    const Bases<typename Mfma<MODE>::T>* table, const int* active) {
  if (d.n_tiles <= 0) return hipSuccess;
  if (!d.ta && !d.tb) fire_mfma<MODE, false, false, BM, BN, WM, WN>(d, b, s, table, active);
  else if (!d.ta && d.tb) fire_mfma<MODE, false, true, BM, BN, WM, WN>(d, b, s, table, active);
  else if (d.ta && !d.tb) fire_mfma<MODE, true, false, BM, BN, WM, WN>(d, b, s, table, active);
  else fire_mfma<MODE, true, true, BM, BN, WM, WN>(d, b, s, table, active);
  return hipGetLastError();
}

template <bool TA, bool TB, int BM, int BN, int WM, int WN>
static void fire_bf(const GemmDesc& d, const Bases<float>& b, hipStream_t s, const Bases<float>* table,
                    const int* active) {
  if (d.packed)
    hipLaunchKernelGGL((gemm_bf16x3_packed_kernel<TA, TB, BM, BN, WM, WN>), dim3(d.n_tiles), dim3(64 * WM * WN), 0, s,
                       d.slots, d.groups, d.tiles, d.n_tiles, b, table, active);
  else
    hipLaunchKernelGGL((gemm_bf16x3_terms_kernel<TA, TB, BM, BN, WM, WN>), dim3(d.n_tiles), dim3(64 * WM * WN), 0, s,
                       d.terms, d.groups, d.tiles, d.n_tiles, b, table, active);
}
template <int BM, int BN, int WM, int WN>
static hipError_t launch_bf_shape(const GemmDesc& d, const Bases<float>& b, hipStream_t s, const Bases<float>* table,
                                  const int* active) {
  if (d.n_tiles <= 0) return hipSuccess;
  if constexpr (BM == 128 && BN == 128 && WM * WN != 4) {
    return launch_bf_shape<128, 128, 2, 2>(d, b, s, table, active);  // four waves of 64x64 (see above)
  } else {
    if (!d.ta && !d.tb) fire_bf<false, false, BM, BN, WM, WN>(d, b, s, table, active);
    else if (!d.ta && d.tb) fire_bf<false, true, BM, BN, WM, WN>(d, b, s, table, active);
    else if (d.ta && !d.tb) fire_bf<true, false, BM, BN, WM, WN>(d, b, s, table, active);
    else fire_bf<true, true, BM, BN, WM, WN>(d, b, s, table, active);
    return hipGetLastError();
  }
}

#define LCC_SHAPE_SWITCH(FN, ...)                                          \
  switch (d.shape) {                                                       \
    case 0: return FN<__VA_ARGS__ 64, 64, 2, 2>(d, b, stream, table, active);   \
    case 1: return FN<__VA_ARGS__ 16, 64, 1, 4>(d, b, stream, table, active);   \
    case 2: return FN<__VA_ARGS__ 64, 16, 4, 1>(d, b, stream, table, active);   \
    case 3: return FN<__VA_ARGS__ 32, 32, 2, 2>(d, b, stream, table, active);   \
    case 4: return FN<__VA_ARGS__ 128, 64, 2, 2>(d, b, stream, table, active);  \
    case 5: return FN<__VA_ARGS__ 64, 128, 2, 2>(d, b, stream, table, active);  \
    case 6: return FN<__VA_ARGS__ 32, 64, 2, 2>(d, b, stream, table, active);   \
    case 7: return FN<__VA_ARGS__ 64, 32, 2, 2>(d, b, stream, table, active);   \
    case 8: return FN<__VA_ARGS__ 128, 128, 4, 2>(d, b, stream, table, active); \
    default: return hipErrorInvalidValue;                                  \
  }

hipError_t launch_gemm_f64(const GemmDesc& d, const Bases<double>& b, hipStream_t stream, const Bases<double>* table,
                           const int* active) {
  LCC_SHAPE_SWITCH(launch_mfma_shape, 0, )
}
hipError_t launch_gemm_f32(const GemmDesc& d, const Bases<float>& b, hipStream_t stream, const Bases<float>* table,
                           const int* active) {
  LCC_SHAPE_SWITCH(launch_mfma_shape, 1, )
}
hipError_t launch_gemm_bf16x3(const GemmDesc& d, const Bases<float>& b, hipStream_t stream, const Bases<float>* table,
                              const int* active) {
  LCC_SHAPE_SWITCH(launch_bf_shape, )
}
#undef LCC_SHAPE_SWITCH

// ------------------------------------------------------------------------------------------
// Split-K reduction of partial output tiles, in a fixed order (deterministic).
// ------------------------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(kThreads)
reduce_kernel(const ReduceGroup* __restrict__ groups, const ReduceTile* __restrict__ tiles, Bases<T> bases,
              const Bases<T>* __restrict__ table, const int* __restrict__ active) {
  const ReduceTile tile = tiles[blockIdx.x];
  const ReduceGroup g = groups[tile.group];
  if (active && !active[table ? g.problem : 0]) return;
  if (table) bases = table[g.problem];
  const int64_t mn = (int64_t)g.m * g.n;
  const T* __restrict__ src = bases.p[BASE_WORK] + g.src_off;
  T* __restrict__ dst = bases.p[BASE_Y] + g.dst_off;
#pragma unroll
  for (int i = 0; i < kReduceChunk / kThreads; ++i) {
    const int64_t e = (int64_t)tile.chunk * kReduceChunk + i * kThreads + threadIdx.x;
    if (e < mn) {
      T s = 0;
      for (int p = 0; p < g.parts; ++p) s += src[p * mn + e];
      const int r = (int)(e / g.n), c = (int)(e % g.n);
      dst[(int64_t)r * g.ldc + c] = s;
    }
  }
}
hipError_t launch_reduce_f64(const ReduceGroup* groups, const ReduceTile* tiles, int n_tiles,
                             const Bases<double>& b, hipStream_t stream, const Bases<double>* table,
                             const int* active) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_kernel<double>, dim3(n_tiles), dim3(kThreads), 0, stream, groups, tiles, b, table, active);
  return hipGetLastError();
}
hipError_t launch_reduce_f32(const ReduceGroup* groups, const ReduceTile* tiles, int n_tiles,
                             const Bases<float>& b, hipStream_t stream, const Bases<float>* table,
                             const int* active) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_kernel<float>, dim3(n_tiles), dim3(kThreads), 0, stream, groups, tiles, b, table, active);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Block mixing: dst_g = sum_t alpha_t src_t over contiguous blocks of equal size.
// ------------------------------------------------------------------------------------------
constexpr int kMixChunk = 1024;

__global__ void __launch_bounds__(kThreads)
mix_kernel(const MixTerm* __restrict__ terms, const MixGroup* __restrict__ groups,
           const MixTile* __restrict__ tiles, Bases<double> bases) {
  const MixTile tile = tiles[blockIdx.x];
  const MixGroup g = groups[tile.group];
  const int base = tile.chunk * kMixChunk;
  double acc[kMixChunk / kThreads];
#pragma unroll
  for (int i = 0; i < kMixChunk / kThreads; ++i) acc[i] = 0.0;
  for (int t = g.term_begin; t < g.term_end; ++t) {
    const MixTerm term = terms[t];
    const double* __restrict__ src = bases.p[g.src_base] + term.src_off;
#pragma unroll
    for (int i = 0; i < kMixChunk / kThreads; ++i) {
      const int e = base + i * kThreads + threadIdx.x;
      if (e < g.count) acc[i] += term.alpha * src[e];
    }
  }
  double* __restrict__ dst = bases.p[g.dst_base] + g.dst_off;
#pragma unroll
  for (int i = 0; i < kMixChunk / kThreads; ++i) {
    const int e = base + i * kThreads + threadIdx.x;
    if (e < g.count) dst[e] = acc[i];
  }
}

hipError_t launch_mix_f64(const MixTerm* terms, const MixGroup* groups, const MixTile* tiles,
                          int n_tiles, const Bases<double>& b, hipStream_t stream) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(mix_kernel, dim3(n_tiles), dim3(kThreads), 0, stream, terms, groups, tiles, b);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Vector operations.  Dot products accumulate in FP64 with a fixed two-level tree
// (kDotBlocks partial sums, then one block), so they are reproducible run to run.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kThreads / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kThreads / 64; ++i) r += red[i];
  }
  return r;
}

template <class T>
__global__ void __launch_bounds__(kThreads) dot_partial_kernel(const T* __restrict__ x, const T* __restrict__ y,
                                                               int64_t n, double* __restrict__ partial) {
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    s += (double)x[i] * (double)y[i];
  s = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kThreads) dot_final_kernel(const double* __restrict__ partial, int n,
                                                             double* __restrict__ out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) s += partial[i];
  s = block_sum(s);
  if (threadIdx.x == 0) out[0] = s;
}

hipError_t launch_dot_f64(const double* x, const double* y, int64_t n, double* partial, double* out,
                          hipStream_t s) {
  hipLaunchKernelGGL(dot_partial_kernel<double>, dim3(kDotBlocks), dim3(kThreads), 0, s, x, y, n, partial);
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(kThreads), 0, s, partial, kDotBlocks, out);
  return hipGetLastError();
}
hipError_t launch_dot_f32(const float* x, const float* y, int64_t n, double* partial, double* out,
                          hipStream_t s) {
  hipLaunchKernelGGL(dot_partial_kernel<float>, dim3(kDotBlocks), dim3(kThreads), 0, s, x, y, n, partial);
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(kThreads), 0, s, partial, kDotBlocks, out);
  return hipGetLastError();
}

static inline dim3 grid_for(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

// A coefficient that is exactly zero drops its operand unread: a fresh output buffer (whose
// contents may be anything, NaN included) can be written with b = 0.
template <class T>
__global__ void axpby_kernel(int64_t n, double a, const T* __restrict__ x, double b, T* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double ax = a == 0.0 ? 0.0 : a * (double)x[i];
    const double by = b == 0.0 ? 0.0 : b * (double)y[i];
    y[i] = (T)(ax + by);
  }
}
hipError_t launch_axpby_f64(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  hipLaunchKernelGGL(axpby_kernel<double>, grid_for(n), dim3(kThreads), 0, s, n, a, x, b, y);
  return hipGetLastError();
}
hipError_t launch_axpby_f32(int64_t n, double a, const float* x, double b, float* y, hipStream_t s) {
  hipLaunchKernelGGL(axpby_kernel<float>, grid_for(n), dim3(kThreads), 0, s, n, a, x, b, y);
  return hipGetLastError();
}

template <class S, class D>
__global__ void convert_kernel(int64_t n, const S* __restrict__ x, D* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (D)x[i];
}
hipError_t launch_convert_f64_f32(int64_t n, const double* x, float* y, hipStream_t s) {
  hipLaunchKernelGGL((convert_kernel<double, float>), grid_for(n), dim3(kThreads), 0, s, n, x, y);
  return hipGetLastError();
}
hipError_t launch_convert_f32_f64(int64_t n, const float* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL((convert_kernel<float, double>), grid_for(n), dim3(kThreads), 0, s, n, x, y);
  return hipGetLastError();
}

__global__ void axpy_f32_into_f64_kernel(int64_t n, double a, const float* __restrict__ x, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] += a * (double)x[i];
}
hipError_t launch_axpy_f32_into_f64(int64_t n, double a, const float* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(axpy_f32_into_f64_kernel, grid_for(n), dim3(kThreads), 0, s, n, a, x, y);
  return hipGetLastError();
}

__global__ void nonfinite_kernel(const double* __restrict__ x, int64_t n, int* __restrict__ flag) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(x[i]);
  if (bad) flag[0] = 1;  // benign race: every writer stores the same value
}
hipError_t launch_nonfinite_f64(const double* x, int64_t n, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(nonfinite_kernel, grid_for(n), dim3(kThreads), 0, s, x, n, flag);
  return hipGetLastError();
}

template <class T>
__global__ void fill_kernel(T* __restrict__ x, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] = v;
}
hipError_t launch_fill_f64(double* x, int64_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel<double>, grid_for(n), dim3(kThreads), 0, s, x, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_f32(float* x, int64_t n, float v, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel<float>, grid_for(n), dim3(kThreads), 0, s, x, n, v);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Diagonal of the effective Hamiltonian: gathers of block diagonals, elementwise products.
// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
diag_gather_kernel(const DiagItem* __restrict__ items, Bases<double> bases, double* __restrict__ out) {
  const DiagItem it = items[blockIdx.x];
  const double* __restrict__ src = bases.p[it.src_base] + it.src_off;
  for (int i = threadIdx.x; i < it.count; i += kThreads) out[it.dst_off + i] = it.alpha * src[(int64_t)i * (it.ld + 1)];
}
hipError_t launch_diag_gather(const DiagItem* items, int n_items, const Bases<double>& b, double* out, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(diag_gather_kernel, dim3(n_items), dim3(kThreads), 0, s, items, b, out);
  return hipGetLastError();
}

template <class T>
__global__ void mul_kernel(int64_t n, const T* __restrict__ a, const T* __restrict__ x, T* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a[i] * x[i];
}
hipError_t launch_mul_f64(int64_t n, const double* a, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(mul_kernel<double>, grid_for(n), dim3(kThreads), 0, s, n, a, x, y);
  return hipGetLastError();
}
hipError_t launch_mul_f32(int64_t n, const float* a, const float* x, float* y, hipStream_t s) {
  hipLaunchKernelGGL(mul_kernel<float>, grid_for(n), dim3(kThreads), 0, s, n, a, x, y);
  return hipGetLastError();
}

// Jacobi preconditioner: m[i] = 1 / (d[i] - e0) (FP64 and FP32 copies); flag[0] = 1 if some
// d[i] - e0 <= 0 (the shifted operator is then not positive definite)
__global__ void jacobi_inverse_kernel(int64_t n, const double* __restrict__ d, double e0, double* __restrict__ m64,
                                      float* __restrict__ m32, int* __restrict__ flag) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = d[i] - e0;
    bad |= !(v > 0.0);
    const double inv = v > 0.0 ? 1.0 / v : 0.0;
    m64[i] = inv;
    m32[i] = (float)inv;
  }
  if (bad) flag[0] = 1;  // benign race: every writer stores the same value
}
hipError_t launch_jacobi_inverse(int64_t n, const double* d, double e0, double* m64, float* m32, int* flag,
                                 hipStream_t s) {
  hipLaunchKernelGGL(jacobi_inverse_kernel, grid_for(n), dim3(kThreads), 0, s, n, d, e0, m64, m32, flag);
  return hipGetLastError();
}

}  // namespace lcc

namespace lcc {
// Counter-based start vectors: splitmix64 of (seed, index) mapped to [-0.5, 0.5).
__global__ void random_fill_kernel(double* __restrict__ x, int64_t n, uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    x[i] = (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
  }
}
hipError_t launch_random_fill_f64(double* x, int64_t n, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(random_fill_kernel, grid_for(n), dim3(kThreads), 0, s, x, n, seed);
  return hipGetLastError();
}
}  // namespace lcc

// ------------------------------------------------------------------------------------------
// Segmented vector operations for batched solves.  The vectors of all problems live in one
// arena; SegBlock b covers elements [begin, end) of problem b.problem.  Per-problem scalars
// are device arrays, so a whole CG iteration runs without the host and can be captured in a
// graph.  mask (may be null) switches problems off.
// ------------------------------------------------------------------------------------------
namespace lcc {

template <class T>
__global__ void __launch_bounds__(kThreads)
seg_dot_partial_kernel(const T* __restrict__ a, const T* __restrict__ b, const SegBlock* __restrict__ blocks,
                       double* __restrict__ partial, const int* __restrict__ mask) {
  const SegBlock blk = blocks[blockIdx.x];
  double s = 0.0;
  if (!mask || mask[blk.problem])
    for (int64_t i = blk.begin + threadIdx.x; i < blk.end; i += kThreads) s += (double)a[i] * (double)b[i];
  s = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// out[p] = sum of the partials of problem p, in block order (one thread per problem)
__global__ void seg_dot_final_kernel(const double* __restrict__ partial, const int32_t* __restrict__ first_block,
                                     int n_problems, double* __restrict__ out, const int* __restrict__ mask) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_problems || (mask && !mask[p])) return;
  double s = 0.0;
  for (int b = first_block[p]; b < first_block[p + 1]; ++b) s += partial[b];
  out[p] = s;
}

template <class T>
hipError_t launch_seg_dot(const T* a, const T* b, const SegBlock* blocks, int n_blocks, const int32_t* first_block,
                          int n_problems, double* partial, double* out, const int* mask, hipStream_t s) {
  hipLaunchKernelGGL(seg_dot_partial_kernel<T>, dim3(n_blocks), dim3(kThreads), 0, s, a, b, blocks, partial, mask);
  hipLaunchKernelGGL(seg_dot_final_kernel, dim3((n_problems + 63) / 64), dim3(64), 0, s, partial, first_block,
                     n_problems, out, mask);
  return hipGetLastError();
}
template hipError_t launch_seg_dot<double>(const double*, const double*, const SegBlock*, int, const int32_t*, int,
                                           double*, double*, const int*, hipStream_t);
template hipError_t launch_seg_dot<float>(const float*, const float*, const SegBlock*, int, const int32_t*, int,
                                          double*, double*, const int*, hipStream_t);

// y = (ca ? ca[p] : 1) * ka * x + (cb ? cb[p] : 1) * kb * y
template <class TX, class TY>
__global__ void __launch_bounds__(kThreads)
seg_axpby_kernel(const SegBlock* __restrict__ blocks, const double* __restrict__ ca, double ka,
                 const TX* __restrict__ x, const double* __restrict__ cb, double kb, TY* __restrict__ y,
                 const int* __restrict__ mask) {
  const SegBlock blk = blocks[blockIdx.x];
  if (mask && !mask[blk.problem]) return;
  const double a = (ca ? ca[blk.problem] : 1.0) * ka;
  const double b = (cb ? cb[blk.problem] : 1.0) * kb;
  if (a == 0.0 && b == 0.0) {
    for (int64_t i = blk.begin + threadIdx.x; i < blk.end; i += kThreads) y[i] = (TY)0;
  } else if (b == 0.0) {
    for (int64_t i = blk.begin + threadIdx.x; i < blk.end; i += kThreads) y[i] = (TY)(a * (double)x[i]);
  } else {
    for (int64_t i = blk.begin + threadIdx.x; i < blk.end; i += kThreads) y[i] = (TY)(a * (double)x[i] + b * (double)y[i]);
  }
}

template <class TX, class TY>
hipError_t launch_seg_axpby(const SegBlock* blocks, int n_blocks, const double* ca, double ka, const TX* x,
                            const double* cb, double kb, TY* y, const int* mask, hipStream_t s) {
  hipLaunchKernelGGL((seg_axpby_kernel<TX, TY>), dim3(n_blocks), dim3(kThreads), 0, s, blocks, ca, ka, x, cb, kb, y, mask);
  return hipGetLastError();
}
template hipError_t launch_seg_axpby<double, double>(const SegBlock*, int, const double*, double, const double*,
                                                     const double*, double, double*, const int*, hipStream_t);
template hipError_t launch_seg_axpby<float, float>(const SegBlock*, int, const double*, double, const float*,
                                                   const double*, double, float*, const int*, hipStream_t);
template hipError_t launch_seg_axpby<float, double>(const SegBlock*, int, const double*, double, const float*,
                                                    const double*, double, double*, const int*, hipStream_t);
template hipError_t launch_seg_axpby<double, float>(const SegBlock*, int, const double*, double, const double*,
                                                    const double*, double, float*, const int*, hipStream_t);

}  // namespace lcc
