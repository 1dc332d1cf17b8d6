// Internal declarations shared by the host planner (C++) and the gfx950 kernels (HIP).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

namespace lcc {

// ----------------------------------------------------------------------------------------
// Quantum numbers (N, 2Sz) and the four local states |0>, |up>, |dn>, |updn>.
// ----------------------------------------------------------------------------------------
struct QN {
  int n = 0, sz = 0;
  QN() = default;
  QN(int n_, int sz_) : n(n_), sz(sz_) {}
  bool operator<(const QN& o) const { return n != o.n ? n < o.n : sz < o.sz; }
  bool operator==(const QN& o) const { return n == o.n && sz == o.sz; }
  bool operator!=(const QN& o) const { return !(*this == o); }
  QN operator+(const QN& o) const { return QN(n + o.n, sz + o.sz); }
  QN operator-(const QN& o) const { return QN(n - o.n, sz - o.sz); }
};
inline QN local_qn(int s) {
  static const int dn[4] = {0, 1, 1, 2};
  static const int dz[4] = {0, 1, -1, 0};
  return QN(dn[s], dz[s]);
}

// ----------------------------------------------------------------------------------------
// MPO: per site a list of nonzero (w_in, w_out, 4x4) entries; per bond the channel shifts.
// ----------------------------------------------------------------------------------------
struct MpoEntry {
  int win, wout;
  double m[16];  // <s'|W|s> row-major, index s'*4 + s
};
struct Mpo {
  int K = 0;
  std::vector<std::vector<QN>> dq;             // per bond 0..K: channel shift
  std::vector<std::vector<int8_t>> kind;       // per bond: 0 = I, 1 = H, 2 = left label, 3 = right label
  std::vector<std::vector<MpoEntry>> W;        // per site 0..K-1
};
struct HamDesc {
  int K, N, two_sz;
  std::vector<double> h, eri, u;  // in chain order
  double e_const;
  int switch_bond;
  std::vector<int> orb_class;     // chain order; empty = no partition
  int part = 0;                   // 0: H, 1: H0 (class-number-preserving terms), 2: U = H - H0
};
// Builds the MPO; returns an empty string on success or an error message.
std::string build_mpo(const HamDesc& d, Mpo& out);

// ----------------------------------------------------------------------------------------
// Device plans.  Operands are addressed as (base index, element offset) so one plan serves
// every call: base 0 = environment data, 1 = input vector, 2 = intermediate, 3 = output,
// 4 = merged environment blocks, 5 = MPS data.
// ----------------------------------------------------------------------------------------
enum { BASE_ENV = 0, BASE_X = 1, BASE_T = 2, BASE_Y = 3, BASE_MERGED = 4, BASE_MPS = 5, BASE_WORK = 6, NUM_BASES = 7 };

struct GemmTerm {
  int64_t a_off, b_off;
  int32_t lda, ldb, k;
  int8_t a_base, b_base;
  int16_t pad;
  double alpha;
};
struct GemmGroup {
  int64_t c_off;
  int32_t ldc, m, n, tiles_n;
  int32_t term_begin, term_end;  // host-side term range
  int8_t c_base, accumulate;
  int16_t pad0;
  int32_t problem;  // index into the base-pointer table of a batched launch (0 otherwise)
  int32_t slot_begin, slot_end;  // the group's k-quads in the launch's slot array
};
// One k-quad of a term: four consecutive k (kv of them valid) of alpha * op(A) * op(B).
// a_off / b_off are the element offsets of the quad's first k in the A and B base arrays
// (row 0 of A, column 0 of B), so that a group's quads, taken in term order, form one packed
// accumulation stream: terms with short k share the kernel's k chunks instead of each
// padding its own.
struct SlotRec {
  int64_t a_off, b_off;
  int32_t lda, ldb;
  double alpha;
  int8_t a_base, b_base, kv, pad0;
  int32_t pad1;
};
struct GemmTile {
  int32_t group, tile;
};

struct MixTerm {
  int64_t src_off;
  double alpha;
};
struct MixGroup {
  int64_t dst_off;
  int32_t count;
  int32_t term_begin, term_end;
  int8_t src_base, dst_base;
  int16_t pad;
};
struct MixTile {
  int32_t group, chunk;
};

// Split-K reduction: dst[r*ldc + c] = sum_{p < parts} src[p*m*n + r*n + c], p ascending.
struct ReduceGroup {
  int64_t dst_off, src_off;
  int32_t ldc, m, n, parts;
  int32_t problem, pad;
};
struct ReduceTile {
  int32_t group, chunk;
};

template <class T>
struct Bases {
  T* p[NUM_BASES];
};

// Tile shapes of the grouped GEMM: output rows x cols per workgroup (four waves; eight for
// 128 x 128).
constexpr int kNumTileShapes = 9;
constexpr int kTileShapes[kNumTileShapes][2] = {{64, 64}, {16, 64}, {64, 16}, {32, 32}, {128, 64},
                                                {64, 128}, {32, 64}, {64, 32}, {128, 128}};
enum TileShape { TILE_64x64 = 0, TILE_16x64 = 1 };

// Launchers (kernels.hip).  All asynchronous on `stream`.
// One grouped-GEMM launch.  Two kernels implement it: the term walk (each term staged in
// chunks of its own, `terms`) and the packed-k walk (the group's k-quads in shared chunks,
// `slots`); `packed` selects which.
struct GemmDesc {
  const GemmTerm* terms;
  const SlotRec* slots;
  const GemmGroup* groups;
  const GemmTile* tiles;
  int n_tiles, shape;
  bool ta, tb, packed;
};
hipError_t launch_gemm_f64(const GemmDesc& d, const Bases<double>& b, hipStream_t stream,
                           const Bases<double>* table = nullptr, const int* active = nullptr);
hipError_t launch_gemm_f32(const GemmDesc& d, const Bases<float>& b, hipStream_t stream,
                           const Bases<float>* table = nullptr, const int* active = nullptr);
hipError_t launch_gemm_bf16x3(const GemmDesc& d, const Bases<float>& b, hipStream_t stream,
                              const Bases<float>* table = nullptr, const int* active = nullptr);
hipError_t launch_reduce_f64(const ReduceGroup* groups, const ReduceTile* tiles, int n_tiles,
                             const Bases<double>& b, hipStream_t stream, const Bases<double>* table = nullptr,
                             const int* active = nullptr);
hipError_t launch_reduce_f32(const ReduceGroup* groups, const ReduceTile* tiles, int n_tiles,
                             const Bases<float>& b, hipStream_t stream, const Bases<float>* table = nullptr,
                             const int* active = nullptr);
constexpr int kReduceChunk = 1024;
hipError_t launch_mix_f64(const MixTerm* terms, const MixGroup* groups, const MixTile* tiles,
                          int n_tiles, const Bases<double>& b, hipStream_t stream);

// Vector kernels.
constexpr int kDotBlocks = 1024;
hipError_t launch_dot_f64(const double* x, const double* y, int64_t n, double* partial,
                          double* out, hipStream_t stream);
hipError_t launch_dot_f32(const float* x, const float* y, int64_t n, double* partial,
                          double* out, hipStream_t stream);
// y = a*x + b*y with FP64 scalars (a, b given by value); an operand whose coefficient is 0 is not read
hipError_t launch_axpby_f64(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);
hipError_t launch_axpby_f32(int64_t n, double a, const float* x, double b, float* y, hipStream_t s);
// z = x (convert)
hipError_t launch_convert_f64_f32(int64_t n, const double* x, float* y, hipStream_t s);
hipError_t launch_convert_f32_f64(int64_t n, const float* x, double* y, hipStream_t s);
// y += a * x (x float, y double)
hipError_t launch_axpy_f32_into_f64(int64_t n, double a, const float* x, double* y, hipStream_t s);
// out[0] = 1 if any element is not finite
hipError_t launch_nonfinite_f64(const double* x, int64_t n, int* flag, hipStream_t s);
// out[dst_off + i] = alpha * src[src_off + i * (ld + 1)], i < count: the diagonal of a square block
struct DiagItem {
  int64_t src_off, dst_off;
  double alpha;
  int32_t ld, count;
  int8_t src_base, pad0;
  int16_t pad1;
  int32_t pad2;
};
hipError_t launch_diag_gather(const DiagItem* items, int n_items, const Bases<double>& b, double* out, hipStream_t s);
// y = a * x elementwise
hipError_t launch_mul_f64(int64_t n, const double* a, const double* x, double* y, hipStream_t s);
hipError_t launch_mul_f32(int64_t n, const float* a, const float* x, float* y, hipStream_t s);
// m = 1 / (d - e0) in FP64 and FP32; flag[0] = 1 where d - e0 <= 0
hipError_t launch_jacobi_inverse(int64_t n, const double* d, double e0, double* m64, float* m32, int* flag,
                                 hipStream_t s);
// fill
hipError_t launch_fill_f64(double* x, int64_t n, double v, hipStream_t s);
hipError_t launch_fill_f32(float* x, int64_t n, float v, hipStream_t s);

}  // namespace lcc

namespace lcc {
hipError_t launch_random_fill_f64(double* x, int64_t n, uint64_t seed, hipStream_t s);

// Segmented (batched) vector operations: block b covers arena elements [begin, end) of one problem.
struct SegBlock {
  int32_t problem, pad;
  int64_t begin, end;
};
template <class T>
hipError_t launch_seg_dot(const T* a, const T* b, const SegBlock* blocks, int n_blocks, const int32_t* first_block,
                          int n_problems, double* partial, double* out, const int* mask, hipStream_t s);
template <class TX, class TY>
hipError_t launch_seg_axpby(const SegBlock* blocks, int n_blocks, const double* ca, double ka, const TX* x,
                            const double* cb, double kb, TY* y, const int* mask, hipStream_t s);
}  // namespace lcc
