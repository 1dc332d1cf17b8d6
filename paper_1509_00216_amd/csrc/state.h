// Library state behind the opaque C handles.
#pragma once

#include <map>
#include <memory>
#include <tuple>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/mpslcc.h"
#include "internal.h"

namespace lcc {

struct Error {
  lcc_status code;
  std::string msg;
};

// Owning device buffer (hipMalloc / hipFree).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p && hipFree(p) != hipSuccess) (void)hipGetLastError();  // leave no stale error behind
    p = nullptr;
    bytes = 0;
  }
  // throws Error on failure
  void alloc(size_t n);
  template <class T> T* as() const { return static_cast<T*>(p); }
};

void check_hip(hipError_t e, const char* what);
// Upload a host vector into a fresh device buffer (synchronous on `stream`).
template <class T>
void upload(DevBuf& buf, const std::vector<T>& v, hipStream_t s) {
  buf.alloc(v.size() * sizeof(T));
  if (!v.empty()) check_hip(hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s), "upload");
  check_hip(hipStreamSynchronize(s), "upload sync");
}

// Planner parameters (the autotuner's search space besides the per-launch kernel choice).
struct PlanParams {
  double tile_overhead = 2048.0;  // per-tile cost, in output elements, of the tile-shape choice
  int64_t split_k = 2048;         // accumulation length per phase-2 part (split-K)
  int p2_order = 0;               // phase-2 group order: 0 output-major, 1 channel-major
  int t_colmajor = 2;             // 0 / 1: left operator first, T row- / column-major; 2: right operator first
};

// Scalars of the single solve's conjugate-gradient recurrence, kept in device memory
// (cg.hip).  The last four words are the status the host reads back.
enum : int32_t { CG_RUNNING = 0, CG_STOP = 1, CG_HALT_ERROR = 2 };
enum : int32_t { CG_WHY_PAP_NAN = 1, CG_WHY_PAP_NOT_POSITIVE = 2, CG_WHY_RESIDUAL_NAN = 3 };
struct CgScalars {
  double pAp, rr_new, rho_new, c;                      // dot-product outputs
  double alpha, beta, rho, rr, rmax, sc, tol_bn, delta;  // recurrence
  double margin;  // last residual over the threshold that stops the recurrence (< 1: stopped)
  int32_t run;      // 1 while halt is CG_RUNNING: the operator products skip their work at 0
  uint32_t ticket;  // arrival count of the blocks of a fused launch (0 between launches)
  int32_t halt;   // CG_RUNNING, CG_STOP (converged or refresh due), CG_HALT_ERROR
  int32_t err;    // lcc_status of an error
  int32_t why;    // CG_WHY_*
  int32_t iters;  // iterations performed
};
// Launchers of cg.hip.  `partial` holds at least kDotBlocks doubles.
// Status words a direction update posts to the host.
struct CgStatus {
  int32_t halt, err, why, iters;
  double margin;
  double pad;
};
hipError_t launch_cg_set(CgScalars* S, double rho, double rr, double rmax, double sc, double tol_bn, double delta,
                         hipStream_t s);
hipError_t launch_cg_reset(CgScalars* S, hipStream_t s);
// the stop test and beta from S->rr_new (after an unfused |r|^2)
hipError_t launch_cg_after_r(CgScalars* S, bool mixed, bool preconditioned, hipStream_t s);
// beta = rho_new / rho (preconditioned: after the dot r^T z into S->rho_new)
hipError_t launch_cg_beta(CgScalars* S, hipStream_t s);
// *out = *S (out: mapped host memory)
hipError_t launch_cg_copy(const CgScalars* S, CgScalars* out, hipStream_t s);
// Ap <- Q (Ap - e0 p) (Q = 1 - v v^T when v is given), then alpha = rho / p^T Ap
template <class T>
hipError_t launch_cg_shift(int64_t n, double e0, const T* p, T* Ap, const T* v, CgScalars* S, double* partial,
                           hipStream_t s);
// s += alpha p, r -= alpha Ap, then |r|^2, the stop test and (unpreconditioned) beta
template <class T>
hipError_t launch_cg_update(int64_t n, const T* p, T* s_, const T* Ap, T* r, CgScalars* S, double* partial, bool mixed,
                            bool preconditioned, hipStream_t s);
// s += alpha p
template <class T>
hipError_t launch_cg_solution(int64_t n, const T* p, T* s_, const CgScalars* S, hipStream_t s);
// p <- z + beta p; post (may be null) receives the status
template <class T>
hipError_t launch_cg_direction(int64_t n, const T* z, T* p, const CgScalars* S, CgStatus* post, hipStream_t s);
// y <- y - (*c) v
template <class T>
hipError_t launch_cg_deflate(int64_t n, const double* c, const T* v, T* y, hipStream_t s);

constexpr int kHostScalars = 32;
static_assert(sizeof(CgScalars) <= 16 * sizeof(double), "CG record does not fit its pinned slot");
static_assert(sizeof(CgStatus) == 4 * sizeof(double), "CG status slot size");

struct Context {
  void* handle = nullptr;  // the owning lcc_context_s
  int device = -1;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  // scratch for reductions
  DevBuf dot_partial, dot_out;
  // pinned and mapped, kHostScalars doubles: [0] dot read-back, [4, 12) two CgStatus slots,
  // [12, 28) a copy of the CG record; host_scalar_dev is the device's address of it
  double* host_scalar = nullptr;
  double* host_scalar_dev = nullptr;
  int64_t t_budget_elems = (int64_t)1 << 31;  // intermediate (phase-1 output) elements per environment
  PlanParams plan_params;                      // defaults for new environments
  std::string tune_cache;                      // autotuner cache file ("" = none)
  // concurrent launches of one GEMM phase: number of side streams (0 = everything in order)
  int overlap = 3;
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev_join;
  hipEvent_t ev_fork = nullptr;
  // the single solve's status copies, one iteration behind (see solver.cpp), and the stream its
  // captured iterations are recorded and replayed on (a capture needs a stream of its own)
  hipEvent_t ev_status[2] = {nullptr, nullptr};
  hipStream_t graph_stream = nullptr;
  hipEvent_t ev_gate = nullptr;
};

struct Bond {
  std::vector<QN> q;
  std::vector<int> dim;
  std::map<QN, int> index;
  int find(const QN& x) const {
    auto it = index.find(x);
    return it == index.end() ? -1 : it->second;
  }
};

// Block-sparse operator environment: one block per (channel w, column sector c);
// the row sector is c shifted by the channel's (N, 2Sz) change.
struct EnvBlock {
  int w, r, c;
  int64_t off;
  int rows, cols;
};
struct Environment {
  std::vector<EnvBlock> blocks;
  std::unordered_map<int64_t, int> lookup;  // w * nsec + c -> block
  int nsec = 0;
  int64_t size = 0;
  DevBuf data;
  int find(int w, int c) const {
    auto it = lookup.find((int64_t)w * nsec + c);
    return it == lookup.end() ? -1 : it->second;
  }
};

// One grouped-GEMM launch resident on the device.
struct GemmLaunch {
  bool ta = false, tb = false;
  int shape = TILE_64x64;
  int n_tiles = 0;
  int64_t n_slots = 0;
  double flops = 0;          // 2 m n k over the launch's block products
  // MFMA work issued, incl. padding of m, n to the kernel's sub-tiles and of k to its k groups;
  // [precision][packed kernel]; a BF16x3 product counts once, not per split product
  double exec_flops[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  double elems_read = 0;     // distinct operand blocks, each counted once
  double elems_written = 0;  // output blocks
  DevBuf terms, slots, groups, tiles;
  bool packed[3] = {false, false, false};  // kernel per precision (lcc_precision index)
  GemmDesc desc(int precision) const {
    return GemmDesc{terms.as<GemmTerm>(), slots.as<SlotRec>(), groups.as<GemmGroup>(), tiles.as<GemmTile>(),
                    n_tiles, shape, ta, tb, packed[precision]};
  }
};

// Host-side list of output blocks ("groups") and their block products ("terms").
struct GemmBuilder {
  std::vector<GemmTerm> terms;
  std::vector<GemmGroup> groups;
  double flops = 0;
  void group(int8_t c_base, int64_t c_off, int ldc, int m, int n, bool accumulate);
  void term(int8_t a_base, int64_t a_off, int lda, int8_t b_base, int64_t b_off, int ldb, int k, double alpha);
};
// tile_overhead: per-tile cost (in output elements) of the shape choice, see shape_for
std::vector<GemmLaunch> finalize(const GemmBuilder& b, bool ta, bool tb, hipStream_t s, double tile_overhead = 2048.0,
                                 bool longest_first = true);
void run_gemm64(const std::vector<GemmLaunch>& Ls, const Bases<double>& b, hipStream_t s);

struct Plan {
  // channel chunks: phase 1 then phase 2 of each chunk, in order; one launch per tile shape
  struct Chunk {
    std::vector<GemmLaunch> phase1, phase2;
  };
  std::vector<Chunk> chunks;
  DevBuf reduce_groups, reduce_tiles;      // split-K reduction of phase 2
  int n_reduce_tiles = 0;
  double flops1 = 0, flops2 = 0;
};

struct MiddleSector {
  QN q;
  int nrows = 0, ncols = 0;
  int64_t off = 0;
  std::vector<std::pair<int, int>> rows;  // (left sector a, s1)
  std::vector<int> row_off;
  std::vector<std::pair<int, int>> cols;  // (s2, right sector b)
  std::vector<int> col_off;
};

// Reference to an operand block of the enlarged operators: base array, offset, coefficient.
struct OperandRef {
  int8_t base;
  int64_t off;
  double alpha;
};
// What the planner needs besides the environments themselves (kept for re-planning).
struct PlanInputs {
  // output (bra) side and input (ket) side; the same for an effective Hamiltonian
  std::map<QN, int> sec_index, sec_index_in;
  std::map<std::pair<int, int>, std::pair<int, int>> row_at, col_at;  // (a,s1) / (s2,b) -> (sector, index)
  std::map<std::pair<int, int>, std::pair<int, int>> row_at_in, col_at_in;
  // Lt: (w1, a', s1') -> [(a, s1, ref)];  Rt: (w1, s2', b') -> [(s2, b, ref)]
  std::map<std::tuple<int, int, int>, std::vector<std::tuple<int, int, OperandRef>>> lt, rt;
  std::vector<QN> dq_mid;
};

// The single solve's low-precision iteration captured as a graph, once per status slot, with
// the key of everything the capture baked in (precision, options, buffers, plan).
struct CgGraph {
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  std::vector<uintptr_t> key;
  CgGraph() = default;
  CgGraph(const CgGraph&) = delete;
  CgGraph& operator=(const CgGraph&) = delete;
  void release() {
    for (hipGraphExec_t& e : exec)
      if (e) {
        (void)hipGraphExecDestroy(e);
        e = nullptr;
      }
    key.clear();
  }
  ~CgGraph() { release(); }
};

struct Env {
  Context* ctx = nullptr;
  int site = 0, K = 0;
  int D_mid = 0;
  Bond bl, br;  // MPS bonds site and site+2 (of the bra: rows of the operator, the output vector);
                // site and site+1 for the one-site problem
  bool one_site = false;  // vectors are one-site tensors x[a, s, b] (columns: one trivial state)
  std::vector<MiddleSector> sectors;
  std::vector<lcc_block_entry> layout;
  int64_t n_elements = 0;
  // input side (the ket: columns of the operator).  For an effective Hamiltonian bra = ket and
  // these equal the output side; a transition operator between two MPS maps the ket's two-site
  // space onto the bra's.
  bool transition = false;
  Bond bl_in, br_in;
  std::vector<MiddleSector> sectors_in;
  std::vector<lcc_block_entry> layout_in;
  int64_t n_in = 0;
  DevBuf x0;  // transition operator: the ket's own two-site tensor (input layout)
  // device data: [L blocks | R blocks] in FP64 (+ FP32 copy), merged blocks (+ FP32 copy)
  DevBuf env64, env32, merged64, merged32, tbuf, work;
  int64_t env_elems = 0, merged_elems = 0, t_elems = 0, work_elems = 0;
  Plan plan;
  int64_t plan_epoch = 0;  // incremented by every (re)plan
  PlanParams params;
  PlanInputs in;
  // CG workspace
  DevBuf w64[6], w32[6];
  DevBuf flag;
  DevBuf cg;  // CgScalars of the single solve
  CgGraph cg_graph;
  bool have32 = false;
  // diagonal of H_eff (FP64, built on first use) and the Jacobi preconditioner 1 / (diag - e0)
  DevBuf diag64, minv64, minv32;
  bool have_diag = false;
};

struct Hamiltonian {
  Context* ctx = nullptr;
  HamDesc desc;
  Mpo mpo;
};

// MPS on the device: per site the blocks (left sector, s, right sector) of one FP64 buffer.
struct SiteBlock {
  int l, s, r;
  int64_t off;
  int rows, cols;
};
struct DeviceMps {
  int K = 0;
  std::vector<Bond> bonds;
  std::vector<std::vector<SiteBlock>> sites;
  DevBuf data;
};
void load_mps(const lcc_mps_desc& d, int N, int two_sz, hipStream_t s, DeviceMps& out);
Environment unit_env(hipStream_t st);
// one site of the left (right) environment recursion, on the device
Environment left_step(const Environment& L, const DeviceMps& mps, int j, const Mpo& mpo, hipStream_t st);
Environment right_step(const Environment& R, const DeviceMps& mps, int j, const Mpo& mpo, hipStream_t st);
// the same between two MPS: rows of the environment from the bra, columns from the ket
Environment left_step(const Environment& L, const DeviceMps& bra, const DeviceMps& ket, int j, const Mpo& mpo,
                      hipStream_t st);
Environment right_step(const Environment& R, const DeviceMps& bra, const DeviceMps& ket, int j, const Mpo& mpo,
                       hipStream_t st);
void check_identity(const Environment& E, int w_id, const Bond& bond, hipStream_t st, const char* which);
int channel_of_kind(const Mpo& mpo, int bond, int kind);
// (re)plan an environment's H_eff x for the given planner parameters
void plan_env(Env& env, const PlanParams& pp);
// autotuner (tune.cpp): signature of the block-size histogram, cached choice, timed search
uint64_t histogram_signature(const Env& env);
bool apply_tuned(Env& env);
void autotune(Env& env, int precision, int reps, lcc_tune_info* info);
// enlarged operators, vector layout and apply plan of the two-site block (site, site+1)
Env* make_env(Context* ctx, const Mpo& mpo, int site, const Bond& bond_l, const Bond& bond_r,
              const Environment& L, const Environment& R);
// the transition operator between a bra (bonds bra_l, bra_r; rows of L and R) and a ket
Env* make_env(Context* ctx, const Mpo& mpo, int site, const Bond& bra_l, const Bond& bra_r, const Bond& ket_l,
              const Bond& ket_r, const Environment& L, const Environment& R, bool transition, bool one_site = false);
Env* build_transition_env(Context* ctx, const Hamiltonian& ham, const lcc_mps_desc& bra, const lcc_mps_desc& ket,
                          int site, bool one_site = false);
// x0 of a transition operator from the ket's site tensors (site from t1, site + 1 from t2)
void build_ket_tensor(Env& env, const DeviceMps& t1, const DeviceMps& t2, hipStream_t st);
// x0 of a one-site transition operator: the ket's site tensor
void build_ket_site_tensor(Env& env, const DeviceMps& ket, hipStream_t st);
Mpo identity_mpo(int K);

// env.cpp
// two-site block (site, site+1), or with one_site the one-site tensor at `site`
Env* build_env(Context* ctx, const Hamiltonian& ham, const lcc_mps_desc& mps, int site, bool one_site = false);
void ensure_fp32(Env& env);
// diag(H_eff) into env.diag64 (once)
void compute_diagonal(Env& env);
void apply_heff(Env& env, int precision, const void* x, void* y, const int* active = nullptr);
// one launch at a time: after_each(phase, kind, launch) runs after each launch is queued
struct LaunchRef {
  int phase, kind;
  const GemmLaunch* gemm;  // null for the reduction
};
void apply_heff_each(Env& env, int precision, const void* x, void* y,
                     void (*after_each)(void*, const LaunchRef&), void* user);
// lanczos.cpp
void lowest_eigenvalue(Env& env, int steps, uint64_t seed, double* theta, double* residual);
bool lowest_eigenpair(Env& env, int steps, int max_restarts, double tol, uint64_t seed, double* x_io, double* theta,
                      double* residual);
// the same on caller-given device workspace (lanczos_workspace_elems doubles) and host workspace
// (lanczos_host_elems doubles); in_order issues every launch on the context stream (no side
// streams are created)
bool lowest_eigenpair_in(Env& env, int steps, int max_restarts, double tol, uint64_t seed, double* x_io,
                         double* theta, double* residual, double* workspace, double* host_ws, bool in_order);
int64_t lanczos_workspace_elems(const Env& env, int steps);
size_t lanczos_host_elems(int steps);
// noalloc.hip
void scratch_register_current_device();
void lowest_eigenvalue_noalloc(Env& env, int steps, uint64_t seed, double* theta, double* residual);
void profile_apply(Env& env, int precision, const void* x, void* y, int reps, float* ms1, float* ms2);
std::vector<lcc_launch_profile> profile_launches(Env& env, int precision, const void* x, void* y, int reps);
// batch.hip
struct Batch;
Batch* batch_create(Context* ctx, const std::vector<Env*>& envs);
void batch_destroy(Batch* b);
lcc_status batch_solve(Batch& B, const lcc_solve_opts& o, const double* const* b, const double* e0,
                       const double* const* v, double* const* x, lcc_solve_info* infos);
// sweep.hip
struct Sweep;
Sweep* sweep_create(Context* ctx, const Hamiltonian& ham, const lcc_mps_desc& md, int first);
void sweep_destroy(Sweep* s);
Env* sweep_env(Sweep& s);
void sweep_advance(Sweep& s, const double* x, int m_max, lcc_sweep_info* info);
void sweep_retreat(Sweep& s, const double* x, int m_max, lcc_sweep_info* info);
void sweep_copy_guess(Sweep& s, double* x);
const std::vector<double>& sweep_singular_values(Sweep& s);
int sweep_site(const Sweep& s);
void sweep_split_block(Sweep& s, const double* x, int m_max, lcc_sweep_info* info);
const Bond& sweep_bond(const Sweep& s, int j);
const DeviceMps& sweep_site_tensor(const Sweep& s, int j);
void sweep_attach_reference(Sweep& s, const Hamiltonian& op, const Hamiltonian* u, const lcc_mps_desc& ref);
void sweep_first_order_rhs(Sweep& s, double c, double* b, double* v, double* v_norm);
void sweep_u_expectation(Sweep& s, const double* x, double* xux, double* xx);
// solver.cpp
lcc_status solve_local(Env& env, const lcc_solve_opts& o, const double* b, double e0, const double* v,
                       double* x, lcc_solve_info* info);

}  // namespace lcc

struct lcc_context_s {
  lcc::Context c;
};
struct lcc_hamiltonian_s {
  lcc::Hamiltonian h;
};
struct lcc_env_s {
  lcc::Env* e = nullptr;
  bool owned = true;  // false for the environment a sweep lends out
  ~lcc_env_s() {
    if (owned) delete e;
  }
};
struct lcc_sweep_s {
  lcc::Sweep* s = nullptr;
  lcc::Context* ctx = nullptr;
  lcc_env_s view;  // non-owning handle of the current environment
  ~lcc_sweep_s() {
    view.e = nullptr;
    lcc::sweep_destroy(s);
  }
};
struct lcc_batch_s {
  lcc::Batch* b = nullptr;
  lcc::Context* ctx = nullptr;
  ~lcc_batch_s() { lcc::batch_destroy(b); }
};
