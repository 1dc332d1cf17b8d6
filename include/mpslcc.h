/*
 * mpslcc.h -- C ABI of the MI355X (gfx950) two-site H_eff x and local LCC solve library.
 *
 * The library implements the hot path of MPS-LCC (Sharma and Alavi, arXiv:1509.00216):
 * the derivative of the transition element <Psi|H|Phi> with respect to the two-site
 * tensor (Implementation section, local-derivative figure), i.e. the effective Hamiltonian
 * of the two-site block applied to a block-sparse vector, and the local linear solve by
 * conjugate gradients of the first-order equation (Theory section, equation for Phi^(n)),
 * equivalently the stationarity of the local Hylleraas functional.
 *
 * Conventions used by every entry point
 *  - Local states of one spatial orbital, in order: |0>, |up>, |dn>, |updn>,
 *    |updn> = c+_up c+_dn |0>.  Quantum numbers (N, 2Sz) = (0,0), (1,1), (1,-1), (2,0).
 *  - Fock ordering: spin orbital 2i (up) before 2i+1 (down), orbital i = chain position i.
 *  - MPS bond j (j = 0..K) lies left of site j and its sectors are labelled by the (N, 2Sz)
 *    of the sites left of it.  Site j maps sector q to q + qn(s).
 *  - All matrices are row-major.  Device vectors are contiguous and on the context's device.
 *  - Status codes: 0 = OK, > 0 warning, < 0 error.  lcc_last_error() gives a message.
 *    No C++ exception or abort crosses this interface.
 *  - Asynchronous calls run on the context's stream; synchronous calls say so.
 *
 * Ownership: handles are owned by the library and freed by their destroy call
 * (destroy(NULL) is a no-op).  A context must outlive every use of the Hamiltonians,
 * environments, batches and sweeps made on it; their destroy calls do not touch the context and
 * may come in any order.  Host input arrays are copied; the caller may free them after
 * the call returns.  Device vectors belong to the caller; the library keeps no pointer to
 * them after a call returns.  A context is not thread safe; distinct contexts are.
 */
#ifndef MPSLCC_H
#define MPSLCC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lcc_status;
#define LCC_OK 0
#define LCC_NOT_CONVERGED 1   /* solve stopped at max_iter / max_outer; x holds the last iterate */
#define LCC_ERR_ARG (-1)      /* invalid argument or inconsistent descriptor */
#define LCC_ERR_QN (-2)       /* a block violates the (N, 2Sz) selection rule */
#define LCC_ERR_NOT_SPD (-3)  /* p^T A p <= 0 met in conjugate gradients */
#define LCC_ERR_NAN (-4)      /* non-finite value in an input or an iterate */
#define LCC_ERR_OOM (-5)      /* device allocation failed */
#define LCC_ERR_HIP (-6)      /* a HIP runtime call failed */
#define LCC_ERR_STATE (-7)    /* handle in the wrong state (e.g. host-only context) */
#define LCC_ERR_NODEV (-8)    /* no usable gfx950 device */

typedef int32_t lcc_precision;
#define LCC_FP64 0    /* FP64 operands, FP64 MFMA */
#define LCC_FP32 1    /* FP32 operands, FP32 MFMA, FP32 accumulation */
#define LCC_BF16X3 2  /* FP32 operands split into bf16 hi + lo; hi*hi + hi*lo + lo*hi on bf16 MFMA,
                         FP32 accumulation */

typedef struct lcc_context_s* lcc_context;
typedef struct lcc_hamiltonian_s* lcc_hamiltonian;
typedef struct lcc_env_s* lcc_env;

/* ---------------------------------------------------------------------------------------
 * Context.  device >= 0 selects a HIP device (must be gfx950); device = -1 makes a host-only
 * context on which only lcc_create_hamiltonian and the Hamiltonian queries work.
 * stream: the hipStream_t all asynchronous work of this context is queued on, borrowed
 * as given (NULL = the device's null stream, which orders with other null-stream work,
 * e.g. PyTorch's default stream).  The caller keeps it alive until the context is
 * destroyed.
 * ------------------------------------------------------------------------------------- */
lcc_status lcc_context_create(int32_t device, void* stream, lcc_context* out);
void lcc_context_destroy(lcc_context ctx);
/* Message of the last failing call on ctx (or of the last context-less failure if ctx is
 * NULL).  Valid until the next call on the same context. */
const char* lcc_last_error(lcc_context ctx);
/* Wait for all work queued on the context's stream. */
lcc_status lcc_context_synchronize(lcc_context ctx);
/* Upper bound, in bytes of FP64 data, of the intermediate (left-enlarged operator times x)
 * that environments built afterwards on this context keep per channel chunk; larger
 * contractions are executed chunk by chunk over the middle-bond channels (default 16 GiB).
 * Smaller values trade launches for memory (e.g. for many environments in one batch). */
lcc_status lcc_context_set_intermediate_limit(lcc_context ctx, int64_t bytes);
/* Concurrency of lcc_apply_heff (and of the solves built on it): the launches of one GEMM
 * phase (one per tile shape) are independent and run on `side_streams` extra streams of
 * default priority next to the context stream, joined by events before the next phase
 * (default 3; 0 issues every launch in order on the context stream).  The results do not
 * depend on it.  The side streams are created on first use and destroyed with the context. */
lcc_status lcc_context_set_overlap(lcc_context ctx, int32_t side_streams);
/* Text file of autotuning results (one line per block-size histogram; created / appended by
 * lcc_env_autotune, read by environment construction).  NULL or "" disables the cache.
 * The path is copied. */
lcc_status lcc_context_set_tune_cache(lcc_context ctx, const char* path);
/* Planner parameters for environments built afterwards on this context when no tuning-cache
 * entry applies (meanings as in lcc_tune_info; defaults 2048, 2048, 0, 2). */
lcc_status lcc_context_set_plan(lcc_context ctx, double tile_overhead, int64_t split_k, int32_t p2_order,
                                int32_t t_colmajor);

/* ---------------------------------------------------------------------------------------
 * Hamiltonian (Theory section, partitioned-Hamiltonian equation, read with the usual 1/2):
 *   H = sum_{ij,s} h[i][j] a+_{is} a_{js}
 *     + 1/2 sum_{ijkl,s,t} eri[i][j][k][l] a+_{is} a+_{kt} a_{lt} a_{js}   (chemists' (ij|kl))
 *     + sum_i u[i] n_{i up} n_{i dn} + e_const
 * restricted to N = n_elec, 2Sz = two_sz.  It is compiled into an MPO (MPO equation) whose
 * bond dimension stays O(k^2) for two-body terms (Implementation section, bound k^2 with
 * spin adaptation; here spin orbitals are used and D is about 2 k^2 at the centre).
 * ------------------------------------------------------------------------------------- */
typedef struct {
  int32_t n_orb;           /* k, number of spatial orbitals = MPS length (1..64) */
  int32_t n_elec;          /* N */
  int32_t two_sz;          /* 2 Sz */
  const double* h;         /* n_orb*n_orb, need not be symmetric (used as given) */
  const double* eri;       /* n_orb^4 or NULL */
  const double* u_onsite;  /* n_orb or NULL */
  double e_const;
  int32_t switch_bond;     /* bond from which two-operator channels are labelled by their
                              right partners; < 0 selects n_orb/2 + 1 */
  const int32_t* site_order; /* n_orb or NULL (identity): chain position p holds orbital
                              site_order[p], a permutation of 0..n_orb-1; h, eri, u_onsite and
                              orb_class are indexed by orbital and mapped to chain order */
  const int32_t* orb_class;  /* n_orb or NULL: 0 core, 1 active, 2 virtual (Theory section: the
                              occupancy constraints of the three orbital sets) */
  int32_t part;              /* 0: H; 1: H0, the terms that move no electron between the classes
                              (partitioned-Hamiltonian equation, Delta n_ex = 0), e_const
                              included; 2: U = H - H0.  1 and 2 need orb_class. */
} lcc_ham_desc;

lcc_status lcc_create_hamiltonian(lcc_context ctx, const lcc_ham_desc* desc, lcc_hamiltonian* out);
void lcc_hamiltonian_destroy(lcc_hamiltonian ham);
/* MPO bond dimensions D_0..D_K (bond_dims has n_orb + 1 entries). */
lcc_status lcc_hamiltonian_bond_dims(lcc_hamiltonian ham, int32_t* bond_dims);
/* Channel quantum-number shifts of MPO bond `bond`: dn[D], d2sz[D] (the change of (N, 2Sz)
 * caused by the channel's operator on the sites left of the bond). */
lcc_status lcc_hamiltonian_channels(lcc_hamiltonian ham, int32_t bond, int32_t* dn, int32_t* d2sz);
/* Nonzero MPO entries of site `site`.  Call with w_in == NULL to get *count; then arrays of
 * *count entries: w_in, w_out and 16 doubles per entry (row-major <s'|W|s>). */
lcc_status lcc_hamiltonian_site_mpo(lcc_hamiltonian ham, int32_t site, int64_t* count,
                                    int32_t* w_in, int32_t* w_out, double* mats);

/* ---------------------------------------------------------------------------------------
 * MPS (MPS equation) as block-sparse site tensors.
 * ------------------------------------------------------------------------------------- */
typedef struct { int32_t n; int32_t two_sz; int32_t dim; } lcc_sector;
typedef struct {
  int32_t left;   /* sector index within bond j */
  int32_t s;      /* local state 0..3 */
  int32_t right;  /* sector index within bond j+1; must equal left + qn(s) */
  const double* data;  /* host, dim(left) x dim(right) row-major */
} lcc_mps_block;
typedef struct {
  int32_t n_sites;               /* K */
  const int32_t* bond_offsets;   /* K+2 entries: bond j owns sectors[bond_offsets[j] .. bond_offsets[j+1]) */
  const lcc_sector* sectors;     /* sectors of each bond, (n, two_sz) strictly increasing */
  const int64_t* block_offsets;  /* K+1 entries: site j owns blocks[block_offsets[j] .. block_offsets[j+1]) */
  const lcc_mps_block* blocks;
} lcc_mps_desc;

/* Build the left environment (sites < site) and right environment (sites > site+1) of
 * the two-site block (site, site+1) and the contraction plan of H_eff (transition-element
 * figure; the derivative graph of the local-derivative figure).  Sites left of the block
 * must be left-canonical and sites right of it right-canonical; this is checked on the
 * device to 1e-10 (LCC_ERR_ARG otherwise).  The block's own tensors are ignored.
 * Synchronous.  The environment keeps its own copies of everything it needs. */
lcc_status lcc_build_environments(lcc_context ctx, lcc_hamiltonian ham, const lcc_mps_desc* mps,
                                  int32_t site, lcc_env* out);
/* The one-site local problem (Implementation section, local-derivative figure and the sweep: one
 * site tensor A^{n_l} with 4 M^2 elements is the unknown): left environment of the sites < site,
 * right environment of the sites > site, and the same H_eff x plan, with the enlarged right
 * operator equal to the right environment itself.  0 <= site < K; sites left of `site` must be
 * left-canonical and sites right of it right-canonical (checked as for lcc_build_environments,
 * LCC_ERR_ARG otherwise); the tensor at `site` is ignored.  The environment's vectors are
 * one-site tensors x[a, s, b] with a a sector of bond site, b a sector of bond site+1 and
 * qn(a) + qn(s) = qn(b): lcc_env_layout lists their blocks as (left = a, s1 = s, s2 = 0,
 * right = b), rows over a and columns over b.  Every call that takes an environment of
 * lcc_build_environments takes this one (apply, flops, layout, diagonal, local solve,
 * eigensolvers, tuner, batches).  Synchronous.  The environment keeps its own copies. */
lcc_status lcc_build_environments_one_site(lcc_context ctx, lcc_hamiltonian ham, const lcc_mps_desc* mps,
                                           int32_t site, lcc_env* out);
void lcc_env_destroy(lcc_env env);

/* Transition operator between two MPS (Implementation section: the transition element <Psi|H|Phi>,
 * contracted site by site between different bra and ket, with the bra's two-site tensor at
 * (site, site+1) removed -- its derivative with respect to that tensor).  Applied to the ket's
 * own two-site tensor x0 (its tensors at site and site+1 contracted over their common bond, in the
 * gauge of the ket's other tensors) it gives P^T H Phi, where P is the bra's two-site isometry
 * and Phi the ket state: the right-hand side of the first-order equation (Theory section,
 * -Q U Phi0 with U the perturbation) projected onto the local space of the first-order MPS, and,
 * with H = 1 (an lcc_ham_desc with h = 0 and e_const = 1), the overlap vector P^T Phi0 of the
 * local projector.  The bra must be left-canonical left of the block and right-canonical right of
 * it (checked to 1e-10, LCC_ERR_ARG otherwise); the ket may be in any gauge and have other bond
 * dimensions.  lcc_apply_heff maps a ket vector (lcc_env_input_layout) to a bra vector
 * (lcc_env_layout); the local solve, the eigensolvers, the tuner and batches refuse such an
 * environment (LCC_ERR_STATE).  Synchronous.  The environment keeps its own copies. */
lcc_status lcc_build_transition_environments(lcc_context ctx, lcc_hamiltonian ham, const lcc_mps_desc* bra,
                                             const lcc_mps_desc* ket, int32_t site, lcc_env* out);
/* The same transition operator with the bra's one site tensor at `site` removed (the derivative
 * of <Psi|H|Phi> with respect to that tensor, local-derivative figure): the right environment
 * covers the sites > site, vectors are one-site tensors as for
 * lcc_build_environments_one_site, and lcc_env_ket_tensor gives the ket's own site tensor at
 * `site`.  0 <= site < K; the bra must be left-canonical left of `site` and right-canonical right
 * of it (checked to 1e-10, LCC_ERR_ARG otherwise).  Synchronous.  The environment keeps its own
 * copies. */
lcc_status lcc_build_transition_environments_one_site(lcc_context ctx, lcc_hamiltonian ham, const lcc_mps_desc* bra,
                                                      const lcc_mps_desc* ket, int32_t site, lcc_env* out);

/* Layout of two-site vectors x, y, b (the unknown tensor of the local problem).
 * Blocks are (left sector a of bond site, s1, s2, right sector b of bond site+2) with
 * qn(a) + qn(s1) + qn(s2) = qn(b); for a one-site environment (left sector a of bond site, s1,
 * s2 = 0, right sector b of bond site+1).  Element (i, j) of a block sits at
 * offset + i * ld + j. */
typedef struct {
  int64_t n_elements;   /* length of a two-site vector */
  int32_t n_blocks;
  int32_t n_sectors;    /* middle-bond sectors (the vector is block diagonal over them) */
  int32_t mpo_bond_dim; /* D of the middle MPO bond: the number of terms L~ (x) R~ */
  int32_t transition;   /* 1 for a transition operator between two MPS (lcc_build_transition_environments) */
  double flops_per_apply;  /* exact algorithmic flops of one H_eff x (see lcc_env_flops) */
} lcc_layout_info;
typedef struct { int32_t left, s1, s2, right; int64_t offset; int32_t ld, rows, cols; } lcc_block_entry;
/* blocks may be NULL; otherwise it receives info->n_blocks entries. */
lcc_status lcc_env_layout(lcc_env env, lcc_layout_info* info, lcc_block_entry* blocks);

/* Layout of the input vectors of an environment: for lcc_build_environments the same as
 * lcc_env_layout; for a transition operator the ket's two-site tensor (x of lcc_apply_heff),
 * while lcc_env_layout describes the bra's (y). */
lcc_status lcc_env_input_layout(lcc_env env, lcc_layout_info* info, lcc_block_entry* blocks);

/* The ket's own two-site tensor at the block of a transition operator (its tensors at site and
 * site+1 contracted over their common bond, on the device when the environment was built), in
 * the input layout: applied to it, the operator gives P^T H Phi of the ket state Phi.  x_dev:
 * double*, lcc_env_input_layout length.  LCC_ERR_STATE for an effective Hamiltonian.  Synchronous. */
lcc_status lcc_env_ket_tensor(lcc_env env, double* x_dev);

/* Diagonal of H_eff in the vector layout: d[(a,s1,i),(s2,b,j)] = sum over the middle MPO channels
 * that keep the sector of the diagonal entries of the enlarged left and right operators' diagonal
 * blocks; one gather and one grouped GEMM per call the first time, cached afterwards.  d_dev:
 * double*, lcc_env_layout length.  LCC_ERR_STATE for a transition operator.  Synchronous. */
lcc_status lcc_env_diagonal(lcc_env env, double* d_dev);

/* Flop counts of one H_eff x: 2*m*n*k summed over every block product the plan performs,
 * split into the products with the enlarged left operator (phase1) and with the enlarged
 * right operator (phase2), whichever order the plan runs them in.  Only symmetry-allowed
 * blocks and nonzero MPO entries are counted; no padding. */
lcc_status lcc_env_flops(lcc_env env, double* phase1, double* phase2);

/* y = H_eff x.  precision LCC_FP64: x, y are double*; LCC_FP32 / LCC_BF16X3: float*.
 * x has the length of lcc_env_input_layout, y of lcc_env_layout (equal unless the environment is
 * a transition operator).  x and y must not overlap.  Asynchronous on the context stream. */
lcc_status lcc_apply_heff(lcc_env env, lcc_precision precision, const void* x_dev, void* y_dev);

/* Time the two grouped-GEMM phases of lcc_apply_heff with HIP events on the context stream:
 * runs `reps` applications y = H_eff x and returns the mean duration of each phase in
 * milliseconds (phase 1: enlarged left operator times x; phase 2: times enlarged right
 * operator, accumulated into y).  Synchronous.  Buffers as for lcc_apply_heff. */
lcc_status lcc_env_profile_apply(lcc_env env, lcc_precision precision, const void* x_dev, void* y_dev,
                                 int32_t reps, float* ms_phase1, float* ms_phase2);

/* Per-launch timing of lcc_apply_heff: every kernel launch of one application (phase-1
 * GEMMs per tile shape, phase-2 GEMMs per tile shape, the phase-2 split-K reduction) is
 * bracketed by HIP events on the context stream, `reps` times.  Call with out == NULL to get
 * *count.  Synchronous. */
typedef struct {
  int32_t phase;    /* 1 or 2 */
  int32_t kind;     /* 0 = grouped GEMM, 1 = split-K reduction */
  int32_t tile_m;   /* workgroup tile rows (GEMM) */
  int32_t tile_n;   /* workgroup tile columns (GEMM) */
  int32_t n_tiles;  /* workgroups in the launch */
  int32_t packed;   /* GEMM kernel: 0 = term walk, 1 = packed k */
  double flops;     /* algorithmic flops of the launch (2 m n k over its block products) */
  double bytes;     /* algorithmic bytes: operands read once + outputs written once */
  double exec_flops; /* MFMA work issued, including padding to the kernel's sub-tiles and k groups */
  float ms;         /* mean duration */
  int32_t layout;   /* GEMM operand storage: bit 0 A k-major (element (k, r) at k lda + r), bit 1 B
                       column-major (element (k, c) at c ldb + k); 0 for the reduction */
} lcc_launch_profile;
lcc_status lcc_env_profile_launches(lcc_env env, lcc_precision precision, const void* x_dev, void* y_dev,
                                    int32_t reps, int32_t* count, lcc_launch_profile* out);

/* Autotuning of the H_eff x plan for the block-size histogram of this environment (bond
 * sectors and dimensions, MPO bond dimension).  Times on the device every candidate of the
 * planner parameters (tile_overhead in {2048, 8192, 32768}: per-tile cost, in output
 * elements, of the tile-shape choice; split_k in {512, 1024, 2048}: accumulation length of
 * a phase-2 split-K part; p2_order in {0, 1}: phase-2 output blocks one after the other, or
 * their parts interleaved by channel so that parts reading the same intermediate columns are
 * neighbours; t_colmajor in {0, 1, 2}: the left enlarged operator first with its intermediate
 * T = Lt X stored row- or column-major (the latter computed as X^T Lt^T so that phase 2 reads
 * long contiguous columns), or the right enlarged operator first, T = X Rt^T row-major and
 * Y += Lt T, which moves the short left-operator products into the accumulation chains; the
 * same flops either way) and, per GEMM
 * launch, both kernels (term walk / packed k), with
 * `reps` timed applications of `precision` per measurement; keeps the fastest plan and
 * chooses the kernels of all three precisions on it.  With a tuning cache set on the
 * context (lcc_context_set_tune_cache) the choice is appended to it, and an entry already
 * there for this histogram is applied without timing.  Environments built later on a
 * context with a cache use a matching entry automatically.  Synchronous; allocates two
 * vectors of workspace.  The environment's apply results do not depend on the choice
 * beyond rounding order. */
typedef struct {
  double tile_overhead;       /* chosen planner parameters */
  int64_t split_k;
  int32_t candidates;         /* plans timed (0 when taken from the cache) */
  int32_t launches;           /* GEMM launches of the chosen plan */
  int32_t packed_launches;    /* ... of which use the packed-k kernel for `precision` */
  int32_t from_cache;         /* 1 if the entry came from the cache */
  int32_t p2_order;           /* phase-2 group order: 0 output-major, 1 channel-major */
  int32_t t_colmajor;         /* 0 / 1: left operator first, T row- / column-major; 2: right operator first */
  float ms_before, ms_after;  /* one H_eff x of `precision`, summed launch times */
} lcc_tune_info;
lcc_status lcc_env_autotune(lcc_env env, lcc_precision precision, int32_t reps, lcc_tune_info* info);

/* Lowest eigenvalue of H_eff by Lanczos with full re-orthogonalisation in FP64 (the DMRG
 * energy functional, Implementation section): `steps` Krylov vectors from a start vector
 * drawn by a counter-based generator from `seed`.  Returns the lowest Ritz value and the
 * norm of its residual ||H_eff u - theta u|| (a rigorous bound: some eigenvalue lies within
 * it).  Synchronous; uses steps+2 device vectors of workspace. */
lcc_status lcc_lowest_eigenvalue(lcc_env env, int32_t steps, uint64_t seed, double* theta, double* residual);

/* lcc_lowest_eigenvalue for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same computation (one
 * Lanczos cycle, same start vector, same results) with the Krylov basis in a fixed 64 MiB
 * device array of the library, one per GPU, held until the process ends; no hipMalloc or
 * hipFree and no stream creation (every launch on the context stream).  Limits:
 * 1 <= steps <= 128 and (steps + 2) * vector length * 8 bytes <= 64 MiB, else LCC_ERR_ARG.
 * The array keeps the last call's contents (every vector is written before it is read); the
 * library runs one such call at a time, as calls overlapping on one GPU would race on the
 * array.  Synchronous. */
lcc_status lcc_lowest_eigenvalue_noalloc(lcc_env env, int32_t steps, uint64_t seed, double* theta, double* residual);

/* Lowest eigenpair of H_eff, the local problem of a DMRG sweep (Implementation section: the
 * DMRG energy functional, stationary at an eigenvector of the effective Hamiltonian; the
 * eigensolver of the sweep that produces the zeroth-order state).  Lanczos cycles of `steps`
 * Krylov vectors with full re-orthogonalisation in FP64, each cycle restarted from the Ritz
 * vector of the previous one, until ||H_eff u - theta u|| <= tol * max(1, |theta|) or
 * `max_restarts` cycles have run.
 * x_dev: double*, length of the layout.  On entry the start vector (all zeros: a start
 * vector drawn by a counter-based generator from `seed`); on return the unit Ritz vector u.
 * theta = u^T H_eff u, residual = ||H_eff u - theta u||.  Returns LCC_NOT_CONVERGED (x_dev
 * still holds the last Ritz vector) when the tolerance was not met, LCC_ERR_ARG for steps < 1,
 * max_restarts < 1 or tol < 0, LCC_ERR_NAN for a non-finite start vector.  Synchronous; uses
 * steps + 2 device vectors of workspace. */
lcc_status lcc_lowest_eigenpair(lcc_env env, int32_t steps, int32_t max_restarts, double tol, uint64_t seed,
                                double* x_dev, double* theta, double* residual);

/* ---------------------------------------------------------------------------------------
 * Local LCC solve:  Q (H_eff - e0) Q x = Q b,  Q = 1 - v v^T (v unit norm) or Q = 1.
 * Conjugate gradients (Implementation section).  precision selects the operator of the
 * iterations: LCC_FP64 runs plain FP64 CG; LCC_FP32 / LCC_BF16X3 run one CG recurrence with
 * the low-precision operator and "reliable updates": whenever the recurrence residual has
 * dropped by inner_tol since the last refresh, the accumulated correction is added to the
 * FP64 solution and the true residual r = Q b - A x is recomputed with the FP64 operator
 * (FP64 iterative refinement that keeps the search direction).  Dot products, scalars, the
 * refreshed residuals and the energy are FP64.  The recurrence's scalars stay in device memory
 * (no host round trip inside an iteration); the low-precision iteration is captured once as a
 * graph on a stream the context creates for it and kept with the environment (recaptured when
 * e0, the precision, v, the preconditioner or the plan change).
 * Synchronous: the call returns after its device work, on the context stream and the graph
 * stream, has finished.  One environment serves one solve at a time.
 * ------------------------------------------------------------------------------------- */
typedef struct {
  lcc_precision precision;
  int32_t max_iter;      /* CG iterations in total (default 1000 when <= 0) */
  double tol;            /* stop when ||Q b - A x|| <= tol ||Q b|| in FP64 (default 1e-10) */
  double inner_tol;      /* mixed precision: residual reduction between two FP64 refreshes
                            (default 0.1) */
  int32_t max_outer;     /* mixed precision: maximum FP64 refreshes (default 200) */
  int32_t replace_every; /* FP64 CG: recompute r = Q b - A x every this many iterations (default 50) */
  int32_t preconditioner; /* 0: none; 1: Jacobi, M = diag(H_eff) - e0 (lcc_env_diagonal), applied as
                             z = Q M^-1 r (Implementation section: the local equations are solved
                             iteratively; the diagonal is the usual preconditioner of those solvers).
                             LCC_ERR_NOT_SPD if an entry of M is <= 0.  Batched solves take 0 only. */
} lcc_solve_opts;
typedef struct {
  int32_t iterations;    /* CG iterations, all precisions */
  int32_t outer;         /* refinement steps (1 for FP64) */
  int32_t applies_fp64;  /* H_eff x products in FP64 */
  int32_t applies_low;   /* H_eff x products in FP32 / BF16X3 */
  double rel_residual;   /* final ||Q b - A x|| / ||Q b|| in FP64 */
  double hylleraas;      /* J(x) = x^T A x - 2 b^T Q x, FP64 */
  double e2;             /* -b^T Q x, equal to J at the exact solution */
  double ms_total;       /* wall time of the call */
} lcc_solve_info;
/* b_dev, v_dev, x_dev: double*.  x_dev holds the initial guess on entry (zeros for none)
 * and the solution on return.  v_dev may be NULL. */
lcc_status lcc_solve_local_lcc(lcc_env env, const lcc_solve_opts* opts, const double* b_dev,
                               double e0, const double* v_dev, double* x_dev, lcc_solve_info* info);

/* ---------------------------------------------------------------------------------------
 * Sweep (Implementation section: one local problem at a time, sweeping over the sites).
 * Two-site blocks starting at `first_site`, moving right (advance) or left (retreat): the
 * environments of every bond are kept.  After each local solve the two-site tensor is split by
 * an SVD per middle-bond sector (a blocked one-sided Jacobi SVD on the device), the m_max
 * largest singular values over all sectors are kept (ties: sector (N, 2Sz) ascending, then
 * index), except those below 1e-10 times the largest, which count as zero.  Moving right, the left factor becomes the new left-canonical site tensor, the left
 * environment is extended by it on the device, and S V^T times the next site's right-canonical
 * tensor becomes the initial guess of the next local problem; moving left, the right factor
 * becomes the right-canonical tensor of the block's right site and the previous site's
 * left-canonical tensor times U S the next guess.
 * ------------------------------------------------------------------------------------- */
typedef struct lcc_sweep_s* lcc_sweep;
typedef struct {
  int32_t site;               /* left site of the block that was split */
  int32_t kept;               /* states kept on the new bond */
  int32_t n_singular;         /* singular values over all sectors */
  int32_t reserved;
  double discarded_weight;    /* sum of discarded s^2 / sum of all s^2 */
  double largest_discarded;   /* largest discarded singular value (0 if none) */
  float ms_svd;               /* wall time: per-sector SVDs */
  float ms_env;               /* wall time: left-environment step and the next block's plan */
  float ms_guess;             /* wall time: next guess */
  float ms_total;             /* wall time of the call */
} lcc_sweep_info;
/* MPS as for lcc_build_environments with the block at first_site.  Synchronous. */
lcc_status lcc_sweep_create(lcc_context ctx, lcc_hamiltonian ham, const lcc_mps_desc* mps, int32_t first_site,
                            lcc_sweep* out);
void lcc_sweep_destroy(lcc_sweep sweep);
/* Environment of the current block (layout, apply, solve).  Borrowed: valid until the next
 * lcc_sweep_advance or lcc_sweep_retreat; lcc_env_destroy on it is a no-op. */
lcc_status lcc_sweep_env(lcc_sweep sweep, lcc_env* out);
/* Copy the initial guess of the current block into x_dev (zeros before the first advance). */
lcc_status lcc_sweep_guess(lcc_sweep sweep, double* x_dev);
/* Split the solved tensor x_dev (current block's layout), truncate to m_max, move one site
 * to the right.  Fails with LCC_ERR_STATE at the last block.  Synchronous. */
lcc_status lcc_sweep_advance(lcc_sweep sweep, const double* x_dev, int32_t m_max, lcc_sweep_info* info);
/* Split as lcc_sweep_advance, keep the right factor, move one site to the left.  Fails with
 * LCC_ERR_STATE at the first block.  Synchronous. */
lcc_status lcc_sweep_retreat(lcc_sweep sweep, const double* x_dev, int32_t m_max, lcc_sweep_info* info);
/* Left site of the current block. */
lcc_status lcc_sweep_position(lcc_sweep sweep, int32_t* site);
/* Split the block tensor x_dev as lcc_sweep_advance does, without moving: the block's left site
 * gets the left-canonical factor, its right site S V^T (the MPS is then complete, canonical
 * around the block, and can be read out with lcc_sweep_bond / lcc_sweep_site_tensor).  The
 * block's environments and local problem are unchanged.  Synchronous. */
lcc_status lcc_sweep_split_block(lcc_sweep sweep, const double* x_dev, int32_t m_max, lcc_sweep_info* info);
/* Sectors of MPS bond `bond` (0..n_sites) of the sweep: call with sectors == NULL for *count. */
lcc_status lcc_sweep_bond(lcc_sweep sweep, int32_t bond, int32_t* count, lcc_sector* sectors);
/* Site tensor `site` of the sweep's MPS, copied to the host: blocks (left sector, s, right
 * sector, rows, cols, offset into data_host; row-major FP64).  Call with blocks == NULL or
 * data_host == NULL for *n_blocks and *n_elements.  The two sites of the current block hold
 * their last split (lcc_sweep_split_block, or the input MPS before any split).  Synchronous. */
typedef struct { int32_t left, s, right, rows, cols; int64_t offset; } lcc_site_block;
lcc_status lcc_sweep_site_tensor(lcc_sweep sweep, int32_t site, int32_t* n_blocks, int64_t* n_elements,
                                 lcc_site_block* blocks, double* data_host);
/* Singular values of the last split, all sectors, descending: call with out == NULL for *count. */
lcc_status lcc_sweep_singular_values(lcc_sweep sweep, int32_t* count, double* out);

/* First-order problems on a sweep (Theory section: the first-order equation of the perturbation
 * series, solved by minimising the Hylleraas functional one block at a time; the projector
 * approximation changes only the right-hand side).  The sweep's MPS is Phi1, built on H0 (the
 * Hamiltonian of lcc_sweep_create, e.g. part = 1 of lcc_ham_desc); `ref` is Phi0 (canonical
 * around any block, norm 1), `op` the operator O of the right-hand side -Q O Phi0 with
 * Q = 1 - |Phi0><Phi0| (O = U for the first-order equation, O = H for the projector
 * approximation), `u` (or NULL) the perturbation U for the third-order energy.  Environments
 * between Phi1 and Phi0 (transition-element figure) for O and for the identity, and of U on
 * Phi1, are kept for every bond and follow the sweep.  The handles must outlive the sweep.
 * Errors: LCC_ERR_QN if the sector or orbital count differs, LCC_ERR_STATE if nothing is
 * attached. */
lcc_status lcc_sweep_attach_reference(lcc_sweep sweep, lcc_hamiltonian op, lcc_hamiltonian u, const lcc_mps_desc* ref);
/* At the current block, with P its environment basis and v = P^T Phi0: b = -(P^T O Phi0 - c v)
 * into b_dev, v / |v| into v_dev (device arrays of the block's layout, n_elements each) and |v|
 * into *v_norm.  With c = <Phi0|O|Phi0>, b is -P^T Q O Phi0; solving (P^T H0 P - E0) x = b with
 * x orthogonal to v (lcc_solve_local_lcc with v_dev; the block's basis follows Phi1 and need
 * not hold Phi0, and when |v| is at rounding level the constraint is void and v_dev is not
 * used) gives the block's Phi1, and the Hylleraas value of the solve is the second-order energy
 * <Phi0|O|Phi1>.  Synchronous. */
lcc_status lcc_sweep_first_order_rhs(lcc_sweep sweep, double c, double* b_dev, double* v_dev, double* v_norm);
/* x^T (P^T U P) x and x^T x for the block's tensor x_dev: with E1 = <Phi0|U|Phi0> the
 * third-order energy of the Wigner 2n+1 expressions is xux - E1 xx.  Synchronous. */
lcc_status lcc_sweep_u_expectation(lcc_sweep sweep, const double* x_dev, double* xux, double* xx);
/* <Phi|H|Phi> of an MPS canonical around the block (site, site + 1) (E0 = <Phi0|H0|Phi0>,
 * c = <Phi0|O|Phi0> of the first-order right-hand side).  Synchronous. */
lcc_status lcc_mps_expectation(lcc_context ctx, lcc_hamiltonian ham, const lcc_mps_desc* mps, int32_t site,
                               double* value);

/* ---------------------------------------------------------------------------------------
 * Batched local solves (many independent two-site problems, e.g. the sites of several sweeps
 * or several perturbation orders).  A batch merges the plans of n environments of one
 * context: each GEMM phase of H_eff x is one launch per tile shape covering every problem,
 * the CG scalars of all problems live on the device with per-problem active flags (converged
 * problems skip all work), and one iteration is captured in a HIP graph and replayed.  The
 * method per problem is the reliable-update mixed-precision CG of lcc_solve_local_lcc
 * (opts->precision must be LCC_FP32 or LCC_BF16X3).
 * ------------------------------------------------------------------------------------- */
typedef struct lcc_batch_s* lcc_batch;
/* The environments must stay alive while the batch exists, and each may appear only once
 * (an environment's intermediate and split-K buffers serve one problem at a time): a repeated
 * environment is LCC_ERR_ARG.  Synchronous. */
lcc_status lcc_batch_create(lcc_context ctx, int32_t n, const lcc_env* envs, lcc_batch* out);
void lcc_batch_destroy(lcc_batch batch);
/* Arrays of n device pointers (b[i], x[i] double*, length of problem i; v may be NULL or hold
 * NULL entries) and n shifts e0[i] (host).  x[i] holds the initial guess on entry and the
 * solution on return; infos (n entries, may be NULL) per problem.  Returns the most severe
 * per-problem status.  Synchronous. */
lcc_status lcc_batch_solve(lcc_batch batch, const lcc_solve_opts* opts, const double* const* b, const double* e0,
                           const double* const* v, double* const* x, lcc_solve_info* infos);
/* One-shot form: creates a batch of the n environments, solves, destroys it. */
lcc_status lcc_solve_local_lcc_batched(int32_t n, const lcc_env* envs, const lcc_solve_opts* opts,
                                       const double* const* b, const double* e0, const double* const* v,
                                       double* const* x, lcc_solve_info* infos);

#ifdef __cplusplus
}
#endif
#endif
