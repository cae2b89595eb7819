/*
 * hmdd — hierarchical-matrix (H-matrix) form of the 3D collocation
 * displacement-discontinuity (DD) boundary-element elasticity operator, on
 * AMD Instinct MI355X (gfx950).
 *
 * The operation (paper Sec. 3.1, "Solid mechanics" and "Final system"):
 * for a mesh of flat elements carrying piecewise-constant DD, collocated at
 * element centroids in an infinite isotropic elastic body (Young's modulus
 * E, Poisson ratio nu), the traction change at every collocation point is
 *     T - T0 = E . delta,
 * written in each element's local frame (s1, s2, n) with element-major
 * ordering [delta_s1, delta_s2, delta_n] per element (Sec. 3.1, "local
 * Cartesian coordinate system").  E is compressed as an H-matrix: far-field
 * admissible blocks become low-rank U V^T factors by adaptive cross
 * approximation, near-field blocks stay dense (Sec. 3.1, hierarchical
 * matrices).  The tangent system solved by the Krylov method is
 *     A11 = E - eta/dt - C^ep
 * (Sec. 3.1.1, mechanical Jacobian), with eta/dt + C^ep block diagonal.
 *
 * Conventions shared by every call:
 *   - SI units: metres, pascals; coefficients of E in Pa/m.
 *   - delta = u+ - u-.  Element frame: s1 = unit(v1 - v0),
 *     n = unit((v1 - v0) x (v2 - v0)), s2 = n x s1; collocation point =
 *     vertex mean.  A pressure p inside a crack is the load t = -p n.
 *   - Vectors of DOFs: float64, column c of a block of nrhs vectors starts
 *     at ptr + c * ld, entries element-major [s1, s2, n].
 *   - Pointers named d_* are device pointers (HIP, current device); all
 *     others are host pointers.  The caller owns every array it passes; the
 *     library owns its opaque handles and the device memory behind them.
 *   - hip_stream may be NULL (the null stream).  Work is enqueued on it;
 *     calls return when the work is enqueued unless stated otherwise.
 *   - Every call returns an hm_status; on failure hm_last_error() gives a
 *     thread-local message.  No C++ exception crosses this boundary.  NaN in
 *     inputs is propagated, not detected.
 */
#ifndef HMDD_H
#define HMDD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HM_OK = 0,
    HM_EINVAL = -1,        /* bad argument (null pointer, size, modulus, option) */
    HM_ENOMEM = -2,        /* host or device allocation failed */
    HM_EDEVICE = -3,       /* HIP runtime error or no usable gfx950 device */
    HM_EBADMESH = -4,      /* degenerate, non-planar or non-rectangular element */
    HM_EUNSUPPORTED = -5,  /* option combination not provided */
    HM_ENOTCONV = -6,      /* solver did not reach the tolerance (best iterate returned) */
    HM_EINTERNAL = -7
} hm_status;

/* Storage precisions.  HM_BF16 (far field only): BF16 factors, the vectors
 * they multiply carried as a BF16 hi/lo pair (two MFMA products), so the
 * factors alone set the rounding error.  HM_BF16_1: BF16 factors and
 * vectors rounded to one BF16 each (half the vector traffic and MFMA work;
 * the far field's rounding error grows by about sqrt(2)). */
enum { HM_F64 = 0, HM_F32 = 1, HM_BF16 = 2, HM_BF16_1 = 3 };

typedef struct hm_mesh hm_mesh;
typedef struct hm_op hm_op;

/* Last error message of the calling thread ("" if none). */
const char* hm_last_error(void);

/* Library version string. */
const char* hm_version(void);

/*
 * Layout check between a caller's copy of this header and the library.
 *   n     : number of entries in sizes (HM_ABI_N_STRUCTS for this header)
 *   sizes : host array of sizeof() of the public structs in the order of
 *           HM_ABI_SIZES below
 * Returns HM_OK when every size matches the library's own, HM_EINVAL (with
 * the first mismatching struct named in hm_last_error) otherwise: a program
 * compiled against an older or newer header would otherwise let the library
 * write past the end of its report structs.  Typical use:
 *   size_t s[] = HM_ABI_SIZES;  if (hm_abi_check(HM_ABI_N_STRUCTS, s)) ...
 */
hm_status hm_abi_check(int n, const size_t* sizes);

/* ------------------------------------------------------------------ */
/* Mesh                                                                */
/* ------------------------------------------------------------------ */
/*
 * Create a mesh of flat elements (paper Sec. 3.1: triangles; planar
 * rectangles are also accepted).
 *   nv_per_elem : 3 (triangles) or 4 (planar rectangles, right angles)
 *   xyz         : [n_vert][3] vertex coordinates (global frame, m)
 *   conn        : [n_elem][nv_per_elem] 0-based vertex ids, counter-
 *                 clockwise about the intended normal
 * Errors: HM_EINVAL (sizes, ids out of range), HM_EBADMESH (element area
 * below 1e-12 diam^2, quad not planar or not a rectangle within 1e-10
 * relative).  Host-only; no device is touched.
 */
hm_status hm_mesh_create(int nv_per_elem, int64_t n_vert, const double* xyz, int64_t n_elem,
                         const int64_t* conn, hm_mesh** out);
void hm_mesh_destroy(hm_mesh* mesh);
int64_t hm_mesh_num_elements(const hm_mesh* mesh);

/*
 * Element geometry in the stated convention (host arrays, any may be NULL):
 *   centroid [N][3], frame [N][3][3] (rows s1, s2, n), area [N].
 * Host-only.
 */
hm_status hm_mesh_frames(const hm_mesh* mesh, double* centroid, double* frame, double* area);

/* ------------------------------------------------------------------ */
/* Planning only                                                        */
/* ------------------------------------------------------------------ */
/*
 * Cluster tree and block tree that hm_operator_build would use for
 * (leaf_size, eta) (paper Sec. 3.1, hierarchical matrices: far field
 * low-rank, near field full).  Host-only; no device is touched.
 *   perm [N] (or NULL): element id at each cluster-order position.
 */
typedef struct {
    int64_t n_leaves, n_dense_blocks, n_lowrank_blocks;
    int64_t dense_entries;      /* sum of 9 m n over dense blocks */
    int64_t lowrank_sum_mn;     /* sum of m + n (elements) over low-rank blocks */
    int64_t max_leaf, min_leaf; /* elements per leaf */
    int depth;
    int64_t lowrank_by_level[64];
} hm_plan_info;

hm_status hm_plan_summary(const hm_mesh* mesh, int leaf_size, double eta, hm_plan_info* info, int64_t* perm);

/* ------------------------------------------------------------------ */
/* Exact influence coefficients                                        */
/* ------------------------------------------------------------------ */
/*
 * Exact FP64 coefficient blocks of E (paper Sec. 3.1: analytical
 * integration of the hypersingular kernel over each flat element, taken
 * before the limit, at the receiver centroid), evaluated on the GPU:
 *   d_out[r][c][a][b] = E^{ab}_{d_rows[r], d_cols[c]}  (Pa/m)
 * traction component a (receiver frame) at element rows[r] due to a unit DD
 * component b (source frame) on element cols[c].
 *   d_rows [nr], d_cols [nc] : int64 element ids (device)
 *   d_out  [nr * nc * 9]     : float64 (device)
 * Errors: HM_EINVAL for bad moduli (E <= 0, nu outside (-1, 1/2)) or
 * sizes.  Ids are not range-checked on the device; the caller guarantees
 * 0 <= id < N.
 */
hm_status hm_kernel_block(const hm_mesh* mesh, double young, double nu, int64_t nr, const int64_t* d_rows,
                          int64_t nc, const int64_t* d_cols, double* d_out, void* hip_stream);

/* ------------------------------------------------------------------ */
/* H-matrix operator                                                    */
/* ------------------------------------------------------------------ */
typedef struct {
    int leaf_size;          /* max elements per cluster-tree leaf (1..64); default 64 */
    double eta;             /* admissibility: min(diam) <= eta * dist; default 2 */
    double aca_tol;         /* relative Frobenius tolerance per block; default 1e-6 */
    int max_rank;           /* cap on the rank of a low-rank block (<= 192): a block whose cross approximation
                               needs more is split into its children; default 128 */
    int near_prec;          /* HM_F64 or HM_F32 for dense leaves */
    int far_prec;           /* HM_F64, HM_F32, HM_BF16 or HM_BF16_1 for low-rank factors */
    int keep_f64_reference; /* also keep an all-FP64 copy (used by refinement) */
    int recompress;         /* 1: truncate each cross approximation by SVD at aca_tol / 2 and store it with
                               orthonormal left factors (any rank); default 1 */
    int stack_rows;         /* product layout: the V^T factors of the blocks sharing a source cluster are stored
                               as stacked panels of at most this many rows (1: no stacking, -1: no cap, 0: 128
                               rows for HM_BF16_1, 64 otherwise); default 0 */
    int phase_a_items;      /* product layout: source-leaf sub-panels per V^T X task (1..4096; 0: 16 when that
                               leaves at least 8 tasks per resident phase-A wavefront, else 8); default 0 */
    int phase_b_window;     /* product layout: 16-row tiles per dense + U T task window (1..8; 0: 8);
                               default 0 */
} hm_build_opts;

/* Fill opts with the defaults above (near = far = HM_F64). */
void hm_build_opts_default(hm_build_opts* opts);

/*
 * Build the H-operator of E for (mesh, young, nu) on the current device:
 * cluster tree (recursive median bisection of centroids), block tree with
 * the admissibility rule above (vertex bounding boxes), dense leaves and
 * ACA factors computed by GPU kernels, packed into the requested
 * precisions.  Blocks on the stream; returns after the build completes.
 * In mixed forms (near_prec != HM_F64) the element self-blocks are kept
 * in FP64 and applied in FP64.
 * Errors: HM_EINVAL, HM_EUNSUPPORTED (precision combination), HM_ENOMEM,
 * HM_EDEVICE, HM_EINTERNAL (an admissible block did not converge within
 * max_rank: message names the block).
 */
hm_status hm_operator_build(const hm_mesh* mesh, double young, double nu, const hm_build_opts* opts,
                            void* hip_stream, hm_op** out);
void hm_op_destroy(hm_op* op);

typedef struct {
    int64_t n_elements, n_dof;
    int64_t n_leaves, n_dense_blocks, n_lowrank_blocks;
    int64_t dense_entries;        /* near-field scalars 9 m n of the dense blocks (see dense_entries_stored) */
    int64_t lowrank_entries;      /* stored U and V scalars, sum k c (m+n) over factorisations of c components */
    int64_t self_f64_entries;     /* FP64 self-block scalars (mixed forms) */
    int64_t bytes_near, bytes_far, bytes_self, bytes_reference;
    int min_rank, max_rank;
    double mean_rank;
    int near_prec, far_prec;
    double build_ms, coef_ms, aca_ms, pack_ms;
    int64_t max_dense_bytes_per_leaf;
    int64_t bytes_far_u, bytes_far_v;  /* far-field bytes read by phase B (U) and phase A (V) */
    int64_t rank_sum;                  /* sum of ranks over low-rank factorisations (stored) */
    int64_t rank_sum_aca;              /* the same before recompression */
    double recompress_ms;
    int64_t apply_workspace_bytes;     /* device workspace of one product of the main form (16 columns): each
                                          stream's own, or the part of the no-allocation scratch it needs */
    int64_t lowrank_entries_u;         /* the U part of lowrank_entries: sum k c m (read by phase B) */
    int64_t dense_entries_stored;      /* near-field entries stored (coplanar leaf pairs keep only their
                                          shear-shear and normal-normal parts), without padding */
    int64_t phase_a_tasks;             /* V^T X tasks of one product (main form) */
    int64_t phase_b_tasks;             /* dense + U T tasks of one product (main form) */
    int64_t phase_a_stacks;            /* stacked V^T panel sets */
    int64_t phase_a_partial_bytes;     /* partial sums of V^T X written and re-read per product */
} hm_op_stats;

hm_status hm_operator_stats(const hm_op* op, hm_op_stats* out);

/* apply flags */
#define HM_APPLY_REFERENCE 1u   /* use the FP64 reference copy */
#define HM_APPLY_TANGENT 2u     /* apply A11 = E - D (mask) instead of E */
#define HM_APPLY_ACCUMULATE 4u  /* add the product to d_Y instead of overwriting it */

/*
 * d_Y = E d_X (or A11 d_X with HM_APPLY_TANGENT; d_Y += ... with
 * HM_APPLY_ACCUMULATE) for nrhs vectors
 * (1 <= nrhs <= 16).  d_X [nrhs][ldx], d_Y [nrhs][ldy] float64 (device),
 * ldx, ldy >= 3N; d_X and d_Y must not overlap.  The product runs in the
 * operator's precisions and is returned in FP64.  Reentrant across
 * streams: the operator keeps one workspace per stream (its in-vector and
 * partial-product buffers, hm_op_stats.apply_workspace_bytes), allocated by
 * the first product on that stream, so products of one operator on
 * different streams (and host threads) may overlap; products on one stream
 * run in order.  The first product on a stream allocates device memory
 * (see hm_operator_apply_noalloc).
 */
hm_status hm_operator_apply(const hm_op* op, int nrhs, const double* d_X, int64_t ldx, double* d_Y,
                            int64_t ldy, unsigned flags, void* hip_stream);

/*
 * hm_operator_apply that also measures its stages with HIP events recorded
 * on hip_stream, then synchronises the stream.  stage_ms[5] receives the
 * durations (ms) of: [0] gather of X into fragment chunks, [1] phase A
 * (V^T X for every low-rank block), [2] reduction of phase-A partials,
 * [3] phase B (dense leaves and U T, one workgroup per target leaf),
 * [4] scatter with self/tangent epilogue.  Same arguments and errors as
 * hm_operator_apply.
 */
hm_status hm_operator_apply_timed(const hm_op* op, int nrhs, const double* d_X, int64_t ldx, double* d_Y,
                                  int64_t ldy, unsigned flags, void* hip_stream, double* stage_ms);

/*
 * hm_operator_apply for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the product's workspace is a fixed array of
 * HM_NOALLOC_SCRATCH_BYTES in the library's device code, one per device,
 * held from the library's load on that device until the process ends.
 * Same arguments, flags and results as hm_operator_apply; allocates nothing
 * and frees nothing.  HM_EINVAL when the operator's workspace
 * (hm_op_stats.apply_workspace_bytes, or the reference copy's with
 * HM_APPLY_REFERENCE) exceeds the array.  Every call on a device shares its
 * array: calls that overlap on one device (several streams or threads) race
 * and must be serialised by the caller.  Each call clears the parts of the
 * array that must start at zero with kernels on hip_stream.
 */
#define HM_NOALLOC_SCRATCH_BYTES (256ull << 20)
hm_status hm_operator_apply_noalloc(const hm_op* op, int nrhs, const double* d_X, int64_t ldx, double* d_Y,
                                    int64_t ldy, unsigned flags, void* hip_stream);

/*
 * Set the tangent terms: A11 = E - D on active elements, identity rows and
 * columns on inactive ones (paper Sec. 3.1.1: D = eta/dt + C^ep, block
 * diagonal 3x3 in local frames).
 *   d_D    [N][3][3] float64 row-major (device) or NULL for D = 0
 *   d_mask [N] uint8 (device), 1 = active, or NULL for all active
 * Copies the data; also rebuilds the block-Jacobi preconditioner.
 * Synchronises the stream.
 */
hm_status hm_tangent_set(hm_op* op, const double* d_D, const uint8_t* d_mask, void* hip_stream);

/* ------------------------------------------------------------------ */
/* Batched products over many operators                                 */
/* ------------------------------------------------------------------ */
/*
 * Several independent operators (e.g. many fault meshes, each its own
 * E, paper Sec. 3.1) applied together: their work lists are merged so one
 * gather, one low-rank phase, one reduction, one dense/low-rank phase and
 * one scatter cover all of them, and the sequence is captured once as a
 * HIP graph (use_graph) and replayed.  The two phases run as queue-driven
 * launches: the resident workgroups claim the merged tasks through
 * per-XCD counters that the gather kernel clears at the start of every
 * product (no memset node in the graph).  autotune times candidate
 * phase-A task sizes, then phase-B window heights, on the batch at
 * creation (each candidate in two rounds, keeping its faster time) and
 * keeps the fastest of each (this also changes the member operators' own
 * task lists and sets one phase-B window for all of them).
 * The operators must outlive the batch, share one precision form, and not
 * be applied concurrently with it, nor the batch on two streams at once.
 */
typedef struct hm_batch hm_batch;
typedef struct {
    int use_graph;  /* 1: capture once, replay (default 1) */
    int autotune;   /* 1: tune the phase-A task size and the phase-B window at creation (default 1) */
} hm_batch_opts;

typedef struct {
    int n_ops;
    int64_t total_elements;
    int use_graph;
    int leaves_per_task_a;     /* chosen phase-A task size (without autotune: the first operator's) */
    int tune_candidates[5];    /* candidate task sizes */
    double tune_ms[5];         /* ms per batched product, 16 columns (faster of two rounds of 5) */
    int64_t bytes_operators;   /* stored panel bytes of all operators */
    int phase_b_window;        /* chosen phase-B window (16-row tiles; without autotune: the first operator's) */
    int tune_b_candidates[3];  /* candidate phase-B windows (timed with the chosen phase-A size) */
    double tune_b_ms[3];       /* ms per batched product, 16 columns (faster of two rounds of 5) */
} hm_batch_info;

void hm_batch_opts_default(hm_batch_opts* opts);
hm_status hm_batch_create(int n_ops, hm_op* const* ops, const hm_batch_opts* opts, void* hip_stream,
                          hm_batch** out);
/*
 * Y_i = E_i X_i for every operator i, nrhs columns each (1..16).
 *   d_X[i], d_Y[i] : device pointers, [nrhs][ld] float64 (host arrays of pointers)
 *   ldx, ldy       : per-operator leading dimensions (host arrays) or NULL for 3 N_i
 */
hm_status hm_batch_apply(hm_batch* batch, int nrhs, const double* const* d_X, const int64_t* ldx,
                         double* const* d_Y, const int64_t* ldy, void* hip_stream);
hm_status hm_batch_get_info(const hm_batch* batch, hm_batch_info* out);
void hm_batch_destroy(hm_batch* batch);

/* ------------------------------------------------------------------ */
/* Krylov solve of the tangent system                                   */
/* ------------------------------------------------------------------ */
/*
 * Preconditioners M of the tangent system (right preconditioning; all FP64):
 *   HM_PC_JACOBI   1 / (A11)_ii (the paper's diagonal preconditioner, Sec. 3.3.1)
 *   HM_PC_BLOCK3   (A11)_ee^-1, the 3x3 block of each element
 *   HM_PC_LEARNED  block-Jacobi plus the attached learned correction
 *   HM_PC_LEAF     inverse of each cluster-tree leaf's diagonal block of
 *                  A11 (3m x 3m, m <= 64 elements; E from the collocation
 *                  coefficients, D subtracted on active elements, identity
 *                  rows and columns for inactive ones), formed in FP64 by
 *                  Gauss-Jordan elimination with partial pivoting on first
 *                  use after each hm_tangent_set; 9 m^2 doubles per leaf.
 *                  HM_EINVAL if a block is numerically singular (a pivot
 *                  below 1e-13 of the block's largest |E_ij| + |D_ij|).
 *   HM_PC_ILU      the paper's second approximation of A11 (Sec. 3.3.1,
 *                  solution of the Jacobian system): the fraction p
 *                  (hm_solve_opts.ilu_fraction, default 1 %) of the
 *                  near-field entries of E (entries of the dense leaf
 *                  blocks) of largest magnitude, minus D on every 3x3
 *                  diagonal block (identity rows and columns for inactive
 *                  elements), factorised by ILU(0) and applied by forward and
 *                  backward substitution.  Kept: k = ceil(p x 9 sum m n)
 *                  entries and all ties, compared by a 48-bit magnitude key
 *                  (|a|'s bit pattern without its last 15 bits).  Elimination
 *                  order: elements coloured greedily in increasing id
 *                  (smallest colour free among lower-id neighbours of the
 *                  pattern), by colour then id, DOFs s1, s2, n; each colour is
 *                  one parallel step of the factorisation and of each
 *                  substitution.  The selection, pattern and order depend
 *                  on E, p and the active mask only: they are formed once
 *                  (coefficients and threshold on the GPU, colouring and
 *                  row sort on the host) and kept while p and the mask
 *                  stay the same; the values and the factorisation are
 *                  redone on the GPU on first use after each
 *                  hm_tangent_set.  HM_EINVAL on a zero or non-finite
 *                  pivot.
 */
enum { HM_PC_NONE = 0, HM_PC_JACOBI = 1, HM_PC_BLOCK3 = 2, HM_PC_LEARNED = 3, HM_PC_LEAF = 4, HM_PC_ILU = 5 };

/* why a solve asked for HM_PC_LEARNED ran with HM_PC_BLOCK3 */
enum {
    HM_FALLBACK_NONE = 0,
    HM_FALLBACK_NOT_ATTACHED = 1,  /* no correction attached for the current tangent */
    HM_FALLBACK_NONFINITE = 2,     /* a NaN/Inf reached the Arnoldi process or the residual */
    HM_FALLBACK_NOT_CONVERGED = 3  /* the learned solve missed rtol within max_iter */
};

typedef struct {
    int restart;        /* GMRES(m) restart length, 1..256; default 50 */
    int max_iter;       /* total inner iterations per right-hand side; default 1000 */
    double rtol;        /* stop when ||b - A x|| <= rtol ||b|| (FP64); default 1e-8 */
    int precond;        /* HM_PC_NONE | HM_PC_JACOBI | HM_PC_BLOCK3 | HM_PC_LEARNED | HM_PC_LEAF | HM_PC_ILU;
                           default BLOCK3 */
    int refine;         /* 1: FP64 iterative refinement around a low-precision inner solve */
    double inner_rtol;  /* inner tolerance when refine = 1; 0 (default): 1e-2 with BF16 far field, else 1e-5 */
    int max_refine;     /* refinement sweeps; default 20 */
    double ilu_fraction;/* HM_PC_ILU: fraction p of the near-field entries kept, (0, 1]; 0 or the default: 0.01 */
} hm_solve_opts;

void hm_solve_opts_default(hm_solve_opts* opts);

typedef struct {
    int iterations;           /* inner GMRES iterations, max over right-hand sides */
    int refinements;          /* outer sweeps (refine = 1) */
    int converged;            /* 1 if every column met rtol */
    double rel_residual;      /* max over columns of ||b - A11 x|| / ||b||, FP64, reference operator */
    double solve_ms;
    int n_history;            /* entries written to history (<= 1024) */
    double history[1024];     /* max over columns of the GMRES residual estimate (relative) after each
                                 inner iteration (the newest Arnoldi column enters with its tentative
                                 norm; it is finished one iteration later) */
    int precond_used;         /* preconditioner of the solve that produced X */
    int fallback;             /* HM_FALLBACK_* */
    int discarded_iterations; /* iterations of a learned attempt that was replaced by the fallback */
    double precond_setup_ms;  /* time this solve spent forming its preconditioner (0 when it was current) */
    int64_t precond_nnz;      /* HM_PC_ILU: entries of the factors */
    int precond_colors;       /* HM_PC_ILU: colours (parallel steps of each substitution) */
} hm_solve_report;

/*
 * Solve A11 X = B for nrhs right-hand sides (1 <= nrhs <= 16) by
 * right-preconditioned restarted GMRES(m) from X = 0, Arnoldi by classical
 * Gram-Schmidt with delayed reorthogonalisation in FP64 (the paper's outer/inner
 * Krylov solves, Sec. 3.3.1, use BiCGSTAB or GMRES).  With refine = 1 the
 * inner solve uses the operator's own precisions and an FP64 residual with
 * the FP64 reference copy (built with keep_f64_reference) drives the
 * correction sweeps.  d_B, d_X: [nrhs][ld] float64 (device).  Synchronous.
 * Returns HM_ENOTCONV (with the best iterate in d_X and rep filled) when
 * the tolerance is not met.  With HM_PC_LEARNED the preconditioner is the
 * attached correction's base (3x3 or leaf block-Jacobi) plus the learned
 * correction (hm_learned_attach); the plain preconditioner is the
 * fallback: 3x3 block-Jacobi when nothing is attached, and the solve is run
 * again from X = 0 with the attached correction's base when the learned
 * attempt meets a NaN/Inf or misses rtol (rep->fallback says which).
 * Convergence is always judged by the FP64 true residual.  Reentrant
 * across streams like hm_operator_apply (each stream has its own Krylov
 * workspace, allocated by the first solve on it; the leaf inverses are
 * formed once per tangent by whichever solve needs them first, the others
 * wait for them); hm_tangent_set and the hm_learned_* calls that change the
 * operator must not overlap a solve.
 */
hm_status hm_solve(const hm_op* op, const hm_solve_opts* opts, int nrhs, const double* d_B, int64_t ldb,
                   double* d_X, int64_t ldx, hm_solve_report* rep, void* hip_stream);

/*
 * Z = M^-1 R with the preconditioner the solve would use (HM_PC_*) for op's
 * current tangent: identity, point Jacobi 1/(A11)_ii, 3x3 block-Jacobi
 * (A11)_ee^-1, block-Jacobi plus the attached learned correction
 * (HM_EINVAL if none is attached), or the leaf block inverses (formed here
 * if the tangent changed since they were last formed).  d_R, d_Z:
 * [nrhs][ld] float64 (device), 1 <= nrhs <= 16, not aliased.  Synchronises
 * the stream.
 */
hm_status hm_precond_apply(const hm_op* op, int precond, int nrhs, const double* d_R, int64_t ldr, double* d_Z,
                           int64_t ldz, void* hip_stream);

/* ------------------------------------------------------------------ */
/* Interface elasto-plastic law and its consistent tangent              */
/* ------------------------------------------------------------------ */
/*
 * The constitutive law of the fault/fracture interfaces (paper Sec. 2.2.2
 * "A poroelastoplastic interface law" and Sec. 2.2.3 "Interface yield
 * criteria, flow rule, and damage"), in each element's local frame
 * (s1, s2, n), effective tractions, tension and opening positive:
 *   T' - T'o = C (delta - delta^p), C = diag(k_s, k_s, k_n);
 *   Coulomb  Fc = |tau| + f(chi_s) T'n - c(chi_t), non-associated flow
 *            d delta^p = dlam (tau/|tau| + psi(chi_s) n);
 *   cut-off  Ft = T'n - sigma_t(chi_t), flow along n;
 *   f = f_res + (f_peak - f_res) W(chi_s/d_c), psi = psi_peak W(chi_s/d_c),
 *   c = c_peak W(chi_t/w_c), sigma_t = sigma_peak W(chi_t/w_c),
 *   W(x) = max(0, 1 - x); chi_s = max over time of |delta^p_s|,
 *   chi_t = max over time of |delta^p|;
 *   mode selection h = |tau| - (c - f sigma_t) - alpha (T'n - sigma_t),
 *   alpha = sqrt(1 + f^2) - f: h > 0 Coulomb, else tension;
 *   a fully damaged interface (chi_t >= w_c, or w_c = 0) that opens carries
 *   no traction until its inelastic opening has closed back to the
 *   residual width w_R (which grows by the dilatant part of shear flow).
 * One step is integrated by an elastic predictor and a backward-Euler
 * corrector (single-surface returns, corner when both surfaces are active),
 * and C^ep = dT'/d(delta increment) is the exact derivative of that
 * algorithm: the consistent tangent of the mechanical Jacobian
 * J = E - eta/dt - C^ep (Sec. 3.1.1).  The integration details are in the
 * paper's supplement, which this library does not follow; the scheme above
 * is its own.  Every surface test allows 1e-12 of the trial traction scale
 * (|T_tr| summed over components + c_peak + sigma_peak), so that states the
 * algorithm puts exactly on a surface are not decided by rounding.  The
 * local problems are assumed well posed: each stiffness exceeds the
 * softening rate of the strength it controls.
 */
typedef struct {
    double k_s, k_n;          /* shear and normal stiffness (Pa/m), finite, > 0 */
    double f_peak, f_res;     /* friction coefficient at zero slip and residual: 0 <= f_res <= f_peak */
    double psi_peak;          /* dilatancy coefficient at zero slip, >= 0 (residual 0) */
    double d_c;               /* slip-weakening distance (m): 0 = residual from the start, INFINITY = none */
    double c_peak;            /* cohesion at zero damage (Pa), >= f_peak * sigma_peak */
    double sigma_peak;        /* tensile strength at zero damage (Pa), >= 0 */
    double w_c;               /* critical inelastic DD of c and sigma_t (m): 0 = fully damaged
                                 (pre-existing fracture), INFINITY = no weakening */
} hm_interface_material;

/* Interface modes reported per element */
enum { HM_IF_ELASTIC = 0, HM_IF_SHEAR = 1, HM_IF_TENSILE = 2, HM_IF_CORNER = 3, HM_IF_OPEN = 4,
       HM_IF_BAD_MATERIAL = -1 };

/*
 * Integrate the interface law of n_elem elements over one step.
 *   mats       host array of n_mat materials (1 <= n_mat <= 16), validated:
 *              HM_EINVAL on a violated bound
 *   d_mat_id   [N] int32 material index per element, or NULL for material 0;
 *              an element whose index is outside [0, n_mat) gets NaN
 *              outputs and mode HM_IF_BAD_MATERIAL
 *   d_ddelta   [N][3] increment of the total DD over the step (m)
 *   d_t        [N][3] effective traction T' at the start of the step (Pa)
 *   d_dp       [N][3] inelastic DD delta^p at the start (m)
 *   d_chi      [N][3] internal variables at the start: chi_s, chi_t (m) and
 *              the residual width w_R (m; initially the paper's alpha w_c for
 *              an intact interface, 0 for a pre-existing fracture)
 *   d_t_new, d_dp_new, d_chi_new  [N][3] the same at the end of the step
 *   d_cep      [N][3][3] row-major consistent tangent dT'/d(d_ddelta) (Pa/m)
 *   d_mode     [N] int32 HM_IF_* per element, or NULL
 *   d_eta_dt   [N][3] diagonal of eta/dt (Pa/m) or NULL for 0
 *   d_D        [N][3][3] or NULL: D = C^ep + eta/dt, ready for hm_tangent_set
 * All arrays are FP64/int32 device memory, element-major.  An output may be
 * the same array as the matching input (in-place update); other overlaps
 * are not allowed.  Asynchronous on hip_stream; n_elem = 0 is a no-op.
 */
hm_status hm_interface_update(int n_mat, const hm_interface_material* mats, int64_t n_elem, const int32_t* d_mat_id,
                              const double* d_ddelta, const double* d_t, const double* d_dp, const double* d_chi,
                              double* d_t_new, double* d_dp_new, double* d_chi_new, double* d_cep, int32_t* d_mode,
                              const double* d_eta_dt, double* d_D, void* hip_stream);

/* ------------------------------------------------------------------ */
/* One implicit step of the mechanical problem                          */
/* ------------------------------------------------------------------ */
/*
 * Newton's method on the mechanical residual of a time step (paper Sec.
 * 3.1.1, "Elasto-plastic solver"), the increment dd of the total DD being
 * the unknown:
 *   r(dd) = dT'o - dT'(dd) + E dd + I_n dp - eta (dd - dd_prev) / dt,
 * dT'(dd) the increment of the interface effective traction given by
 * hm_interface_update from the start-of-step state, I_n dp the pore-pressure
 * increment at the collocation points along each element normal; the
 * Jacobian is J = E - eta/dt - C^ep.  Each iteration evaluates the law, the
 * FP64 product E dd (the operator's FP64 reference copy when its main form
 * is lower precision), the residual and its 2-norm, sets the operator's
 * tangent to D = C^ep + eta/dt and solves J y = r with hm_solve (opts.lin:
 * preconditioner, restart, tolerance, refinement); then dd -= y.
 */
typedef struct {
    int max_newton;        /* Newton iterations, 0..63; default 25 */
    double rtol;           /* stop when ||r|| <= max(rtol ||r_0||, atol); default 1e-10 */
    double atol;           /* absolute residual tolerance (Pa); default 0 */
    hm_solve_opts lin;     /* linear solves; default hm_solve_opts_default with rtol 1e-10, max_iter 3000 */
    int forcing;           /* 0 (default): every linear solve to lin.rtol; 1: Eisenstat-Walker forcing
                              (choice 2: 0.9 (||r_k|| / ||r_k-1||)^2, safeguarded, at most 0.1, at least
                              lin.rtol and half the final tolerance over ||r_k||) */
} hm_newton_opts;

typedef struct {
    int iterations;            /* Newton iterations (linear solves) taken */
    int converged;             /* 1 when the residual tolerance was met */
    int n_history;             /* residual evaluations (iterations + 1) */
    double residual[64];       /* ||r_k|| (Pa, 2-norm over all DOF) */
    int gmres_iterations[64];  /* GMRES iterations of each linear solve */
    int64_t modes[5];          /* elements per interface mode (HM_IF_*) at the returned state */
    double ms;                 /* wall time of the step */
} hm_newton_report;

void hm_newton_opts_default(hm_newton_opts* opts);
/*
 * One step.  Interface materials and state as for hm_interface_update
 * (d_t, d_dp, d_chi: [N][3] at the start of the step, not modified);
 *   d_dT0     [N][3] increment of the in-situ effective traction, or NULL
 *   d_dpress  [N] pore-pressure increment at the collocation points, or NULL
 *   d_eta_dt  [N][3] diagonal of eta/dt, or NULL
 *   d_dd_prev [N][3] dt times the previous step's DD rate, i.e. its increment
 *             rescaled to this step (increment_prev * dt / dt_prev), so that
 *             eta (dd - dd_prev) / dt = eta (dd / dt - increment_prev / dt_prev),
 *             the backward-Euler rate change; NULL for zero (first step)
 *   d_dd      [N][3] in: initial guess; out: the returned increment
 *   d_t_new, d_dp_new, d_chi_new  [N][3] the interface state at d_dd
 * All device FP64 arrays, element-major in local frames; the operator is
 * the mesh's (N elements).  On return the operator's tangent is D at the
 * returned state.  HM_ENOTCONV (report filled, last iterate returned) when
 * the tolerance is not met within max_newton iterations; HM_EINVAL when an
 * output array is one of d_t, d_dp, d_chi (the start-of-step state is read
 * at every iteration) or the operator has no FP64 form for the residual.
 * Synchronises the stream; the operator is used by one caller at a time.
 */
hm_status hm_newton_step(hm_op* op, int n_mat, const hm_interface_material* mats, const int32_t* d_mat_id,
                         const double* d_t, const double* d_dp, const double* d_chi, const double* d_dT0,
                         const double* d_dpress, const double* d_eta_dt, const double* d_dd_prev, double* d_dd,
                         double* d_t_new, double* d_dp_new, double* d_chi_new, const hm_newton_opts* opts,
                         hm_newton_report* rep, void* hip_stream);

/* ------------------------------------------------------------------ */
/* Fluid flow in the discontinuities and the fully coupled step         */
/* ------------------------------------------------------------------ */
/*
 * Paper Sec. 3.2 ("Fluid-flow in the discontinuities"): Galerkin P1
 * finite elements on the triangles of the mesh, pressure at its vertices
 * (nodes).  Per element e (area A_e): V picks the normal DD, V_e[a] = A_e/3;
 * storage S_e = (w_e / M) A_e (1 + [a = b]) / 12; transmissibility
 * L_e = (w_e k(w_e) / mu) A_e grad N_a . grad N_b, with the hydraulic width
 * w_e = w0_e + delta_n,e and k(w) = w^2 / 12 (cubic law) or k0; N_p takes
 * the mean of an element's nodes to its collocation point (normal row).  A
 * vertex no element uses carries a decoupled unit storage row.  Only
 * meshes of triangles (HM_EUNSUPPORTED otherwise).  Independently meshed
 * fractures do not share nodes, so no fluid passes between them.
 */
enum { HM_PERM_CUBIC = 0, HM_PERM_CONSTANT = 1 };
typedef struct {
    double M;        /* storage modulus (Pa) of the storage term, > 0 */
    double mu;       /* fluid viscosity (Pa s), > 0 */
    int perm_law;    /* HM_PERM_CUBIC (k = w^2 / 12) or HM_PERM_CONSTANT (k = k0) */
    double k0;       /* permeability (m^2) of HM_PERM_CONSTANT, > 0 */
} hm_flow_params;

typedef struct hm_flow hm_flow;
/* Flow problem on the mesh's triangles (host connectivity copied; the
 * pattern, its node colouring and the assembly maps are built here). */
hm_status hm_flow_create(const hm_mesh* mesh, const hm_flow_params* params, void* hip_stream, hm_flow** out);
void hm_flow_destroy(hm_flow* flow);
int64_t hm_flow_num_nodes(const hm_flow* flow);
int64_t hm_flow_nnz(const hm_flow* flow);
/*
 * S and L assembled on the GPU at hydraulic widths d_w [N] (device), as
 * CSR copies on the host: rowptr [n + 1], col [nnz] (node ids; each row's
 * columns in the order of the node colouring), S [nnz], L [nnz]; any
 * output may be NULL.  Synchronous.
 */
hm_status hm_flow_matrices(const hm_flow* flow, const double* d_w, int64_t* rowptr, int32_t* col, double* S,
                           double* L, void* hip_stream);

/*
 * One implicit step of the coupled hydro-mechanical problem (Sec. 3.3):
 * Newton's method on the unknowns (dd [N][3], dp [n]) of
 *   r_m = dT'o - dT'(dd) + E dd + N_p dp - eta (dd - dd_prev) / dt
 *   r_f = V dd + (S + dt L)(w) dp + dt L(w) (p_n - p_o) - dt f
 * (w at the end of the step, dT'(dd) from hm_interface_update), with the
 * exact Jacobian [A11 N_p; A21 S + dt L], A11 = E - eta/dt - C^ep,
 * A21 = V + dS/dd dp + dt dL/dd (dp + p_n - p_o).  Each Jacobian system is
 * solved by right-preconditioned flexible GMRES with the paper's upper
 * block-triangular preconditioner P_up = [A11 N_p; 0 S~],
 * S~ = S + dt L - A21 diag(A11)^-1 N_p (Sec. 3.3.1): z2 = S~^-1 y2 by ILU(0)
 * of S~ (nodes coloured greedily, elimination by colour), then
 * A11 z1 = y1 - N_p z2 by GMRES on the operator's tangent system
 * (opts.inner).  Unknowns and residuals are scaled per block (Sec. 3.3.2):
 * the solver works on diag(s_R) J diag(1/s_X); convergence is judged on
 * sqrt(|s_R,m r_m|^2 + |s_R,f r_f|^2).
 *   d_p_n, d_p_o [n]  pressure at the start of the step and the initial one
 *   d_source [n]      fluid source rate per node (m^3/s), or NULL
 *   d_w0 [N]          hydraulic width at zero normal DD (m)
 *   d_dn_start [N]    total normal DD at the start of the step, or NULL (0)
 *   d_dd, d_dpn       in: initial guess; out: the increments
 * Other arguments as hm_newton_step (no inactive elements: HM_EUNSUPPORTED
 * if the operator has a mask).  Synchronises the stream; the operator's
 * tangent is left at the returned state.  HM_ENOTCONV when the tolerance
 * is not met within max_newton iterations.
 */
typedef struct {
    int max_newton;        /* Newton iterations, 0..63; default 25 */
    double rtol, atol;     /* stop when the scaled norm <= max(rtol x first, atol); default 1e-8, 0 */
    double scales[4];      /* s_X mechanics (1/m), s_X flow (1/Pa), s_R mechanics (1/Pa), s_R flow (1/m^3);
                              <= 0: 1 */
    int outer_restart;     /* FGMRES restart, 1..200; default 30 */
    int outer_max_iter;    /* FGMRES iterations per Jacobian solve; default 300 */
    double outer_rtol;     /* relative tolerance of each Jacobian solve (scaled); default 1e-6 */
    hm_solve_opts inner;   /* the A11 solves inside P_up; default: 3x3 block-Jacobi, rtol 1e-4, max_iter 500 */
    int schur;             /* 0 (default): S~ = S + dt L - A21 diag(A11)^-1 N_p, sparse, applied by its ILU(0);
                              1: the paper's second choice, S~ = S + dt L - A21 A~11^-1 N_p with A~11 the ILU(0)
                              of C^ep plus the fraction inner.ilu_fraction of the near field (HM_PC_ILU), applied
                              matrix-free and inverted by GMRES preconditioned with the first choice */
    double schur_rtol;     /* relative tolerance of that GMRES; default 1e-2 */
    int schur_max_iter;    /* its iterations, 1..200 (no restart); default 30 */
} hm_coupled_opts;

typedef struct {
    int iterations;            /* Newton iterations (Jacobian solves) */
    int converged;
    int n_history;             /* residual evaluations */
    double residual[64];       /* scaled residual norm */
    double residual_mech[64];  /* ||r_m|| (Pa) */
    double residual_flow[64];  /* ||r_f|| (m^3) */
    int outer_iterations[64];  /* FGMRES iterations of each Jacobian solve */
    int inner_iterations[64];  /* A11 GMRES iterations summed over that solve's preconditioner applications */
    int64_t modes[5];          /* elements per interface mode at the returned state */
    double ms;
    int schur_iterations[64];  /* schur = 1: S~ GMRES iterations summed over that solve's applications */
} hm_coupled_report;

void hm_coupled_opts_default(hm_coupled_opts* opts);
hm_status hm_coupled_step(hm_op* op, const hm_flow* flow, int n_mat, const hm_interface_material* mats,
                          const int32_t* d_mat_id, const double* d_t, const double* d_dp, const double* d_chi,
                          const double* d_dT0, const double* d_eta_dt, const double* d_dd_prev, const double* d_p_n,
                          const double* d_p_o, const double* d_source, const double* d_w0, const double* d_dn_start,
                          double dt, double* d_dd, double* d_dpn, double* d_t_new, double* d_dp_new,
                          double* d_chi_new, const hm_coupled_opts* opts, hm_coupled_report* rep, void* hip_stream);

/*
 * Scale update of Sec. 3.3.2 (host): L = alpha L_old + (1 - alpha) L_new,
 * then L_old times its ratio to L_old clipped to [rho_min, rho_max] (the
 * paper uses alpha 0.62, rho_min 0.84, rho_max 1.16); the scaling factors
 * are s_X = 1 / (L_rate dt_next) and s_R = 1 / L_residual.  HM_EINVAL when
 * L_old <= 0, L_new < 0, alpha outside [0, 1] or rho_min > 1 > rho_max.
 */
hm_status hm_scale_update(double L_old, double L_new, double alpha, double rho_min, double rho_max, double* out);

/* ------------------------------------------------------------------ */
/* Adaptive time stepping                                               */
/* ------------------------------------------------------------------ */
/*
 * Paper Sec. 3.4 ("Adaptive time-stepping").  The local truncation error of
 * a backward-Euler step is estimated from the change of rate,
 *   e_{n+1} = (dt_n / 2) ||dd_{n+1}/dt_n - dd_n/dt_{n-1}|| / ||d_{n+1}||
 * (dd the DD increments of the two steps, d the total DD after the step;
 * 2-norms over all DOF), and the next step size follows the controller
 *   dt_{n+1} = dt_n (dt_n/dt_{n-1})^(-1/4) (eps/e_{n+1})^(1/4)
 *              (e_n/eps)^(-1/4) (n_its/n_target)^(-1/3),
 * written here as the paper prints it, with sqrt(machine epsilon) added to
 * both errors, the growth limited to dt_{n+1} <= growth_max dt_n and the
 * result kept in [dt_min, dt_max].  Only the DD estimate is built (pore
 * pressures are inputs of hm_newton_step, not unknowns).
 */
typedef struct {
    double eps_tol;     /* target relative truncation error; default 1e-3 */
    int n_target;       /* target Newton iterations per step; default 6 */
    double growth_max;  /* largest dt_{n+1} / dt_n; default 1.2 */
    double dt_min;      /* smallest step; default 0 */
    double dt_max;      /* largest step; default INFINITY */
} hm_timestep_opts;

void hm_timestep_opts_default(hm_timestep_opts* opts);
/* Host only.  dt_n > 0 and n_its >= 1 (else HM_EINVAL); a first step passes
 * dt_prev <= 0 and e_n <= 0, which drops the factors that need them. */
hm_status hm_timestep_next(const hm_timestep_opts* opts, double dt_n, double dt_prev, double e_next, double e_n,
                           int n_its, double* dt_next);
/* e_{n+1} above from device FP64 vectors of length n (d_dd_prev may be NULL
 * for a first step: zero rate); deterministic reduction; synchronises the
 * stream.  dt, dt_prev > 0 (dt_prev ignored when d_dd_prev is NULL). */
hm_status hm_lte_estimate(int64_t n, const double* d_dd, double dt, const double* d_dd_prev, double dt_prev,
                          const double* d_total, double* e, void* hip_stream);

/* ------------------------------------------------------------------ */
/* Learned correction of the block preconditioner                       */
/* ------------------------------------------------------------------ */
/*
 * The inner A11 solves (paper Sec. 3.3.1) use a cheap approximate inverse
 * of A11 as preconditioner; the paper uses point Jacobi.  Here a plain
 * block preconditioner M_base gets a learned linear correction over each
 * element's K nearest elements f (e itself first, exact search, ties by
 * id):
 *     (M^-1 r)_e = (M_base r)_e + sum_f W_ef r_f,   W_ef = (h_e / E') net(phi_ef),
 * with M_base the 3x3 block-Jacobi inverse, (M_base r)_e = B_e r_e,
 * B_e = (E_ee - D_e)^-1 (default), or the leaf block inverses of
 * HM_PC_LEAF (hm_learned_set_base); M_base is also the fallback;
 * net a small MLP (32 -> H -> H -> 9, ReLU, FP32) of 20 dimensionless pair
 * features phi_ef of geometry and tangent stiffness, h_e = sqrt(area_e),
 * E' = E / (1 - nu^2); W_ef = 0 when e or f is inactive.  M^-1 is linear
 * and fixed for a given tangent, so right-preconditioned GMRES applies.
 * Training minimises L = (1/ns) sum_s ||M^-1 b_s - x_s||^2 / ||x_s||^2 over
 * pairs A11 x_s = b_s with Adam (beta 0.9/0.999, eps 1e-8), all on the GPU
 * with the library's own forward/backward kernels; loss, residuals and
 * gradient sums are FP64 in a fixed order (deterministic).
 *
 * Parameter layout (float, count from hm_learned_num_params):
 *   W1 [32][H], b1 [H], W2 [H][H], b2 [H], W3 [H][9], b3 [9],
 *   layer output o = b[o] + sum_k in[k] W[k][o]; output 3a+b = W_ef(a, b).
 * Feature k of pair (e, f), dimensionless (entries 20..31 are 0):
 *   0-2 centroid offset f - e in e's frame (s1, s2, n) / h_e; 3 distance / h_e;
 *   4 n_e.n_f; 5 s1_e.s1_f; 6 s2_e.s2_f; 7-9 diag(D_e) h_e/E';
 *   10-12 diag(D_f) h_f/E'; 13 D_e(s1,n) h_e/E'; 14 D_f(s1,n) h_f/E';
 *   15 D_e(n,s1) h_e/E'; 16 h_f/h_e; 17 [f = e];
 *   18 mean of D_nn h/E' and 19 mean of (D_s1s1 + D_s2s2) h/(2E') over the
 *   active elements of e's cluster-tree leaf.
 * A handle is used by one thread at a time.
 */
typedef struct hm_learned hm_learned;

/* hidden: 16, 32 or 64; neighbors: 1..64 (K); seed: initialisation
 * (Glorot-uniform W1, W2; W3 scaled by 0.01, biases 0, so M^-1 starts
 * next to block-Jacobi). */
hm_status hm_learned_create(int hidden, int neighbors, uint64_t seed, hm_learned** out);
void hm_learned_destroy(hm_learned* net);
hm_status hm_learned_num_params(const hm_learned* net, int64_t* n);
/* The base M_base of the correction: HM_PC_BLOCK3 (default) or HM_PC_LEAF.
 * Training, hm_learned_loss_grad and hm_learned_attach use it, and a solve
 * with the attached correction falls back to it.  Clears the Adam moments. */
hm_status hm_learned_set_base(hm_learned* net, int base);
/* host copies of the parameters; set also clears the Adam moments */
hm_status hm_learned_get_params(const hm_learned* net, float* host_params, int64_t n);
hm_status hm_learned_set_params(hm_learned* net, const float* host_params, int64_t n);

/*
 * Pairs and features of op's current tangent for K neighbours (host
 * outputs).  *n_pairs receives the count (N * min(K, N)); the arrays are
 * written only when cap >= that count (pass cap = 0 to query).
 *   pe, pf [P] int32: element and neighbour (pairs of e are contiguous,
 *   nearest first); feat [P][32] float; scale [P] double (h_e / E', or 0).
 */
hm_status hm_learned_features(hm_op* op, int neighbors, int64_t cap, int64_t* n_pairs, int32_t* pe, int32_t* pf,
                              float* feat, double* scale, void* hip_stream);

/*
 * Loss L and its gradient at the current parameters for ns samples
 * (1..16) of op's current tangent: d_B, d_X [ns][ld] float64 (device),
 * x_s the solution of A11 x_s = b_s.  host_grad [n_params] float receives
 * dL/dtheta; the parameters do not change.  Synchronous.
 */
hm_status hm_learned_loss_grad(hm_learned* net, hm_op* op, int ns, const double* d_B, int64_t ldb,
                               const double* d_X, int64_t ldx, double* loss, float* host_grad, void* hip_stream);

/*
 * steps Adam steps (learning rate lr) on n samples of op's current tangent,
 * `batch` (1..16) samples per step taken cyclically.  host_loss (optional,
 * [steps]) receives the loss before each step.  Detaches op's correction.
 */
hm_status hm_learned_train(hm_learned* net, hm_op* op, int n, const double* d_B, int64_t ldb, const double* d_X,
                           int64_t ldx, int steps, int batch, double lr, double* host_loss, void* hip_stream);

/* Predict the W blocks for op's current tangent and attach them for
 * HM_PC_LEARNED; hm_tangent_set detaches them.  Synchronous. */
hm_status hm_learned_attach(hm_op* op, const hm_learned* net, void* hip_stream);
void hm_learned_detach(hm_op* op);

/* Struct sizes in the order hm_abi_check expects. */
#define HM_ABI_N_STRUCTS 14
#define HM_ABI_SIZES                                                                                   \
    {sizeof(hm_plan_info),       sizeof(hm_build_opts),   sizeof(hm_op_stats),    sizeof(hm_batch_opts), \
     sizeof(hm_batch_info),      sizeof(hm_solve_opts),   sizeof(hm_solve_report),                        \
     sizeof(hm_interface_material), sizeof(hm_newton_opts), sizeof(hm_newton_report),                    \
     sizeof(hm_flow_params),     sizeof(hm_coupled_opts), sizeof(hm_coupled_report),                      \
     sizeof(hm_timestep_opts)}

#ifdef __cplusplus
}
#endif
#endif /* HMDD_H */
