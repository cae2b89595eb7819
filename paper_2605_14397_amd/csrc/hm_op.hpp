// Operator handle: plan, packed H-matrix data per precision variant, and
// the workspaces of apply and solve.
#pragma once

#include <map>
#include <mutex>

#include "hm_internal.hpp"

namespace hm {

// Layout of the workspace of one product of a variant, as one contiguous
// block: in-vector chunks (near precision; far hi/lo when the far field has
// its own precision), T chunks (hi/lo), phase-A partial slots, phase-B
// output rows, and the device table of base pointers the kernels read.
// Sections start on 256-byte boundaries.  The chunk sections (xf_*, tf_*)
// must be zero where no element writes (padding of every leaf section and
// of every rank); the others are written before they are read.
struct WsLayout {
    size_t xn = 0, xfh = 0, xfl = 0, tph = 0, tpl = 0, tpart = 0, y = 0, bases = 0;
    size_t zero_end = 0;   // [0, zero_end) holds every section that must start at zero
    size_t total = 0;
};

// A workspace owned by a stream's pool or by a batch.
struct ApplyWs {
    DevBuf block;
    uint64_t gen = 0;      // task-list generation its sizes and base table were made for
};

// One packed copy of the H-matrix in a given (near, far) precision pair.
// Accumulation is FP64 when near is FP64, FP32 otherwise.
struct Variant {
    int near_prec = HM_F64, far_prec = HM_F64;
    bool self_separate = false;   // element self blocks applied from the FP64 store
    DevBuf near_a, far_a;         // panels
    DevBuf tasksB, itemsB, tasksA, itemsA, membersA, reduce;
    int nTasksB = 0, nTasksA = 0, nReduce = 0;
    XcdSplit splitA{}, splitB{};
    int64_t tpart_elems = 0, tfrag_elems = 0;
    int64_t bytes_near = 0, bytes_far = 0, bytes_far_u = 0, bytes_far_v = 0;
    int64_t near_entries = 0;     // dense-piece entries stored, without padding
    int64_t xel = 0;              // elements of one in-vector buffer (padded dofs x 16 columns)
    uint64_t gen = 1;             // bumped when the task lists are rebuilt (partial slots resize)
    // per-stream workspaces: a product on stream s uses the pool's block of
    // s, allocated and zeroed on the first product on s
    mutable std::mutex ws_mu;
    mutable std::map<hipStream_t, std::unique_ptr<ApplyWs>> ws_pool;
    // host copies of the task lists (merged by batches)
    std::vector<TaskA> hTasksA;
    std::vector<PanelRef> hItemsA;
    std::vector<MemberT> hMembersA;
    std::vector<ReduceDesc> hReduce;
    std::vector<TaskB> hTasksB;
    std::vector<PanelRef> hItemsB;
    int leavesPerTaskA = 8;
    int stackRowsA = 64;                        // row cap of a stacked V^T panel set (-1: none)
    int windowB = kTileWindowB;                 // row tiles per phase-B task window
    int maxNtB = kTileWindowB;                  // tallest window in hTasksB
    std::vector<TaskB> sectionsB;               // one per (target leaf, section): its rows and items (r0 = 0)
    // factorisations with one source cluster and one section set: their
    // V^T sub-panels are stacked (phase-A items)
    struct VGroup {
        int K = 0;                    // stacked rows (sum of the members' ranks)
        std::vector<int> blocks;      // member factorisations
        std::vector<int> lo;          // first stacked row of each member
        std::vector<PanelRef> items;  // one stacked sub-panel per (source leaf, section)
    };
    std::vector<VGroup> vgroups;
    std::vector<int64_t> t_off;                 // per block: T chunk offset
    bool acc_f64() const { return near_prec == HM_F64; }
    bool far_is_near() const { return far_prec == near_prec; }
    WsLayout ws_layout() const;
    Bases host_bases(void* block) const;
    // the workspace of stream s (created on first use; resized and its base
    // table rewritten after the task lists changed); returns the block base
    void* workspace(hipStream_t s) const;
    // a workspace owned by the caller (batches), zeroed and with its table
    std::unique_ptr<ApplyWs> new_workspace(hipStream_t s) const;
    // zero the chunk sections of a block and write its base table (kernels
    // only: usable on memory the library did not allocate)
    void prepare_block(void* block, hipStream_t s) const;
};

// Everything one product launches: task lists (single operator or merged).
// bases points at the device table of base pointers (one entry per operator).
struct LaunchSet {
    int near_prec = HM_F64, far_prec = HM_F64;
    const Bases* bases = nullptr;
    const TaskA* tasksA = nullptr;
    int nTasksA = 0;
    const PanelRef* itemsA = nullptr;
    const MemberT* membersA = nullptr;
    const ReduceDesc* reduce = nullptr;
    int nReduce = 0;
    const TaskB* tasksB = nullptr;
    int nTasksB = 0;
    XcdSplit splitA{}, splitB{};
    const PanelRef* itemsB = nullptr;
    int* queue = nullptr;   // kQueueInts claim counters: queue-driven phase launches (batches)
    int maxNtB = kTileWindowB;  // tallest phase-B window of the task list (row tiles)
};

// One low-rank factorisation U V^T of the components comp0 .. comp0 + comps - 1
// of every element of a block: comps = 3 for a coupled block, 2 (shear) and
// 1 (normal) for the two parts of a coplanar one.
struct LowRank {
    int t_node = 0, s_node = 0;
    int64_t m = 0, n = 0;       // elements
    int rank = 0;
    int comps = 3, comp0 = 0;
    int64_t u_off = 0, v_off = 0;  // compact FP64 factors: U [rank][comps m], V [rank][comps n]
};

// Learned correction of the block preconditioner: network parameters and
// Adam moments (FP32, device), see hm_learned.hip for the layout.
struct Learned {
    int H = 64, K = 8;      // hidden width, neighbours per element (self included)
    int base = HM_PC_BLOCK3;  // preconditioner the correction is added to (HM_PC_BLOCK3 or HM_PC_LEAF)
    int64_t n = 0;          // parameter count
    int64_t step = 0;       // Adam steps taken
    DevBuf params, m, v, grad;
    DevBuf ws;              // training workspace (activations, residuals, partial sums)
    Learned(int hidden, int neighbors, uint64_t seed);
    void reset_moments();
};

// Per-operator pairs (element e, neighbour f), their features for the
// current tangent, and the predicted 3x3 blocks W_ef (FP32).
struct LearnedPairs {
    int K = 0;              // neighbours the pair list was built for (0: none)
    int64_t P = 0;
    DevBuf pe, pf, off;     // int32 [P], int32 [P], int64 [N + 1] (pairs of e are off[e] .. off[e+1])
    DevBuf feat, scale;     // float [P][32], double [P] (h_e / E', 0 when e or f is inactive)
    bool features_current = false;
    DevBuf W;               // float [P][9]
    bool attached = false;
    int base = HM_PC_BLOCK3;  // base preconditioner of the attached correction
};

// The ILU(0) preconditioner of the sparse approximation of A11 (hm_ilu.hip):
// CSR rows in the original DOF numbering, each row's entries in
// elimination order (elements by colour then id), factors in place.
struct IluPc {
    double fraction = -1.0;           // p the structure was built for
    bool structure = false;           // selection, pattern and order valid for (fraction, mask_key)
    uint64_t mask_key = 0;            // hash of the active mask the structure was built for
    bool current = false;             // factors valid for the current tangent
    int n_colors = 0;
    std::vector<int64_t> color_begin; // offsets of each colour in `order`
    DevBuf order;                     // int32 [N]: elements by (colour, id)
    DevBuf pos;                       // int32 [N]: each element's place in that order
    DevBuf rowptr, col, diag, val;    // int64 [3N+1], int32 [nnz], int64 [3N], double [nnz] (factors)
    DevBuf val0;                      // double [nnz]: E's kept entries (identity rows of inactive elements)
    DevBuf dpos;                      // int64 [9N]: position of each diagonal-block entry in val (-1: none)
    int64_t nnz = 0, n_kept = 0, near_entries = 0;
    uint64_t threshold_key = 0;
    double setup_ms = 0.0;
};

enum { kWsKrylov = 0, kWsIlu = 1 };

struct Op {
    int device = 0;
    double young = 0, nu = 0, G = 0;
    int64_t ne = 0;
    Plan plan;
    std::vector<int64_t> leaf_xoff;   // padded dof offset of each leaf chunk
    int64_t xtot = 0;                 // total padded dofs
    std::vector<LowRank> lr;
    // element tables in original order
    DevBuf d_leaf_io;                 // LeafIo [leaves]: chunk offset, first cluster position, size
    DevBuf d_self;                    // double [N][9]: FP64 self blocks (original order)
    Variant main;
    std::unique_ptr<Variant> ref;     // FP64 copy when main is not FP64
    // tangent
    bool has_D = false, has_mask = false;
    DevBuf d_D, d_mask, d_pc_block, d_pc_diag;
    // leaf block-Jacobi preconditioner: element geometry and permutation in
    // cluster order (kept to recompute the diagonal leaf coefficients), leaf
    // descriptors, and the FP64 inverses (column-major, built on first use
    // after each tangent change)
    DevBuf d_geo, d_perm, d_leaf_desc, d_leaf_inv;
    int64_t leaf_inv_elems = 0;
    bool leaf_pc_current = false;
    IluPc ilu;
    // element geometry kept for the learned preconditioner (original order)
    std::vector<double> e_cent, e_frame, e_h;  // [N][3], [N][9], [N] (sqrt of area)
    LearnedPairs lp;
    // solver workspaces, one per (stream, purpose), allocated on first use:
    // kWsKrylov for GMRES, kWsIlu for the ILU substitutions
    std::mutex solve_mu;
    std::map<std::pair<hipStream_t, int>, std::unique_ptr<DevBuf>> solve_ws;
    double* solve_workspace(hipStream_t s, size_t bytes, int purpose = 0);
    // serialises the lazy preconditioner set-up of concurrent solves
    std::mutex pc_mu;
    hm_op_stats stats{};
    const Variant& ref_variant() const { return ref ? *ref : main; }
};

// build helpers (hm_build.hip)
void build_operator(Op& op, const Mesh& mesh, const hm_build_opts& o, hipStream_t s);
void kernel_block(Mesh& mesh, double young, double nu, int64_t nr, const int64_t* d_rows, int64_t nc,
                  const int64_t* d_cols, double* d_out, hipStream_t s);
void ensure_mesh_geo(Mesh& mesh);

// E on every diagonal leaf block, row-major [3m][3m] at each leaf's offset (hm_build.hip)
void leaf_blocks_coef(const Op& op, double* out, hipStream_t s);

// G, G / (4 pi), G / (4 pi (1 - nu)) from Young's modulus and Poisson's ratio
void moduli(double young, double nu, double& G, double& kG, double& kN);

// ILU(0) of the sparse approximation of A11 (hm_ilu.hip)
void ilu_pc_prepare(Op& op, double fraction, hipStream_t s);
void ilu_pc_apply(Op& op, int nrhs, const double* r, int64_t ldr, double* z, int64_t ldz, hipStream_t s);

// leaf block-Jacobi preconditioner (hm_leafpc.hip)
void leaf_pc_prepare(Op& op, hipStream_t s);
void leaf_pc_apply(const Op& op, int nrhs, const double* r, int64_t ldr, double* z, int64_t ldz, hipStream_t s);

// apply (hm_apply.hip)
// ev (optional): 6 events recorded before, between and after the 5 stages
void apply(const Op& op, const Variant& v, int nrhs, const double* d_X, int64_t ldx, double* d_Y, int64_t ldy,
           bool tangent, hipStream_t s, hipEvent_t* ev = nullptr, bool accumulate = false);
// the same product in a workspace block supplied by the caller (ws_layout()
// bytes at least, 256-byte aligned); zeroes its chunk sections first
void apply_in(const Op& op, const Variant& v, void* block, int nrhs, const double* d_X, int64_t ldx, double* d_Y,
              int64_t ldy, bool tangent, hipStream_t s, bool accumulate);
LaunchSet launch_set(const Variant& v, void* block);
Segment make_segment(const Op& op, const Variant& v, const double* X, int64_t ldx, double* Y, int64_t ldy,
                     bool tangent, int op_index, bool accumulate = false);
// gather (one segment per operator, segs on the device when nseg > 1), phases, scatter
void launch_product(const LaunchSet& L, int nrhs, const Segment* segs_dev, const Segment* seg_host, int nseg,
                    int64_t total_leaves, hipStream_t s, hipEvent_t* ev);
// (re)build the phase-A task list of a variant with a given task size
void build_tasksA(const Op& op, Variant& v, int leaves_per_task);
// phase-A wavefronts resident at once on the current device for a form
int phaseA_resident_waves(int near_prec, int far_prec);
// phase-B tasks: windows of `window` row tiles (1 .. kTileWindowB) over each section
void build_tasksB(Variant& v, int window);
// Order a phase-A task list for launch: grouped by row-tile count (one
// launch per group, largest first); inside a group ordered by the in-vector
// chunk of the first sub-panel, then longest first inside each XCD's share.
// sort phase-A tasks for one launch (by operator and source chunk, then XCD
// ranges of equal load, longest first inside each when asked) and return
// the ranges
XcdSplit order_tasksA(std::vector<TaskA>& ta, const std::vector<PanelRef>& items, bool longest_first);
// the same for phase-B tasks (leaf order, then XCD ranges of equal load)
XcdSplit order_tasksB(std::vector<TaskB>& tb, const std::vector<PanelRef>& items, int near_prec, int far_prec,
                      bool longest_first);
void upload_tasks(Variant& v, hipStream_t s);
void tangent_set(Op& op, const double* d_D, const uint8_t* d_mask, hipStream_t s);
void interface_update(int n_mat, const hm_interface_material* mats, int64_t n, const int32_t* d_mat_id,
                      const double* d_dd, const double* d_t, const double* d_dp, const double* d_chi, double* d_t_new,
                      double* d_dp_new, double* d_chi_new, double* d_cep, int32_t* d_mode, const double* d_eta_dt,
                      double* d_D, hipStream_t s);

hm_status newton_step(Op& op, int n_mat, const hm_interface_material* mats, const int32_t* d_mat_id,
                      const double* d_t, const double* d_dp, const double* d_chi, const double* d_dT0,
                      const double* d_dpress, const double* d_eta_dt, const double* d_dd_prev, double* d_dd,
                      double* d_t_new, double* d_dp_new, double* d_chi_new, const hm_newton_opts& o,
                      hm_newton_report* rep, hipStream_t s);

double lte_estimate(int64_t n, const double* d_dd, double dt, const double* d_dd_prev, double dt_prev,
                    const double* d_total, hipStream_t s);

// solve (hm_solve.hip)
hm_status solve(Op& op, const hm_solve_opts& o, int nrhs, const double* d_B, int64_t ldb, double* d_X,
                int64_t ldx, hm_solve_report* rep, hipStream_t s);
void precond_apply(Op& op, int kind, int nrhs, const double* R, int64_t ldr, double* Z, int64_t ldz, hipStream_t s);

// learned preconditioner (hm_learned.hip)
void learned_prepare(Op& op, int K, hipStream_t s);
double learned_loss_grad(Learned& L, Op& op, int ns, const double* B, int64_t ldb, const double* X, int64_t ldx,
                         hipStream_t s);
void learned_train(Learned& L, Op& op, int n, const double* B, int64_t ldb, const double* X, int64_t ldx, int steps,
                   int batch, double lr, double* hist, hipStream_t s);
void learned_attach(Op& op, const Learned& L, hipStream_t s);
void learned_apply(const Op& op, int nrhs, const double* r, int64_t ldr, double* z, int64_t ldz, hipStream_t s);

// flow in the discontinuities and the coupled step (hm_flow.hip)
struct Flow;
Flow* flow_create(const Mesh& m, const hm_flow_params& p, hipStream_t s);
void flow_destroy(Flow* f);
int64_t flow_num_nodes(const Flow& f);
int64_t flow_nnz(const Flow& f);
void flow_matrices(const Flow& F, const double* d_w, int64_t* rowptr, int32_t* col, double* S, double* L,
                   hipStream_t s);
hm_status coupled_step(Op& op, const Flow& F, int n_mat, const hm_interface_material* mats, const int32_t* d_mat_id,
                       const double* d_t, const double* d_dp, const double* d_chi, const double* d_dT0,
                       const double* d_eta_dt, const double* d_dd_prev, const double* d_p_n, const double* d_p_o,
                       const double* d_source, const double* d_w0, const double* d_dn_start, double dt, double* d_dd,
                       double* d_dpn, double* d_t_new, double* d_dp_new, double* d_chi_new, const hm_coupled_opts& o,
                       hm_coupled_report* rep, hipStream_t s);
double scale_update(double L_old, double L_new, double alpha, double rho_min, double rho_max);

// batches (hm_batch.cpp)
struct Batch;
Batch* batch_create(const std::vector<Op*>& ops, const hm_batch_opts& o, hipStream_t s);
void batch_apply(Batch& b, int nrhs, const double* const* X, const int64_t* ldx, double* const* Y, const int64_t* ldy,
                 hipStream_t s);
void batch_info(const Batch& b, hm_batch_info* out);
void batch_destroy(Batch* b);

}  // namespace hm
