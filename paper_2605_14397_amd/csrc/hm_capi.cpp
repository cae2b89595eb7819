// extern "C" boundary of the hmdd library: argument checks, error codes,
// thread-local messages.  No C++ exception crosses these functions.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>

#include "hm_handles.hpp"

namespace hm {
static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace hm

static void require_gfx950()
{
    int dev = 0;
    HM_CHECK_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HM_CHECK_HIP(hipGetDeviceProperties(&prop, dev));
    HM_REQUIRE(std::string(prop.gcnArchName).find("gfx950") != std::string::npos, HM_EDEVICE,
               std::string("device is ") + prop.gcnArchName + ", the library is built for gfx950 only");
}

extern "C" {

const char* hm_last_error(void) { return hm::g_last_error.c_str(); }

const char* hm_version(void) { return "hmdd 0.1 (gfx950)"; }

hm_status hm_abi_check(int n, const size_t* sizes)
{
    return guarded([&] {
        static const size_t mine[] = HM_ABI_SIZES;
        static const char* names[] = {"hm_plan_info",   "hm_build_opts",          "hm_op_stats",
                                      "hm_batch_opts",  "hm_batch_info",          "hm_solve_opts",
                                      "hm_solve_report", "hm_interface_material", "hm_newton_opts",
                                      "hm_newton_report", "hm_flow_params",       "hm_coupled_opts",
                                      "hm_coupled_report", "hm_timestep_opts"};
        static_assert(sizeof(mine) / sizeof(mine[0]) == HM_ABI_N_STRUCTS, "HM_ABI_SIZES length");
        static_assert(sizeof(names) / sizeof(names[0]) == HM_ABI_N_STRUCTS, "struct name table length");
        HM_REQUIRE(sizes, HM_EINVAL, "sizes is null");
        HM_REQUIRE(n == HM_ABI_N_STRUCTS, HM_EINVAL,
                   "caller lists " + std::to_string(n) + " structs, the library " +
                       std::to_string(HM_ABI_N_STRUCTS) + ": header and library differ");
        for (int i = 0; i < n; ++i)
            HM_REQUIRE(sizes[i] == mine[i], HM_EINVAL,
                       std::string(names[i]) + " is " + std::to_string(sizes[i]) + " bytes in the caller, " +
                           std::to_string(mine[i]) + " in the library: rebuild against this header");
    });
}

hm_status hm_mesh_create(int nv_per_elem, int64_t n_vert, const double* xyz, int64_t n_elem, const int64_t* conn,
                         hm_mesh** out)
{
    return guarded([&] {
        HM_REQUIRE(out, HM_EINVAL, "out is null");
        *out = nullptr;
        HM_REQUIRE(xyz && conn, HM_EINVAL, "xyz or conn is null");
        HM_REQUIRE(n_vert > 0 && n_elem > 0, HM_EINVAL, "empty mesh");
        HM_REQUIRE(nv_per_elem == 3 || nv_per_elem == 4, HM_EINVAL, "nv_per_elem must be 3 or 4");
        std::unique_ptr<hm_mesh> h(new hm_mesh());
        h->m.nvpe = nv_per_elem;
        h->m.nv = n_vert;
        h->m.ne = n_elem;
        h->m.xyz.assign(xyz, xyz + 3 * n_vert);
        h->m.conn.assign(conn, conn + nv_per_elem * n_elem);
        hm::mesh_validate_and_frame(h->m);
        *out = h.release();
    });
}

void hm_mesh_destroy(hm_mesh* mesh) { delete mesh; }

int64_t hm_mesh_num_elements(const hm_mesh* mesh) { return mesh ? mesh->m.ne : 0; }

hm_status hm_mesh_frames(const hm_mesh* mesh, double* centroid, double* frame, double* area)
{
    return guarded([&] {
        HM_REQUIRE(mesh, HM_EINVAL, "mesh is null");
        const hm::Mesh& m = mesh->m;
        if (centroid) std::memcpy(centroid, m.cent.data(), sizeof(double) * 3 * m.ne);
        if (frame) std::memcpy(frame, m.frame.data(), sizeof(double) * 9 * m.ne);
        if (area) std::memcpy(area, m.area.data(), sizeof(double) * m.ne);
    });
}

hm_status hm_plan_summary(const hm_mesh* mesh, int leaf_size, double eta, hm_plan_info* info, int64_t* perm)
{
    return guarded([&] {
        HM_REQUIRE(mesh && info, HM_EINVAL, "null argument");
        hm::Plan p = hm::make_plan(mesh->m, leaf_size, eta);
        std::memset(info, 0, sizeof(*info));
        info->n_leaves = (int64_t)p.leaves.size();
        info->n_dense_blocks = (int64_t)p.dense.size();
        info->n_lowrank_blocks = (int64_t)p.lowrank.size();
        info->depth = p.depth;
        for (const auto& d : p.dense)
            info->dense_entries += 9 * p.nodes[d.first].size() * p.nodes[d.second].size();
        for (const auto& l : p.lowrank) {
            int lev = p.nodes[l.first].level;
            if (lev < 64) info->lowrank_by_level[lev]++;
            info->lowrank_sum_mn += p.nodes[l.first].size() + p.nodes[l.second].size();
        }
        int64_t mx = 0, mn = INT64_MAX;
        for (int id : p.leaves) {
            mx = std::max(mx, p.nodes[id].size());
            mn = std::min(mn, p.nodes[id].size());
        }
        info->max_leaf = mx;
        info->min_leaf = mn;
        if (perm) std::memcpy(perm, p.perm.data(), sizeof(int64_t) * p.perm.size());
    });
}

hm_status hm_kernel_block(const hm_mesh* mesh, double young, double nu, int64_t nr, const int64_t* d_rows, int64_t nc,
                          const int64_t* d_cols, double* d_out, void* hip_stream)
{
    return guarded([&] {
        HM_REQUIRE(mesh, HM_EINVAL, "mesh is null");
        require_gfx950();
        hm::kernel_block(const_cast<hm::Mesh&>(mesh->m), young, nu, nr, d_rows, nc, d_cols, d_out,
                         (hipStream_t)hip_stream);
    });
}

void hm_build_opts_default(hm_build_opts* o)
{
    if (!o) return;
    o->leaf_size = 64;
    o->eta = 2.0;
    o->aca_tol = 1e-6;
    o->max_rank = 128;
    o->near_prec = HM_F64;
    o->far_prec = HM_F64;
    o->keep_f64_reference = 0;
    o->recompress = 1;
    o->stack_rows = 0;
    o->phase_a_items = 0;
    o->phase_b_window = 0;
}

hm_status hm_operator_build(const hm_mesh* mesh, double young, double nu, const hm_build_opts* opts, void* hip_stream,
                            hm_op** out)
{
    return guarded([&] {
        HM_REQUIRE(out, HM_EINVAL, "out is null");
        *out = nullptr;
        HM_REQUIRE(mesh, HM_EINVAL, "mesh is null");
        hm_build_opts o;
        hm_build_opts_default(&o);
        if (opts) o = *opts;
        require_gfx950();
        std::unique_ptr<hm_op> h(new hm_op());
        h->op.young = young;
        h->op.nu = nu;
        hipStream_t s = (hipStream_t)hip_stream;
        hm::build_operator(h->op, mesh->m, o, s);
        hm::tangent_set(h->op, nullptr, nullptr, s);
        HM_CHECK_HIP(hipStreamSynchronize(s));
        *out = h.release();
    });
}

void hm_op_destroy(hm_op* op) { delete op; }

hm_status hm_operator_stats(const hm_op* op, hm_op_stats* out)
{
    return guarded([&] {
        HM_REQUIRE(op && out, HM_EINVAL, "null argument");
        *out = op->op.stats;
        const hm::Variant& v = op->op.main;
        out->apply_workspace_bytes = (int64_t)v.ws_layout().total;
        out->phase_a_tasks = v.nTasksA;
        out->phase_b_tasks = v.nTasksB;
        out->phase_a_stacks = (int64_t)v.vgroups.size();
        out->phase_a_partial_bytes = v.tpart_elems * (v.acc_f64() ? 8 : 4);
    });
}

hm_status hm_operator_apply(const hm_op* op, int nrhs, const double* d_X, int64_t ldx, double* d_Y, int64_t ldy,
                            unsigned flags, void* hip_stream)
{
    return guarded([&] {
        HM_REQUIRE(op, HM_EINVAL, "op is null");
        HM_REQUIRE((flags & ~(HM_APPLY_REFERENCE | HM_APPLY_TANGENT | HM_APPLY_ACCUMULATE)) == 0, HM_EINVAL,
                   "unknown flag");
        const hm::Op& o = op->op;
        HM_REQUIRE(!(flags & HM_APPLY_REFERENCE) || o.ref || o.main.near_prec == HM_F64, HM_EINVAL,
                   "no FP64 reference copy (build with keep_f64_reference)");
        const hm::Variant& v = (flags & HM_APPLY_REFERENCE) ? o.ref_variant() : o.main;
        hm::apply(o, v, nrhs, d_X, ldx, d_Y, ldy, (flags & HM_APPLY_TANGENT) != 0, (hipStream_t)hip_stream, nullptr,
                  (flags & HM_APPLY_ACCUMULATE) != 0);
    });
}

hm_status hm_operator_apply_timed(const hm_op* op, int nrhs, const double* d_X, int64_t ldx, double* d_Y,
                                  int64_t ldy, unsigned flags, void* hip_stream, double* stage_ms)
{
    return guarded([&] {
        HM_REQUIRE(op && stage_ms, HM_EINVAL, "null argument");
        HM_REQUIRE((flags & ~(HM_APPLY_REFERENCE | HM_APPLY_TANGENT | HM_APPLY_ACCUMULATE)) == 0, HM_EINVAL,
                   "unknown flag");
        const hm::Op& o = op->op;
        HM_REQUIRE(!(flags & HM_APPLY_REFERENCE) || o.ref || o.main.near_prec == HM_F64, HM_EINVAL,
                   "no FP64 reference copy (build with keep_f64_reference)");
        const hm::Variant& v = (flags & HM_APPLY_REFERENCE) ? o.ref_variant() : o.main;
        hipStream_t s = (hipStream_t)hip_stream;
        hipEvent_t ev[6] = {};
        struct Events {
            hipEvent_t* e;
            ~Events()
            {
                for (int i = 0; i < 6; ++i)
                    if (e[i]) (void)hipEventDestroy(e[i]);
            }
        } guard{ev};
        for (int i = 0; i < 6; ++i) HM_CHECK_HIP(hipEventCreate(&ev[i]));
        hm::apply(o, v, nrhs, d_X, ldx, d_Y, ldy, (flags & HM_APPLY_TANGENT) != 0, s, ev,
                  (flags & HM_APPLY_ACCUMULATE) != 0);
        HM_CHECK_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < 5; ++i) {
            float ms = 0.f;
            HM_CHECK_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
            stage_ms[i] = ms;
        }
    });
}

hm_status hm_tangent_set(hm_op* op, const double* d_D, const uint8_t* d_mask, void* hip_stream)
{
    return guarded([&] {
        HM_REQUIRE(op, HM_EINVAL, "op is null");
        hm::tangent_set(op->op, d_D, d_mask, (hipStream_t)hip_stream);
    });
}

hm_status hm_flow_create(const hm_mesh* mesh, const hm_flow_params* params, void* hip_stream, hm_flow** out)
{
    return guarded([&] {
        HM_REQUIRE(out, HM_EINVAL, "out is null");
        *out = nullptr;
        HM_REQUIRE(mesh && params, HM_EINVAL, "null argument");
        require_gfx950();
        std::unique_ptr<hm_flow> h(new hm_flow());
        h->f = hm::flow_create(mesh->m, *params, (hipStream_t)hip_stream);
        *out = h.release();
    });
}

void hm_flow_destroy(hm_flow* flow) { delete flow; }
int64_t hm_flow_num_nodes(const hm_flow* flow) { return flow ? hm::flow_num_nodes(*flow->f) : 0; }
int64_t hm_flow_nnz(const hm_flow* flow) { return flow ? hm::flow_nnz(*flow->f) : 0; }

hm_status hm_flow_matrices(const hm_flow* flow, const double* d_w, int64_t* rowptr, int32_t* col, double* S,
                           double* L, void* hip_stream)
{
    return guarded([&] {
        HM_REQUIRE(flow && d_w, HM_EINVAL, "null argument");
        hm::flow_matrices(*flow->f, d_w, rowptr, col, S, L, (hipStream_t)hip_stream);
    });
}

void hm_coupled_opts_default(hm_coupled_opts* o)
{
    if (!o) return;
    o->max_newton = 25;
    o->rtol = 1e-8;
    o->atol = 0.0;
    for (int k = 0; k < 4; ++k) o->scales[k] = 1.0;
    o->outer_restart = 30;
    o->outer_max_iter = 300;
    o->outer_rtol = 1e-6;
    hm_solve_opts_default(&o->inner);
    o->inner.rtol = 1e-4;
    o->inner.max_iter = 500;
    o->schur = 0;
    o->schur_rtol = 1e-2;
    o->schur_max_iter = 30;
}

hm_status hm_coupled_step(hm_op* op, const hm_flow* flow, int n_mat, const hm_interface_material* mats,
                          const int32_t* d_mat_id, const double* d_t, const double* d_dp, const double* d_chi,
                          const double* d_dT0, const double* d_eta_dt, const double* d_dd_prev, const double* d_p_n,
                          const double* d_p_o, const double* d_source, const double* d_w0, const double* d_dn_start,
                          double dt, double* d_dd, double* d_dpn, double* d_t_new, double* d_dp_new,
                          double* d_chi_new, const hm_coupled_opts* opts, hm_coupled_report* rep, void* hip_stream)
{
    hm_status st = HM_OK;
    hm_status g = guarded([&] {
        HM_REQUIRE(op && flow, HM_EINVAL, "null operator or flow problem");
        hm_coupled_opts o;
        hm_coupled_opts_default(&o);
        if (opts) o = *opts;
        st = hm::coupled_step(op->op, *flow->f, n_mat, mats, d_mat_id, d_t, d_dp, d_chi, d_dT0, d_eta_dt, d_dd_prev,
                              d_p_n, d_p_o, d_source, d_w0, d_dn_start, dt, d_dd, d_dpn, d_t_new, d_dp_new, d_chi_new,
                              o, rep, (hipStream_t)hip_stream);
        if (st == HM_ENOTCONV) hm::set_last_error("the coupled Newton iteration did not reach rtol");
    });
    return g != HM_OK ? g : st;
}

hm_status hm_scale_update(double L_old, double L_new, double alpha, double rho_min, double rho_max, double* out)
{
    return guarded([&] {
        HM_REQUIRE(out, HM_EINVAL, "out is null");
        *out = hm::scale_update(L_old, L_new, alpha, rho_min, rho_max);
    });
}

void hm_batch_opts_default(hm_batch_opts* o)
{
    if (!o) return;
    o->use_graph = 1;
    o->autotune = 1;
}

hm_status hm_batch_create(int n_ops, hm_op* const* ops, const hm_batch_opts* opts, void* hip_stream, hm_batch** out)
{
    return guarded([&] {
        HM_REQUIRE(out, HM_EINVAL, "out is null");
        *out = nullptr;
        HM_REQUIRE(n_ops >= 1 && ops, HM_EINVAL, "no operators");
        hm_batch_opts o;
        hm_batch_opts_default(&o);
        if (opts) o = *opts;
        std::vector<hm::Op*> v;
        for (int i = 0; i < n_ops; ++i) {
            HM_REQUIRE(ops[i], HM_EINVAL, "null operator " + std::to_string(i));
            v.push_back(&ops[i]->op);
        }
        std::unique_ptr<hm_batch> h(new hm_batch());
        h->b = hm::batch_create(v, o, (hipStream_t)hip_stream);
        *out = h.release();
    });
}

hm_status hm_batch_apply(hm_batch* batch, int nrhs, const double* const* d_X, const int64_t* ldx, double* const* d_Y,
                         const int64_t* ldy, void* hip_stream)
{
    return guarded([&] {
        HM_REQUIRE(batch && batch->b, HM_EINVAL, "batch is null");
        hm::batch_apply(*batch->b, nrhs, d_X, ldx, d_Y, ldy, (hipStream_t)hip_stream);
    });
}

hm_status hm_batch_get_info(const hm_batch* batch, hm_batch_info* out)
{
    return guarded([&] {
        HM_REQUIRE(batch && batch->b && out, HM_EINVAL, "null argument");
        hm::batch_info(*batch->b, out);
    });
}

void hm_batch_destroy(hm_batch* batch) { delete batch; }

void hm_solve_opts_default(hm_solve_opts* o)
{
    if (!o) return;
    o->restart = 50;
    o->max_iter = 1000;
    o->rtol = 1e-8;
    o->precond = HM_PC_BLOCK3;
    o->refine = 0;
    o->inner_rtol = 0.0;
    o->max_refine = 20;
    o->ilu_fraction = 0.01;
}

hm_status hm_solve(const hm_op* op, const hm_solve_opts* opts, int nrhs, const double* d_B, int64_t ldb, double* d_X,
                   int64_t ldx, hm_solve_report* rep, void* hip_stream)
{
    hm_status st = HM_OK;
    hm_status g = guarded([&] {
        HM_REQUIRE(op, HM_EINVAL, "op is null");
        hm_solve_opts o;
        hm_solve_opts_default(&o);
        if (opts) o = *opts;
        st = hm::solve(const_cast<hm::Op&>(op->op), o, nrhs, d_B, ldb, d_X, ldx, rep, (hipStream_t)hip_stream);
        if (st == HM_ENOTCONV) hm::set_last_error("GMRES did not reach rtol (best iterate returned)");
    });
    return g != HM_OK ? g : st;
}

hm_status hm_precond_apply(const hm_op* op, int precond, int nrhs, const double* d_R, int64_t ldr, double* d_Z,
                           int64_t ldz, void* hip_stream)
{
    return guarded([&] {
        HM_REQUIRE(op, HM_EINVAL, "op is null");
        // the leaf preconditioner caches its inverses in the operator (as hm_solve's workspaces)
        hm::precond_apply(const_cast<hm::Op&>(op->op), precond, nrhs, d_R, ldr, d_Z, ldz, (hipStream_t)hip_stream);
    });
}

hm_status hm_interface_update(int n_mat, const hm_interface_material* mats, int64_t n_elem, const int32_t* d_mat_id,
                              const double* d_ddelta, const double* d_t, const double* d_dp, const double* d_chi,
                              double* d_t_new, double* d_dp_new, double* d_chi_new, double* d_cep, int32_t* d_mode,
                              const double* d_eta_dt, double* d_D, void* hip_stream)
{
    return guarded([&] {
        require_gfx950();
        hm::interface_update(n_mat, mats, n_elem, d_mat_id, d_ddelta, d_t, d_dp, d_chi, d_t_new, d_dp_new, d_chi_new,
                             d_cep, d_mode, d_eta_dt, d_D, (hipStream_t)hip_stream);
    });
}

void hm_newton_opts_default(hm_newton_opts* o)
{
    if (!o) return;
    o->max_newton = 25;
    o->rtol = 1e-10;
    o->atol = 0.0;
    hm_solve_opts_default(&o->lin);
    o->lin.rtol = 1e-10;
    o->lin.max_iter = 3000;
    o->forcing = 0;
}

hm_status hm_newton_step(hm_op* op, int n_mat, const hm_interface_material* mats, const int32_t* d_mat_id,
                         const double* d_t, const double* d_dp, const double* d_chi, const double* d_dT0,
                         const double* d_dpress, const double* d_eta_dt, const double* d_dd_prev, double* d_dd,
                         double* d_t_new, double* d_dp_new, double* d_chi_new, const hm_newton_opts* opts,
                         hm_newton_report* rep, void* hip_stream)
{
    hm_status st = HM_OK;
    const hm_status g = guarded([&] {
        HM_REQUIRE(op, HM_EINVAL, "op is null");
        require_gfx950();
        hm_newton_opts o;
        hm_newton_opts_default(&o);
        if (opts) o = *opts;
        st = hm::newton_step(op->op, n_mat, mats, d_mat_id, d_t, d_dp, d_chi, d_dT0, d_dpress, d_eta_dt, d_dd_prev,
                             d_dd, d_t_new, d_dp_new, d_chi_new, o, rep, (hipStream_t)hip_stream);
        if (st == HM_ENOTCONV) hm::set_last_error("Newton did not reach the residual tolerance (last iterate returned)");
    });
    return g != HM_OK ? g : st;
}

void hm_timestep_opts_default(hm_timestep_opts* o)
{
    if (!o) return;
    o->eps_tol = 1e-3;
    o->n_target = 6;
    o->growth_max = 1.2;
    o->dt_min = 0.0;
    o->dt_max = INFINITY;
}

hm_status hm_timestep_next(const hm_timestep_opts* opts, double dt_n, double dt_prev, double e_next, double e_n,
                           int n_its, double* dt_next)
{
    return guarded([&] {
        HM_REQUIRE(dt_next, HM_EINVAL, "dt_next is null");
        HM_REQUIRE(dt_n > 0.0 && n_its >= 1, HM_EINVAL, "need dt_n > 0 and n_its >= 1");
        hm_timestep_opts o;
        hm_timestep_opts_default(&o);
        if (opts) o = *opts;
        HM_REQUIRE(o.eps_tol > 0.0 && o.n_target >= 1 && o.growth_max > 0.0 && o.dt_min >= 0.0 &&
                       o.dt_max >= o.dt_min,
                   HM_EINVAL, "invalid controller options");
        const double floor_e = std::sqrt(2.220446049250313e-16);   // sqrt of the FP64 unit roundoff
        double dt = dt_n;
        if (dt_prev > 0.0) dt *= std::pow(dt_n / dt_prev, -0.25);
        dt *= std::pow(o.eps_tol / (std::max(e_next, 0.0) + floor_e), 0.25);
        if (e_n > 0.0) dt *= std::pow((e_n + floor_e) / o.eps_tol, -0.25);
        dt *= std::pow((double)n_its / o.n_target, -1.0 / 3.0);
        dt = std::min(dt, o.growth_max * dt_n);
        *dt_next = std::max(o.dt_min, std::min(dt, o.dt_max));
    });
}

hm_status hm_lte_estimate(int64_t n, const double* d_dd, double dt, const double* d_dd_prev, double dt_prev,
                          const double* d_total, double* e, void* hip_stream)
{
    return guarded([&] {
        HM_REQUIRE(e, HM_EINVAL, "e is null");
        require_gfx950();
        *e = hm::lte_estimate(n, d_dd, dt, d_dd_prev, dt_prev, d_total, (hipStream_t)hip_stream);
    });
}

hm_status hm_learned_create(int hidden, int neighbors, uint64_t seed, hm_learned** out)
{
    return guarded([&] {
        HM_REQUIRE(out, HM_EINVAL, "out is null");
        *out = nullptr;
        require_gfx950();
        *out = new hm_learned(hidden, neighbors, seed);
    });
}

void hm_learned_destroy(hm_learned* net) { delete net; }

hm_status hm_learned_set_base(hm_learned* net, int base)
{
    return guarded([&] {
        HM_REQUIRE(net, HM_EINVAL, "net is null");
        HM_REQUIRE(base == HM_PC_BLOCK3 || base == HM_PC_LEAF, HM_EINVAL,
                   "the correction is added to HM_PC_BLOCK3 or HM_PC_LEAF");
        net->net.base = base;
        net->net.reset_moments();
    });
}

hm_status hm_learned_num_params(const hm_learned* net, int64_t* n)
{
    return guarded([&] {
        HM_REQUIRE(net && n, HM_EINVAL, "null argument");
        *n = net->net.n;
    });
}

hm_status hm_learned_get_params(const hm_learned* net, float* host_params, int64_t n)
{
    return guarded([&] {
        HM_REQUIRE(net && host_params, HM_EINVAL, "null argument");
        HM_REQUIRE(n == net->net.n, HM_EINVAL, "parameter count mismatch");
        HM_CHECK_HIP(hipMemcpy(host_params, net->net.params.get(), n * sizeof(float), hipMemcpyDeviceToHost));
    });
}

hm_status hm_learned_set_params(hm_learned* net, const float* host_params, int64_t n)
{
    return guarded([&] {
        HM_REQUIRE(net && host_params, HM_EINVAL, "null argument");
        HM_REQUIRE(n == net->net.n, HM_EINVAL, "parameter count mismatch");
        HM_CHECK_HIP(hipMemcpy(net->net.params.get(), host_params, n * sizeof(float), hipMemcpyHostToDevice));
        net->net.reset_moments();
    });
}

hm_status hm_learned_features(hm_op* op, int neighbors, int64_t cap, int64_t* n_pairs, int32_t* pe, int32_t* pf,
                              float* feat, double* scale, void* hip_stream)
{
    return guarded([&] {
        HM_REQUIRE(op && n_pairs, HM_EINVAL, "null argument");
        hipStream_t s = (hipStream_t)hip_stream;
        hm::learned_prepare(op->op, neighbors, s);
        const hm::LearnedPairs& lp = op->op.lp;
        *n_pairs = lp.P;
        if (cap < lp.P || lp.P == 0) return;
        HM_REQUIRE(pe && pf && feat && scale, HM_EINVAL, "null output array");
        HM_CHECK_HIP(hipMemcpyAsync(pe, lp.pe.get(), lp.P * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HM_CHECK_HIP(hipMemcpyAsync(pf, lp.pf.get(), lp.P * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HM_CHECK_HIP(hipMemcpyAsync(feat, lp.feat.get(), lp.P * 32 * sizeof(float), hipMemcpyDeviceToHost, s));
        HM_CHECK_HIP(hipMemcpyAsync(scale, lp.scale.get(), lp.P * sizeof(double), hipMemcpyDeviceToHost, s));
        HM_CHECK_HIP(hipStreamSynchronize(s));
    });
}

hm_status hm_learned_loss_grad(hm_learned* net, hm_op* op, int ns, const double* d_B, int64_t ldb,
                               const double* d_X, int64_t ldx, double* loss, float* host_grad, void* hip_stream)
{
    return guarded([&] {
        HM_REQUIRE(net && op && loss && host_grad, HM_EINVAL, "null argument");
        hipStream_t s = (hipStream_t)hip_stream;
        *loss = hm::learned_loss_grad(net->net, op->op, ns, d_B, ldb, d_X, ldx, s);
        HM_CHECK_HIP(hipMemcpy(host_grad, net->net.grad.get(), net->net.n * sizeof(float), hipMemcpyDeviceToHost));
    });
}

hm_status hm_learned_train(hm_learned* net, hm_op* op, int n, const double* d_B, int64_t ldb, const double* d_X,
                           int64_t ldx, int steps, int batch, double lr, double* host_loss, void* hip_stream)
{
    return guarded([&] {
        HM_REQUIRE(net && op, HM_EINVAL, "null argument");
        hm::learned_train(net->net, op->op, n, d_B, ldb, d_X, ldx, steps, batch, lr, host_loss,
                          (hipStream_t)hip_stream);
    });
}

hm_status hm_learned_attach(hm_op* op, const hm_learned* net, void* hip_stream)
{
    return guarded([&] {
        HM_REQUIRE(net && op, HM_EINVAL, "null argument");
        hm::learned_attach(op->op, net->net, (hipStream_t)hip_stream);
    });
}

void hm_learned_detach(hm_op* op)
{
    if (op) op->op.lp.attached = false;
}

}  // extern "C"
