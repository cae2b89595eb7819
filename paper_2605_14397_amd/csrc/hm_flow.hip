// Fluid flow in the discontinuities and the fully coupled hydro-mechanical
// step (paper Sec. 3.2 "Fluid-flow in the discontinuities", Sec. 3.3 "A
// fully-coupled hydro-mechanical solver", Sec. 3.3.2 scaling).
//
// Galerkin P1 elements on the triangles of the mesh, pressure at the
// vertices (nodes).  Per element: V_e[a] = A_e/3 (normal DD), S_e = (w/M)
// A_e (1 + [a=b]) / 12, L_e = (w k(w)/mu) A_e grad N_a . grad N_b, N_p
// averages the element's nodes at its collocation point; w = w0 + delta_n.
// The flow matrices are assembled on the GPU into a fixed CSR pattern (the
// node pairs that share an element), each entry summing its own element
// contributions in a fixed order (no atomics): the paper's second GPU
// kernel.
//
// One implicit step solves r(dd, dp) = 0 by Newton's method with the exact
// 2x2 Jacobian
//   [A11 A12; A21 A22] = [E - eta/dt - C^ep, N_p;
//                         V + dS/dd dp + dt dL/dd (dp + p_n - p_o), S + dt L],
// each Jacobian system by right-preconditioned flexible GMRES with the
// paper's upper block-triangular preconditioner P_up = [A11 A12; 0 S~],
// S~ = A22 - A21 diag(A11)^-1 A12: z2 = S~^-1 y2 (ILU(0) of S~, node
// colouring), then A11 z1 = y1 - A12 z2 by an inner GMRES on the operator's
// tangent system.  Unknowns and residuals are scaled block by block
// (Sec. 3.3.2): the solver works on diag(s_R) J diag(1/s_X).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>

#include "hm_op.hpp"

namespace hm {

namespace {

constexpr int kRedBlock = 256;
constexpr int kRedPer = 8;     // entries per thread in the reductions

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ assembly
__global__ void k_flow_coef(int64_t ne, const double* __restrict__ w0, const double* __restrict__ dn0,
                            const double* __restrict__ dd, double inv_M, double inv_mu, int law, double k0,
                            double* __restrict__ s, double* __restrict__ ds, double* __restrict__ t,
                            double* __restrict__ dtr)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const double w = w0[e] + (dn0 ? dn0[e] : 0.0) + (dd ? dd[3 * e + 2] : 0.0);
    s[e] = w * inv_M;
    ds[e] = inv_M;
    if (law == HM_PERM_CUBIC) {
        t[e] = w * w * w * (inv_mu / 12.0);
        dtr[e] = w * w * (inv_mu / 4.0);
    } else {
        t[e] = w * k0 * inv_mu;
        dtr[e] = k0 * inv_mu;
    }
}

// one CSR entry per thread: S[q] and L[q] summed over the entry's element
// contributions (element, local a*3+b) in their stored order
__global__ void k_flow_assemble(int64_t nnz, const int64_t* __restrict__ cptr, const int32_t* __restrict__ cel,
                                const uint8_t* __restrict__ cab, const double* __restrict__ area,
                                const double* __restrict__ stiff, const double* __restrict__ s,
                                const double* __restrict__ t, double* __restrict__ S, double* __restrict__ L)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nnz) return;
    // an entry without contributions is the diagonal of a vertex no element
    // uses: a decoupled unit storage row keeps its pressure increment at zero
    double sv = cptr[q] == cptr[q + 1] ? 1.0 : 0.0, lv = 0.0;
    for (int64_t c = cptr[q]; c < cptr[q + 1]; ++c) {
        const int32_t e = cel[c];
        const int ab = cab[c];
        const double m = area[e] * ((ab % 4 == 0) ? 2.0 : 1.0) / 12.0;   // diagonal of the 3x3 when a == b
        sv += s[e] * m;
        lv += t[e] * stiff[9 * (int64_t)e + ab];
    }
    S[q] = sv;
    L[q] = lv;
}

// per element: column 3e+2 of A21 restricted to its three nodes
//   a21[e][a] = A_e/3 + ds_e (mass_e dp_e)_a + dt dtr_e (stiff_e (dp + p_n - p_o)_e)_a
__global__ void k_flow_a21(int64_t ne, const int32_t* __restrict__ conn, const double* __restrict__ area,
                           const double* __restrict__ stiff, const double* __restrict__ ds,
                           const double* __restrict__ dtr, const double* __restrict__ dp,
                           const double* __restrict__ pnpo, double dt, double* __restrict__ a21)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    double pe[3], qe[3];
    for (int a = 0; a < 3; ++a) {
        const int32_t n = conn[3 * e + a];
        pe[a] = dp ? dp[n] : 0.0;
        qe[a] = pe[a] + (pnpo ? pnpo[n] : 0.0);
    }
    for (int a = 0; a < 3; ++a) {
        double mp = 0.0, kq = 0.0;
        for (int b = 0; b < 3; ++b) {
            mp += area[e] * ((a == b) ? 2.0 : 1.0) / 12.0 * pe[b];
            kq += stiff[9 * e + 3 * a + b] * qe[b];
        }
        a21[3 * e + a] = area[e] / 3.0 + ds[e] * mp + dt * dtr[e] * kq;
    }
}

// A22 = S + dt L and S~ = A22 - A21 diag(A11)^-1 N_p on the CSR pattern:
// contribution (e, a b) adds -a21[e][a] * (1 / A11_{3e+2,3e+2}) / 3
__global__ void k_flow_schur(int64_t nnz, const int64_t* __restrict__ cptr, const int32_t* __restrict__ cel,
                             const uint8_t* __restrict__ cab, const double* __restrict__ S,
                             const double* __restrict__ L, double dt, const double* __restrict__ a21,
                             const double* __restrict__ diag_inv, double* __restrict__ A22, double* __restrict__ St)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nnz) return;
    const double a = S[q] + dt * L[q];
    double c = 0.0;
    for (int64_t k = cptr[q]; k < cptr[q + 1]; ++k) {
        const int32_t e = cel[k];
        c += a21[3 * (int64_t)e + cab[k] / 3] * diag_inv[3 * (int64_t)e + 2] * (1.0 / 3.0);
    }
    A22[q] = a;
    St[q] = a - c;
}

// ------------------------------------------------------------------ products
// flow rows of the Jacobian: y2[i] = sum over the elements e at node i of
// a21[e][a] x1[3e+2]  +  sum_q A22[q] x2[col q]
__global__ void k_flow_rows(int64_t nn, const int64_t* __restrict__ nptr, const int32_t* __restrict__ nel,
                            const uint8_t* __restrict__ na, const double* __restrict__ a21,
                            const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                            const double* __restrict__ A22, const double* __restrict__ x1, const double* __restrict__ x2,
                            double* __restrict__ y2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    double v = 0.0;
    for (int64_t k = nptr[i]; k < nptr[i + 1]; ++k) {
        const int32_t e = nel[k];
        v += a21[3 * (int64_t)e + na[k]] * x1[3 * (int64_t)e + 2];
    }
    for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) v += A22[q] * x2[col[q]];
    y2[i] = v;
}

// y1[3e+2] += scale * (x2[n0] + x2[n1] + x2[n2]) / 3   (N_p x2)
__global__ void k_np_add(int64_t ne, const int32_t* __restrict__ conn, const double* __restrict__ x2, double scale,
                         double* __restrict__ y1)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    y1[3 * e + 2] += scale * (x2[conn[3 * e]] + x2[conn[3 * e + 1]] + x2[conn[3 * e + 2]]) * (1.0 / 3.0);
}

// pressure increment at the collocation points (N_p dp, normal rows)
__global__ void k_np_centroid(int64_t ne, const int32_t* __restrict__ conn, const double* __restrict__ dp,
                              double* __restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    out[e] = (dp[conn[3 * e]] + dp[conn[3 * e + 1]] + dp[conn[3 * e + 2]]) * (1.0 / 3.0);
}

// r_f[i] = sum_e V dd + sum_q ((S + dt L)[q] dp[j] + dt L[q] pnpo[j]) - dt f[i]
__global__ void k_flow_residual(int64_t nn, const int64_t* __restrict__ nptr, const int32_t* __restrict__ nel,
                                const double* __restrict__ area, const double* __restrict__ dd,
                                const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                const double* __restrict__ S, const double* __restrict__ L,
                                const double* __restrict__ dp, const double* __restrict__ pnpo,
                                const double* __restrict__ f, double dt, double* __restrict__ r)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    double v = 0.0;
    for (int64_t k = nptr[i]; k < nptr[i + 1]; ++k) {
        const int32_t e = nel[k];
        v += area[e] * (1.0 / 3.0) * dd[3 * (int64_t)e + 2];
    }
    for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
        const int32_t j = col[q];
        v += (S[q] + dt * L[q]) * dp[j] + dt * L[q] * (pnpo ? pnpo[j] : 0.0);
    }
    r[i] = v - dt * (f ? f[i] : 0.0);
}

// mechanical residual with the pressure at the collocation points
__global__ void k_coupled_mech_residual(int64_t ne, const double* __restrict__ dT0, const double* __restrict__ t_new,
                                        const double* __restrict__ t_n, const double* __restrict__ Ex,
                                        const double* __restrict__ dpress, const double* __restrict__ eta_dt,
                                        const double* __restrict__ dd, const double* __restrict__ dd_prev,
                                        double* __restrict__ r)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    for (int i = 0; i < 3; ++i) {
        const int64_t k = 3 * e + i;
        double v = (dT0 ? dT0[k] : 0.0) - (t_new[k] - t_n[k]) + Ex[k];
        if (i == 2) v += dpress[e];
        if (eta_dt) v -= eta_dt[k] * (dd[k] - (dd_prev ? dd_prev[k] : 0.0));
        r[k] = v;
    }
}

// ------------------------------------------------------------------ ILU(0) of S~
// rows sorted by elimination order (node colour, id); one thread per node of a colour
__global__ void k_node_ilu_factor(const int32_t* __restrict__ nodes, int n, const int32_t* __restrict__ pos,
                                  const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                  const int64_t* __restrict__ diag, double* __restrict__ val, int* __restrict__ status)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t i = nodes[t];
    const int64_t re = rowptr[i + 1], di = diag[i];
    for (int64_t x = rowptr[i]; x < di; ++x) {
        const int32_t k = col[x];
        const double lik = val[x] / val[diag[k]];
        val[x] = lik;
        int64_t y = diag[k] + 1, z = x + 1;
        const int64_t ye = rowptr[k + 1];
        while (y < ye && z < re) {
            const int32_t py = pos[col[y]], pz = pos[col[z]];
            if (py == pz) {
                val[z] -= lik * val[y];
                ++y;
                ++z;
            } else if (py < pz) {
                ++y;
            } else {
                ++z;
            }
        }
    }
    const double piv = val[di];
    if (!(fabs(piv) > 0.0) || !isfinite(piv)) atomicExch(status, 1);
}

__global__ void k_node_ilu_forward(const int32_t* __restrict__ nodes, int n, const int64_t* __restrict__ rowptr,
                                   const int32_t* __restrict__ col, const int64_t* __restrict__ diag,
                                   const double* __restrict__ val, const double* __restrict__ r, double* __restrict__ z)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t i = nodes[t];
    double s = r[i];
    for (int64_t x = rowptr[i]; x < diag[i]; ++x) s -= val[x] * z[col[x]];
    z[i] = s;
}

__global__ void k_node_ilu_backward(const int32_t* __restrict__ nodes, int n, const int64_t* __restrict__ rowptr,
                                    const int32_t* __restrict__ col, const int64_t* __restrict__ diag,
                                    const double* __restrict__ val, double* __restrict__ z)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t i = nodes[t];
    double s = z[i];
    for (int64_t x = diag[i] + 1; x < rowptr[i + 1]; ++x) s -= val[x] * z[col[x]];
    z[i] = s / val[diag[i]];
}

// ------------------------------------------------------------------ vector kernels
// partial dot products of w against J vectors V_j (V_j = V + j ld), two stages
__global__ __launch_bounds__(kRedBlock) void k_mdot(int64_t n, const double* __restrict__ V, int64_t ld, int J,
                                                    const double* __restrict__ w, double* __restrict__ partial,
                                                    int nblk)
{
    __shared__ double red[kRedBlock];
    const int j = blockIdx.y;
    const double* v = V + (int64_t)j * ld;
    const int64_t base = (int64_t)blockIdx.x * kRedBlock * kRedPer + threadIdx.x;
    double s = 0.0;
    for (int k = 0; k < kRedPer; ++k) {
        const int64_t i = base + (int64_t)k * kRedBlock;
        if (i < n) s += v[i] * w[i];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kRedBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)j * nblk + blockIdx.x] = red[0];
    (void)J;
}

// w -= sum_j h[j] V_j
__global__ void k_vsub(int64_t n, const double* __restrict__ V, int64_t ld, int J, const double* __restrict__ h,
                       double* __restrict__ w)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = w[i];
    for (int j = 0; j < J; ++j) s -= h[j] * V[(int64_t)j * ld + i];
    w[i] = s;
}

// y = a x (+ y when acc)
__global__ void k_axpy(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y, int acc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = a * x[i] + (acc ? y[i] : 0.0);
}

// x = sum_j c[j] Z_j  (added to x)
__global__ void k_vadd(int64_t n, const double* __restrict__ Z, int64_t ld, int J, const double* __restrict__ c,
                       double* __restrict__ x)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = x[i];
    for (int j = 0; j < J; ++j) s += c[j] * Z[(int64_t)j * ld + i];
    x[i] = s;
}

}  // namespace

// ------------------------------------------------------------------ the flow problem
struct Flow {
    int64_t ne = 0, nn = 0, nnz = 0, ncon = 0;
    hm_flow_params prm{};
    DevBuf conn, area, stiff;          // int32 [N][3], double [N], double [N][9]
    DevBuf rowptr, col;                // nodal CSR, rows in elimination order of the node colouring
    DevBuf cptr, cel, cab;             // per entry: element contributions (element, a * 3 + b)
    DevBuf nptr, nel, na;              // per node: incident (element, local index)
    int n_colors = 0;
    std::vector<int64_t> color_begin;
    DevBuf order, pos, diag;           // int32 [n], int32 [n], int64 [n]
};

Flow* flow_create(const Mesh& m, const hm_flow_params& p, hipStream_t s)
{
    HM_REQUIRE(m.nvpe == 3, HM_EUNSUPPORTED, "the flow elements are the mesh's triangles");
    HM_REQUIRE(p.M > 0.0 && p.mu > 0.0, HM_EINVAL, "storage modulus and viscosity must be positive");
    HM_REQUIRE(p.perm_law == HM_PERM_CUBIC || (p.perm_law == HM_PERM_CONSTANT && p.k0 > 0.0), HM_EINVAL,
               "permeability law: HM_PERM_CUBIC, or HM_PERM_CONSTANT with k0 > 0");
    std::unique_ptr<Flow> F(new Flow());
    F->prm = p;
    const int64_t ne = m.ne, nn = m.nv;
    HM_REQUIRE(nn < (int64_t)1 << 31 && ne < (int64_t)1 << 31, HM_EUNSUPPORTED, "flow: more than 2^31 nodes");
    F->ne = ne;
    F->nn = nn;
    // element geometry: area, unit-coefficient stiffness A grad N_a . grad N_b
    std::vector<int32_t> conn(3 * ne);
    std::vector<double> area(ne), stiff(9 * ne);
    for (int64_t e = 0; e < ne; ++e) {
        double x[3][3];
        for (int a = 0; a < 3; ++a) {
            conn[3 * e + a] = (int32_t)m.conn[3 * e + a];
            for (int k = 0; k < 3; ++k) x[a][k] = m.xyz[3 * m.conn[3 * e + a] + k];
        }
        double u[3], v[3], c[3];
        for (int k = 0; k < 3; ++k) {
            u[k] = x[1][k] - x[0][k];
            v[k] = x[2][k] - x[0][k];
        }
        c[0] = u[1] * v[2] - u[2] * v[1];
        c[1] = u[2] * v[0] - u[0] * v[2];
        c[2] = u[0] * v[1] - u[1] * v[0];
        const double two_a = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        const double n[3] = {c[0] / two_a, c[1] / two_a, c[2] / two_a};
        double g[3][3];
        for (int a = 0; a < 3; ++a) {
            double ed[3];
            for (int k = 0; k < 3; ++k) ed[k] = x[(a + 2) % 3][k] - x[(a + 1) % 3][k];
            g[a][0] = (n[1] * ed[2] - n[2] * ed[1]) / two_a;
            g[a][1] = (n[2] * ed[0] - n[0] * ed[2]) / two_a;
            g[a][2] = (n[0] * ed[1] - n[1] * ed[0]) / two_a;
        }
        area[e] = 0.5 * two_a;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                stiff[9 * e + 3 * a + b] = area[e] * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]);
    }
    // node -> incident elements
    std::vector<int64_t> nptr(nn + 1, 0);
    for (int32_t x : conn) nptr[x + 1]++;
    for (int64_t i = 0; i < nn; ++i) nptr[i + 1] += nptr[i];
    std::vector<int32_t> nel(3 * ne);
    std::vector<uint8_t> na(3 * ne);
    {
        std::vector<int64_t> at(nptr.begin(), nptr.end() - 1);
        for (int64_t e = 0; e < ne; ++e)
            for (int a = 0; a < 3; ++a) {
                const int64_t q = at[conn[3 * e + a]]++;
                nel[q] = (int32_t)e;
                na[q] = (uint8_t)a;
            }
    }
    // node graph, greedy colouring in increasing id, elimination order
    std::vector<std::vector<int32_t>> nb(nn);
    for (int64_t i = 0; i < nn; ++i) {
        nb[i].push_back((int32_t)i);
        for (int64_t k = nptr[i]; k < nptr[i + 1]; ++k)
            for (int b = 0; b < 3; ++b) nb[i].push_back(conn[3 * (int64_t)nel[k] + b]);
        std::sort(nb[i].begin(), nb[i].end());
        nb[i].erase(std::unique(nb[i].begin(), nb[i].end()), nb[i].end());
    }
    std::vector<int32_t> colour(nn, 0);
    int n_colors = 0;
    {
        std::vector<int64_t> seen;
        for (int64_t i = 0; i < nn; ++i) {
            for (int32_t j : nb[i])
                if (j < i) {
                    const int32_t c = colour[j];
                    if ((size_t)c >= seen.size()) seen.resize(c + 1, -1);
                    seen[c] = i;
                }
            int32_t c = 0;
            while ((size_t)c < seen.size() && seen[c] == i) ++c;
            colour[i] = c;
            n_colors = std::max(n_colors, c + 1);
        }
    }
    std::vector<int32_t> order(nn), pos(nn);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return colour[a] < colour[b]; });
    for (int64_t q = 0; q < nn; ++q) pos[order[q]] = (int32_t)q;
    std::vector<int64_t> color_begin(n_colors + 1, 0);
    for (int64_t i = 0; i < nn; ++i) color_begin[colour[i] + 1]++;
    for (int c = 0; c < n_colors; ++c) color_begin[c + 1] += color_begin[c];
    // CSR rows (sorted by elimination order) and each entry's contributions
    std::vector<int64_t> rowptr(nn + 1, 0), diag(nn, -1), cptr;
    std::vector<int32_t> col, cel;
    std::vector<uint8_t> cab;
    cptr.push_back(0);
    for (int64_t i = 0; i < nn; ++i) {
        std::vector<int32_t> row = nb[i];
        std::sort(row.begin(), row.end(), [&](int32_t a, int32_t b) { return pos[a] < pos[b]; });
        for (int32_t j : row) {
            if (j == i) diag[i] = (int64_t)col.size();
            col.push_back(j);
            // contributions: every element holding both i and j, in incidence order of i
            for (int64_t k = nptr[i]; k < nptr[i + 1]; ++k) {
                const int64_t e = nel[k];
                for (int b = 0; b < 3; ++b)
                    if (conn[3 * e + b] == j) {
                        cel.push_back((int32_t)e);
                        cab.push_back((uint8_t)(3 * na[k] + b));
                    }
            }
            cptr.push_back((int64_t)cel.size());
        }
        rowptr[i + 1] = (int64_t)col.size();
        HM_REQUIRE(diag[i] >= 0, HM_EINTERNAL, "flow: node row without diagonal");
    }
    F->nnz = (int64_t)col.size();
    F->ncon = (int64_t)cel.size();
    upload(F->conn, conn, s);
    upload(F->area, area, s);
    upload(F->stiff, stiff, s);
    upload(F->rowptr, rowptr, s);
    upload(F->col, col, s);
    upload(F->cptr, cptr, s);
    upload(F->cel, cel, s);
    upload(F->cab, cab, s);
    upload(F->nptr, nptr, s);
    upload(F->nel, nel, s);
    upload(F->na, na, s);
    upload(F->order, order, s);
    upload(F->pos, pos, s);
    upload(F->diag, diag, s);
    HM_CHECK_HIP(hipStreamSynchronize(s));
    F->n_colors = n_colors;
    F->color_begin = color_begin;
    return F.release();
}

void flow_destroy(Flow* f) { delete f; }
int64_t flow_num_nodes(const Flow& f) { return f.nn; }
int64_t flow_nnz(const Flow& f) { return f.nnz; }

static void flow_coefficients(const Flow& F, const double* w0, const double* dn0, const double* dd, double* s,
                              double* ds, double* t, double* dtr, hipStream_t st)
{
    hipLaunchKernelGGL(k_flow_coef, dim3((unsigned)((F.ne + 255) / 256)), dim3(256), 0, st, F.ne, w0, dn0, dd,
                       1.0 / F.prm.M, 1.0 / F.prm.mu, F.prm.perm_law, F.prm.k0, s, ds, t, dtr);
}

static void flow_assemble(const Flow& F, const double* s, const double* t, double* S, double* L, hipStream_t st)
{
    hipLaunchKernelGGL(k_flow_assemble, dim3((unsigned)((F.nnz + 255) / 256)), dim3(256), 0, st, F.nnz,
                       F.cptr.as<int64_t>(), F.cel.as<int32_t>(), F.cab.as<uint8_t>(), F.area.as<double>(),
                       F.stiff.as<double>(), s, t, S, L);
}

void flow_matrices(const Flow& F, const double* d_w, int64_t* rowptr, int32_t* col, double* S, double* L,
                   hipStream_t st)
{
    DevBuf c(sizeof(double) * 4 * F.ne), m(sizeof(double) * 2 * F.nnz);
    double* cs = c.as<double>();
    flow_coefficients(F, d_w, nullptr, nullptr, cs, cs + F.ne, cs + 2 * F.ne, cs + 3 * F.ne, st);
    flow_assemble(F, cs, cs + 2 * F.ne, m.as<double>(), m.as<double>() + F.nnz, st);
    HM_CHECK_HIP(hipGetLastError());
    if (rowptr) HM_CHECK_HIP(hipMemcpyAsync(rowptr, F.rowptr.get(), (F.nn + 1) * 8, hipMemcpyDeviceToHost, st));
    if (col) HM_CHECK_HIP(hipMemcpyAsync(col, F.col.get(), F.nnz * 4, hipMemcpyDeviceToHost, st));
    if (S) HM_CHECK_HIP(hipMemcpyAsync(S, m.get(), F.nnz * 8, hipMemcpyDeviceToHost, st));
    if (L) HM_CHECK_HIP(hipMemcpyAsync(L, m.as<double>() + F.nnz, F.nnz * 8, hipMemcpyDeviceToHost, st));
    HM_CHECK_HIP(hipStreamSynchronize(st));
}

// ------------------------------------------------------------------ the coupled step
namespace {

// Everything one coupled Newton step keeps on the device.
struct CoupledWs {
    int64_t n3, nn, ntot, nblk;
    DevBuf buf;
    double *Ex, *r, *dpress, *cep, *D, *coef, *S, *L, *A22, *St, *Sf, *a21, *pnpo;
    double *V, *Z, *w, *t1, *t2, *partial, *hdev, *x;
    double *Vs, *sq, *sx, *u3;   // the Schur-complement GMRES of the second choice
    int32_t* mode;
    int m, ms;
};

struct Coupled {
    Op& op;
    const Flow& F;
    hipStream_t s;
    CoupledWs W;
    double sX[2], sR[2];   // unknown and residual scales (mechanics, flow)
    double dt;
    hm_solve_opts inner;
    int inner_its = 0;
    int schur = 0;             // 0: S~ from diag(A11); 1: S~ from the ILU approximation of A11
    double schur_rtol = 1e-2;
    int schur_its = 0;

    unsigned g(int64_t n) const { return (unsigned)((n + 255) / 256); }

    // vector of length ntot: [mechanics 3N | flow n]
    // y = diag(sR) J diag(1/sX) x
    void jac(const double* x, double* y)
    {
        const int64_t n3 = W.n3;
        // unscaled unknowns in t1 (mechanics) and t2 (flow)
        hipLaunchKernelGGL(k_axpy, dim3(g(n3)), dim3(256), 0, s, n3, 1.0 / sX[0], x, W.t1, 0);
        hipLaunchKernelGGL(k_axpy, dim3(g(W.nn)), dim3(256), 0, s, W.nn, 1.0 / sX[1], x + n3, W.t2, 0);
        apply(op, op.main, 1, W.t1, n3, y, n3, true, s);       // A11 x1 (tangent)
        hipLaunchKernelGGL(k_np_add, dim3(g(op.ne)), dim3(256), 0, s, op.ne, F.conn.as<int32_t>(), W.t2, 1.0, y);
        hipLaunchKernelGGL(k_flow_rows, dim3(g(W.nn)), dim3(256), 0, s, W.nn, F.nptr.as<int64_t>(),
                           F.nel.as<int32_t>(), F.na.as<uint8_t>(), W.a21, F.rowptr.as<int64_t>(), F.col.as<int32_t>(),
                           W.A22, W.t1, W.t2, y + n3);
        hipLaunchKernelGGL(k_axpy, dim3(g(n3)), dim3(256), 0, s, n3, sR[0], y, y, 0);
        hipLaunchKernelGGL(k_axpy, dim3(g(W.nn)), dim3(256), 0, s, W.nn, sR[1], y + n3, y + n3, 0);
    }

    // z = ILU(0)(S~ of the first choice)^-1 r, colour by colour
    void schur_diag_solve(const double* r, double* z)
    {
        for (int c = 0; c < F.n_colors; ++c) {
            const int n = (int)(F.color_begin[c + 1] - F.color_begin[c]);
            hipLaunchKernelGGL(k_node_ilu_forward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                               F.order.as<int32_t>() + F.color_begin[c], n, F.rowptr.as<int64_t>(),
                               F.col.as<int32_t>(), F.diag.as<int64_t>(), W.Sf, r, z);
        }
        for (int c = F.n_colors - 1; c >= 0; --c) {
            const int n = (int)(F.color_begin[c + 1] - F.color_begin[c]);
            hipLaunchKernelGGL(k_node_ilu_backward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                               F.order.as<int32_t>() + F.color_begin[c], n, F.rowptr.as<int64_t>(),
                               F.col.as<int32_t>(), F.diag.as<int64_t>(), W.Sf, z);
        }
    }

    // y = S~ x of the second choice: A22 x - A21 A~11^-1 N_p x, with A~11^-1
    // the ILU solve of C^ep plus the kept near-field entries
    void schur_apply(const double* x, double* y)
    {
        const int64_t n3 = W.n3;
        HM_CHECK_HIP(hipMemsetAsync(W.t1, 0, sizeof(double) * n3, s));
        hipLaunchKernelGGL(k_np_add, dim3(g(op.ne)), dim3(256), 0, s, op.ne, F.conn.as<int32_t>(), x, 1.0, W.t1);
        ilu_pc_apply(op, 1, W.t1, n3, W.u3, n3, s);
        hipLaunchKernelGGL(k_axpy, dim3(g(n3)), dim3(256), 0, s, n3, -1.0, W.u3, W.u3, 0);
        hipLaunchKernelGGL(k_flow_rows, dim3(g(W.nn)), dim3(256), 0, s, W.nn, F.nptr.as<int64_t>(),
                           F.nel.as<int32_t>(), F.na.as<uint8_t>(), W.a21, F.rowptr.as<int64_t>(), F.col.as<int32_t>(),
                           W.A22, W.u3, x, y);
    }

    // x = S~^-1 b (second choice) by GMRES without restart, right-preconditioned
    // with the first choice's ILU(0), to schur_rtol
    void schur_solve(const double* b, double* x)
    {
        const int64_t nn = W.nn;
        const int m = W.ms;
        std::vector<double> h, h2, nrm, H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), y(m);
        dots_n(nn, b, nn, 1, b, nrm);
        const double beta = std::sqrt(nrm[0]);
        if (beta == 0.0) {
            HM_CHECK_HIP(hipMemsetAsync(x, 0, sizeof(double) * nn, s));
            return;
        }
        hipLaunchKernelGGL(k_axpy, dim3(g(nn)), dim3(256), 0, s, nn, 1.0 / beta, b, W.Vs, 0);
        gv[0] = beta;
        int k = 0;
        for (; k < m; ++k) {
            double* vk = W.Vs + (int64_t)k * nn;
            double* vn = W.Vs + (int64_t)(k + 1) * nn;
            schur_diag_solve(vk, W.sq);
            schur_apply(W.sq, vn);
            dots_n(nn, W.Vs, nn, k + 1, vn, h);
            HM_CHECK_HIP(hipMemcpyAsync(W.hdev, h.data(), sizeof(double) * (k + 1), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_vsub, dim3(g(nn)), dim3(256), 0, s, nn, W.Vs, nn, k + 1, W.hdev, vn);
            dots_n(nn, W.Vs, nn, k + 1, vn, h2);
            HM_CHECK_HIP(hipMemcpyAsync(W.hdev, h2.data(), sizeof(double) * (k + 1), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_vsub, dim3(g(nn)), dim3(256), 0, s, nn, W.Vs, nn, k + 1, W.hdev, vn);
            dots_n(nn, vn, nn, 1, vn, nrm);
            double* col = &H[(size_t)k * (m + 1)];
            for (int i = 0; i <= k; ++i) col[i] = h[i] + h2[i];
            col[k + 1] = std::sqrt(nrm[0]);
            if (col[k + 1] > 0.0)
                hipLaunchKernelGGL(k_axpy, dim3(g(nn)), dim3(256), 0, s, nn, 1.0 / col[k + 1], vn, vn, 0);
            for (int i = 0; i < k; ++i) {
                const double t = cs[i] * col[i] + sn[i] * col[i + 1];
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
                col[i] = t;
            }
            const double r = std::hypot(col[k], col[k + 1]);
            cs[k] = r == 0.0 ? 1.0 : col[k] / r;
            sn[k] = r == 0.0 ? 0.0 : col[k + 1] / r;
            col[k] = r;
            col[k + 1] = 0.0;
            gv[k + 1] = -sn[k] * gv[k];
            gv[k] = cs[k] * gv[k];
            ++schur_its;
            if (std::fabs(gv[k + 1]) <= schur_rtol * beta || !std::isfinite(gv[k + 1])) {
                ++k;
                break;
            }
        }
        for (int i = k - 1; i >= 0; --i) {
            double sum = gv[i];
            for (int l = i + 1; l < k; ++l) sum -= H[(size_t)l * (m + 1) + i] * y[l];
            const double d = H[(size_t)i * (m + 1) + i];
            y[i] = d != 0.0 ? sum / d : 0.0;
        }
        HM_CHECK_HIP(hipMemsetAsync(W.sx, 0, sizeof(double) * nn, s));
        HM_CHECK_HIP(hipMemcpyAsync(W.hdev, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_vadd, dim3(g(nn)), dim3(256), 0, s, nn, W.Vs, nn, k, W.hdev, W.sx);
        schur_diag_solve(W.sx, x);
    }

    // z = diag(sX) P_up^-1 diag(1/sR) y
    void prec(const double* y, double* z)
    {
        const int64_t n3 = W.n3;
        // z2 = S~^-1 (y2 / sR_f)
        hipLaunchKernelGGL(k_axpy, dim3(g(W.nn)), dim3(256), 0, s, W.nn, 1.0 / sR[1], y + n3, W.t2, 0);
        double* z2 = z + n3;
        if (schur == 1)
            schur_solve(W.t2, z2);
        else
            schur_diag_solve(W.t2, z2);
        // A11 z1 = y1 / sR_m - N_p z2
        hipLaunchKernelGGL(k_axpy, dim3(g(n3)), dim3(256), 0, s, n3, 1.0 / sR[0], y, W.t1, 0);
        hipLaunchKernelGGL(k_np_add, dim3(g(op.ne)), dim3(256), 0, s, op.ne, F.conn.as<int32_t>(), z2, -1.0, W.t1);
        HM_CHECK_HIP(hipGetLastError());
        hm_solve_report rep{};
        const hm_status st = solve(op, inner, 1, W.t1, n3, z, n3, &rep, s);
        HM_REQUIRE(st == HM_OK || st == HM_ENOTCONV, st, "inner A11 solve failed");
        inner_its += rep.iterations;
        hipLaunchKernelGGL(k_axpy, dim3(g(n3)), dim3(256), 0, s, n3, sX[0], z, z, 0);
        hipLaunchKernelGGL(k_axpy, dim3(g(W.nn)), dim3(256), 0, s, W.nn, sX[1], z2, z2, 0);
    }

    // h[j] = V_j . w for j < J, vectors of length n with stride ld
    // (deterministic: fixed blocks, host sum in order)
    void dots_n(int64_t n, const double* V, int64_t ld, int J, const double* w, std::vector<double>& h)
    {
        const int64_t nb = (n + kRedBlock * kRedPer - 1) / (kRedBlock * kRedPer);
        hipLaunchKernelGGL(k_mdot, dim3((unsigned)nb, J), dim3(kRedBlock), 0, s, n, V, ld, J, w, W.partial, (int)nb);
        std::vector<double> part((size_t)J * nb);
        HM_CHECK_HIP(hipMemcpyAsync(part.data(), W.partial, sizeof(double) * part.size(), hipMemcpyDeviceToHost, s));
        HM_CHECK_HIP(hipStreamSynchronize(s));
        h.assign(J, 0.0);
        for (int j = 0; j < J; ++j)
            for (int64_t b = 0; b < nb; ++b) h[j] += part[(size_t)j * nb + b];
    }
    void dots(const double* V, int J, const double* w, std::vector<double>& h) { dots_n(W.ntot, V, W.ntot, J, w, h); }

    // right-preconditioned restarted FGMRES with CGS2 on diag(sR) J diag(1/sX) x^ = b^ (x0 = 0);
    // returns iterations, writes x^ to W.x
    int fgmres(const double* b, double rtol, int restart, int max_iter)
    {
        const int64_t nt = W.ntot;
        const int m = std::min(restart, W.m);
        std::vector<double> h, h2, H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), y(m);
        HM_CHECK_HIP(hipMemsetAsync(W.x, 0, sizeof(double) * nt, s));
        std::vector<double> bb;
        dots(b, 1, b, bb);
        const double bnorm = std::sqrt(bb[0]);
        if (bnorm == 0.0) return 0;
        int its = 0;
        // residual r = b - A x in V_0
        HM_CHECK_HIP(hipMemcpyAsync(W.V, b, sizeof(double) * nt, hipMemcpyDeviceToDevice, s));
        double beta = bnorm;
        while (its < max_iter) {
            hipLaunchKernelGGL(k_axpy, dim3(g(nt)), dim3(256), 0, s, nt, 1.0 / beta, W.V, W.V, 0);
            std::fill(gv.begin(), gv.end(), 0.0);
            gv[0] = beta;
            int k = 0;
            double res = beta;
            for (; k < m && its < max_iter; ++k, ++its) {
                double* vk = W.V + (int64_t)k * nt;
                double* zk = W.Z + (int64_t)k * nt;
                double* vn = W.V + (int64_t)(k + 1) * nt;
                prec(vk, zk);
                jac(zk, vn);
                dots(W.V, k + 1, vn, h);
                HM_CHECK_HIP(hipMemcpyAsync(W.hdev, h.data(), sizeof(double) * (k + 1), hipMemcpyHostToDevice, s));
                hipLaunchKernelGGL(k_vsub, dim3(g(nt)), dim3(256), 0, s, nt, W.V, nt, k + 1, W.hdev, vn);
                dots(W.V, k + 1, vn, h2);
                HM_CHECK_HIP(hipMemcpyAsync(W.hdev, h2.data(), sizeof(double) * (k + 1), hipMemcpyHostToDevice, s));
                hipLaunchKernelGGL(k_vsub, dim3(g(nt)), dim3(256), 0, s, nt, W.V, nt, k + 1, W.hdev, vn);
                std::vector<double> nn2;
                dots(vn, 1, vn, nn2);
                double* col = &H[(size_t)k * (m + 1)];
                for (int i = 0; i <= k; ++i) col[i] = h[i] + h2[i];
                col[k + 1] = std::sqrt(nn2[0]);
                if (col[k + 1] > 0.0)
                    hipLaunchKernelGGL(k_axpy, dim3(g(nt)), dim3(256), 0, s, nt, 1.0 / col[k + 1], vn, vn, 0);
                for (int i = 0; i < k; ++i) {
                    const double t = cs[i] * col[i] + sn[i] * col[i + 1];
                    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
                    col[i] = t;
                }
                const double r = std::hypot(col[k], col[k + 1]);
                cs[k] = r == 0.0 ? 1.0 : col[k] / r;
                sn[k] = r == 0.0 ? 0.0 : col[k + 1] / r;
                col[k] = r;
                col[k + 1] = 0.0;
                gv[k + 1] = -sn[k] * gv[k];
                gv[k] = cs[k] * gv[k];
                res = std::fabs(gv[k + 1]);
                if (!std::isfinite(res) || res <= rtol * bnorm) {
                    ++k;
                    ++its;
                    break;
                }
            }
            // x += Z y
            for (int i = k - 1; i >= 0; --i) {
                double sum = gv[i];
                for (int l = i + 1; l < k; ++l) sum -= H[(size_t)l * (m + 1) + i] * y[l];
                const double d = H[(size_t)i * (m + 1) + i];
                y[i] = d != 0.0 ? sum / d : 0.0;
            }
            HM_CHECK_HIP(hipMemcpyAsync(W.hdev, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_vadd, dim3(g(nt)), dim3(256), 0, s, nt, W.Z, nt, k, W.hdev, W.x);
            if (res <= rtol * bnorm || !std::isfinite(res)) break;
            // true residual for the restart: V_0 = b - A x
            jac(W.x, W.w);
            hipLaunchKernelGGL(k_axpy, dim3(g(nt)), dim3(256), 0, s, nt, -1.0, W.w, W.V, 0);
            hipLaunchKernelGGL(k_axpy, dim3(g(nt)), dim3(256), 0, s, nt, 1.0, b, W.V, 1);
            std::vector<double> rr;
            dots(W.V, 1, W.V, rr);
            beta = std::sqrt(rr[0]);
            if (beta <= rtol * bnorm) break;
        }
        HM_CHECK_HIP(hipGetLastError());
        return its;
    }
};

}  // namespace

hm_status coupled_step(Op& op, const Flow& F, int n_mat, const hm_interface_material* mats, const int32_t* d_mat_id,
                       const double* d_t, const double* d_dp, const double* d_chi, const double* d_dT0,
                       const double* d_eta_dt, const double* d_dd_prev, const double* d_p_n, const double* d_p_o,
                       const double* d_source, const double* d_w0, const double* d_dn_start, double dt, double* d_dd,
                       double* d_dpn, double* d_t_new, double* d_dp_new, double* d_chi_new, const hm_coupled_opts& o,
                       hm_coupled_report* rep, hipStream_t s)
{
    HM_REQUIRE(F.ne == op.ne, HM_EINVAL, "the flow problem and the operator have different meshes");
    HM_REQUIRE(dt > 0.0, HM_EINVAL, "dt must be positive");
    HM_REQUIRE(o.max_newton >= 0 && o.max_newton <= 63, HM_EINVAL, "max_newton must be in [0, 63]");
    HM_REQUIRE(o.outer_restart >= 1 && o.outer_restart <= 200 && o.outer_max_iter >= 1, HM_EINVAL,
               "outer solver: restart in [1, 200], max_iter >= 1");
    HM_REQUIRE(d_t && d_dp && d_chi && d_p_n && d_w0 && d_dd && d_dpn && d_t_new && d_dp_new && d_chi_new,
               HM_EINVAL, "state and increment arrays must not be null");
    HM_REQUIRE(d_t_new != d_t && d_dp_new != d_dp && d_chi_new != d_chi, HM_EINVAL,
               "the start-of-step state is read at every iteration: outputs must be other arrays");
    HM_REQUIRE(op.ref || op.main.near_prec == HM_F64, HM_EINVAL,
               "the residual needs the FP64 operator (build FP64 or with keep_f64_reference)");
    HM_REQUIRE(!op.has_mask, HM_EUNSUPPORTED, "the coupled step runs on an operator without inactive elements");
    HM_REQUIRE(o.schur == 0 || (o.schur == 1 && o.schur_max_iter >= 1 && o.schur_max_iter <= 200 && o.schur_rtol > 0),
               HM_EINVAL, "schur: 0, or 1 with schur_max_iter in [1, 200] and schur_rtol > 0");
    const double t0 = now_ms();
    const int64_t ne = op.ne, n3 = 3 * ne, nn = F.nn;
    Coupled C{op, F, s, {}, {1, 1}, {1, 1}, dt, o.inner, 0};
    for (int k = 0; k < 2; ++k) {
        C.sX[k] = o.scales[k] > 0.0 ? o.scales[k] : 1.0;
        C.sR[k] = o.scales[2 + k] > 0.0 ? o.scales[2 + k] : 1.0;
    }
    CoupledWs& W = C.W;
    W.n3 = n3;
    W.nn = nn;
    W.ntot = n3 + nn;
    W.nblk = (W.ntot + kRedBlock * kRedPer - 1) / (kRedBlock * kRedPer);
    W.m = o.outer_restart;
    W.ms = o.schur == 1 ? o.schur_max_iter : 0;
    C.schur = o.schur;
    C.schur_rtol = o.schur_rtol;
    const int64_t nnz = F.nnz;
    // carve the workspace: the same sequence sizes it (base = null) and then places it
    auto carve = [&](double* base) -> size_t {
        size_t at = 0;
        auto take = [&](size_t n) {
            double* q = base ? base + at : nullptr;
            at += n;
            return q;
        };
        W.Ex = take(n3);
        W.r = take(W.ntot);
        W.dpress = take(ne);
        W.cep = take(9 * ne);
        W.D = take(9 * ne);
        W.coef = take(4 * ne);
        W.S = take(nnz);
        W.L = take(nnz);
        W.A22 = take(nnz);
        W.St = take(nnz);
        W.a21 = take(3 * ne);
        W.pnpo = take(nn);
        W.V = take((size_t)(W.m + 1) * W.ntot);
        W.Z = take((size_t)W.m * W.ntot);
        W.w = take(W.ntot);
        W.x = take(W.ntot);
        W.t1 = take(n3);
        W.t2 = take(nn);
        W.partial = take((size_t)(std::max(W.m, W.ms) + 2) * W.nblk);
        W.hdev = take(std::max(W.m, W.ms) + 2);
        W.Vs = take((size_t)(W.ms + 1) * nn);
        W.sq = take(nn);
        W.sx = take(nn);
        W.u3 = take(n3);
        double* mode = take((ne + 1) / 2);   // int32 [N]
        W.mode = reinterpret_cast<int32_t*>(mode);
        return at;
    };
    const size_t nd = carve(nullptr);
    W.buf.alloc(nd * sizeof(double));
    HM_REQUIRE(carve(W.buf.as<double>()) == nd, HM_EINTERNAL, "coupled workspace layout");
    W.Sf = W.St;   // ILU factors in place of S~
    const unsigned ge = (unsigned)((ne + 255) / 256), gn = (unsigned)((nn + 255) / 256);
    // p_n - p_o (the pressure change already reached at the start of the step)
    if (d_p_o)
        hipLaunchKernelGGL(k_axpy, dim3(gn), dim3(256), 0, s, nn, -1.0, d_p_o, W.pnpo, 0);
    else
        HM_CHECK_HIP(hipMemsetAsync(W.pnpo, 0, sizeof(double) * nn, s));
    hipLaunchKernelGGL(k_axpy, dim3(gn), dim3(256), 0, s, nn, 1.0, d_p_n, W.pnpo, 1);
    double* cs = W.coef;   // s, ds, t, dtr
    const Variant& vref = op.ref_variant();
    std::vector<double> hist, hm_, hf_;
    std::vector<int> outer, inner, schur_its;
    std::vector<double> rr;
    for (int k = 0;; ++k) {
        // residuals at (dd, dp)
        interface_update(n_mat, mats, ne, d_mat_id, d_dd, d_t, d_dp, d_chi, d_t_new, d_dp_new, d_chi_new, W.cep,
                         W.mode, d_eta_dt, W.D, s);
        apply(op, vref, 1, d_dd, n3, W.Ex, n3, false, s);
        hipLaunchKernelGGL(k_np_centroid, dim3(ge), dim3(256), 0, s, ne, F.conn.as<int32_t>(), d_dpn, W.dpress);
        hipLaunchKernelGGL(k_coupled_mech_residual, dim3(ge), dim3(256), 0, s, ne, d_dT0, d_t_new, d_t, W.Ex,
                           W.dpress, d_eta_dt, d_dd, d_dd_prev, W.r);
        flow_coefficients(F, d_w0, d_dn_start, d_dd, cs, cs + ne, cs + 2 * ne, cs + 3 * ne, s);
        flow_assemble(F, cs, cs + 2 * ne, W.S, W.L, s);
        hipLaunchKernelGGL(k_flow_residual, dim3(gn), dim3(256), 0, s, nn, F.nptr.as<int64_t>(), F.nel.as<int32_t>(),
                           F.area.as<double>(), d_dd, F.rowptr.as<int64_t>(), F.col.as<int32_t>(), W.S, W.L, d_dpn,
                           W.pnpo, d_source, dt, W.r + n3);
        HM_CHECK_HIP(hipGetLastError());
        std::vector<double> a, b;
        C.dots(W.r, 1, W.r, a);   // the full vector; split by a second pass over the flow part
        hipLaunchKernelGGL(k_mdot, dim3((unsigned)((nn + kRedBlock * kRedPer - 1) / (kRedBlock * kRedPer)), 1),
                           dim3(kRedBlock), 0, s, nn, W.r + n3, nn, 1, W.r + n3, W.partial,
                           (int)((nn + kRedBlock * kRedPer - 1) / (kRedBlock * kRedPer)));
        {
            const int64_t nb = (nn + kRedBlock * kRedPer - 1) / (kRedBlock * kRedPer);
            std::vector<double> part(nb);
            HM_CHECK_HIP(hipMemcpyAsync(part.data(), W.partial, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
            HM_CHECK_HIP(hipStreamSynchronize(s));
            double sf = 0.0;
            for (double x : part) sf += x;
            b.assign(1, sf);
        }
        const double rf2 = b[0], rm2 = std::max(0.0, a[0] - b[0]);
        hm_.push_back(std::sqrt(rm2));
        hf_.push_back(std::sqrt(rf2));
        hist.push_back(std::sqrt(C.sR[0] * C.sR[0] * rm2 + C.sR[1] * C.sR[1] * rf2));
        const bool done = hist.back() <= std::max(o.rtol * hist.front(), o.atol);
        if (done || k == o.max_newton || !std::isfinite(hist.back())) break;
        // Jacobian: tangent of A11, flow blocks, S~ and its ILU(0)
        tangent_set(op, W.D, nullptr, s);
        if (o.schur == 1) ilu_pc_prepare(op, o.inner.ilu_fraction == 0.0 ? 0.01 : o.inner.ilu_fraction, s);
        hipLaunchKernelGGL(k_flow_a21, dim3(ge), dim3(256), 0, s, ne, F.conn.as<int32_t>(), F.area.as<double>(),
                           F.stiff.as<double>(), cs + ne, cs + 3 * ne, d_dpn, W.pnpo, dt, W.a21);
        hipLaunchKernelGGL(k_flow_schur, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, nnz,
                           F.cptr.as<int64_t>(), F.cel.as<int32_t>(), F.cab.as<uint8_t>(), W.S, W.L, dt, W.a21,
                           op.d_pc_diag.as<double>(), W.A22, W.St);
        DevBuf status(sizeof(int));
        HM_CHECK_HIP(hipMemsetAsync(status.get(), 0, sizeof(int), s));
        for (int c = 0; c < F.n_colors; ++c) {
            const int n = (int)(F.color_begin[c + 1] - F.color_begin[c]);
            hipLaunchKernelGGL(k_node_ilu_factor, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s,
                               F.order.as<int32_t>() + F.color_begin[c], n, F.pos.as<int32_t>(),
                               F.rowptr.as<int64_t>(), F.col.as<int32_t>(), F.diag.as<int64_t>(), W.Sf,
                               status.as<int>());
        }
        HM_CHECK_HIP(hipGetLastError());
        int hs = 0;
        HM_CHECK_HIP(hipMemcpyAsync(&hs, status.get(), sizeof(int), hipMemcpyDeviceToHost, s));
        HM_CHECK_HIP(hipStreamSynchronize(s));
        HM_REQUIRE(hs == 0, HM_EINVAL, "ILU(0) of the approximate Schur complement met a zero pivot");
        // solve J delta = -r on the scaled system: b^ = -diag(sR) r
        hipLaunchKernelGGL(k_axpy, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s, n3, -C.sR[0], W.r, W.w, 0);
        hipLaunchKernelGGL(k_axpy, dim3(gn), dim3(256), 0, s, nn, -C.sR[1], W.r + n3, W.w + n3, 0);
        // b^ lives in W.w; fgmres uses W.w as scratch only after the first cycle, so keep b^ in r
        HM_CHECK_HIP(hipMemcpyAsync(W.r, W.w, sizeof(double) * W.ntot, hipMemcpyDeviceToDevice, s));
        C.inner_its = 0;
        C.schur_its = 0;
        const int its = C.fgmres(W.r, o.outer_rtol, o.outer_restart, o.outer_max_iter);
        outer.push_back(its);
        inner.push_back(C.inner_its);
        schur_its.push_back(C.schur_its);
        // unknowns += diag(1/sX) x^
        hipLaunchKernelGGL(k_axpy, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s, n3, 1.0 / C.sX[0], W.x, d_dd,
                           1);
        hipLaunchKernelGGL(k_axpy, dim3(gn), dim3(256), 0, s, nn, 1.0 / C.sX[1], W.x + n3, d_dpn, 1);
        HM_CHECK_HIP(hipGetLastError());
    }
    tangent_set(op, W.D, nullptr, s);
    const bool converged = hist.back() <= std::max(o.rtol * hist.front(), o.atol);
    if (rep) {
        *rep = hm_coupled_report{};
        rep->iterations = (int)outer.size();
        rep->converged = converged ? 1 : 0;
        rep->n_history = (int)std::min<size_t>(hist.size(), 64);
        for (int i = 0; i < rep->n_history; ++i) {
            rep->residual[i] = hist[i];
            rep->residual_mech[i] = hm_[i];
            rep->residual_flow[i] = hf_[i];
        }
        for (size_t i = 0; i < outer.size() && i < 64; ++i) {
            rep->outer_iterations[i] = outer[i];
            rep->inner_iterations[i] = inner[i];
            rep->schur_iterations[i] = schur_its[i];
        }
        std::vector<int32_t> hmode(ne);
        HM_CHECK_HIP(hipMemcpyAsync(hmode.data(), W.mode, sizeof(int32_t) * ne, hipMemcpyDeviceToHost, s));
        HM_CHECK_HIP(hipStreamSynchronize(s));
        for (int32_t m : hmode)
            if (m >= 0 && m < 5) rep->modes[m]++;
        rep->ms = now_ms() - t0;
    }
    return converged ? HM_OK : HM_ENOTCONV;
}

double scale_update(double L_old, double L_new, double alpha, double rho_min, double rho_max)
{
    HM_REQUIRE(L_old > 0.0 && L_new >= 0.0, HM_EINVAL, "scales must be positive");
    HM_REQUIRE(alpha >= 0.0 && alpha <= 1.0 && rho_min > 0.0 && rho_min <= 1.0 && rho_max >= 1.0, HM_EINVAL,
               "alpha in [0, 1], 0 < rho_min <= 1 <= rho_max");
    const double smooth = alpha * L_old + (1.0 - alpha) * L_new;
    return L_old * std::max(rho_min, std::min(smooth / L_old, rho_max));
}

}  // namespace hm
