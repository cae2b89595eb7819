// Krylov solve of the tangent system A11 x = b (paper Sec. 3.1.1 mechanical
// Jacobian A11 = E - eta/dt - C^ep; Sec. 3.3.1: the A11 systems are solved
// iteratively, BiCGSTAB or GMRES, with a diagonal/block preconditioner).
//
// Restarted GMRES(m) with right preconditioning, x0 = 0, Arnoldi by
// classical Gram-Schmidt with delayed reorthogonalisation (one projection
// pass and one update pass over the basis per step), all vector arithmetic
// in FP64 on the GPU.  nrhs independent systems advance in lock-step so
// that every operator application streams the H-matrix once for all of them.  The
// Hessenberg least-squares problem (at most (m+1) x m per column) is solved
// on the host with Givens rotations; only O(m) scalars per column cross to
// the host per iteration.  With refinement, an outer loop computes the
// FP64 residual with the FP64 reference operator and solves for the
// correction with the operator's own (lower) precisions.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "hm_op.hpp"

namespace hm {

// z = M^-1 v for every column (block 3x3, point Jacobi or identity)
__global__ void k_precond(int kind, int64_t ne, int nrhs, const double* __restrict__ v, int64_t ldv,
                          double* __restrict__ z, int64_t ldz, const double* __restrict__ pcb,
                          const double* __restrict__ pcd)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ne * nrhs) return;
    int c = (int)(idx / ne);
    int64_t e = idx - (int64_t)c * ne;
    const double* x = v + c * ldv + 3 * e;
    double* o = z + c * ldz + 3 * e;
    double x0 = x[0], x1 = x[1], x2 = x[2];
    if (kind == HM_PC_BLOCK3) {
        const double* B = pcb + 9 * e;
        o[0] = B[0] * x0 + B[1] * x1 + B[2] * x2;
        o[1] = B[3] * x0 + B[4] * x1 + B[5] * x2;
        o[2] = B[6] * x0 + B[7] * x1 + B[8] * x2;
    } else if (kind == HM_PC_JACOBI) {
        o[0] = pcd[3 * e] * x0;
        o[1] = pcd[3 * e + 1] * x1;
        o[2] = pcd[3 * e + 2] * x2;
    } else {
        o[0] = x0;
        o[1] = x1;
        o[2] = x2;
    }
}

// Basis vectors are streamed (read once per pass, far larger than the
// caches): their loads are non-temporal; the few vectors a pass re-reads
// (its targets) keep the default policy.
constexpr int kDotChunk = 4096;
constexpr int kDotGroup = 4;  // basis vectors per workgroup of the dot kernel

// Dot products of J basis vectors A_0 .. A_{J-1} (A_j[c] = A + j strideJ +
// c ldA) with NT target vectors (u, and w when NT = 2), every column c;
// each workgroup covers kDotChunk rows of one column and kDotGroup basis
// vectors, so the targets are read once per group.
// partial[((t J + j) nrhs + c) nchunk + chunk] = sum over the chunk.
template <int NT>
__global__ __launch_bounds__(256) void k_mdot_partial(int nrhs, int64_t n, const double* __restrict__ A,
                                                      int64_t strideJ, int64_t ldA, int J,
                                                      const double* __restrict__ u, int64_t ldu,
                                                      const double* __restrict__ w, int64_t ldw,
                                                      double* __restrict__ partial, int nchunk)
{
    const int c = blockIdx.y, j0 = blockIdx.z * kDotGroup;
    const int nj = min(kDotGroup, J - j0);
    const int64_t x0 = (int64_t)blockIdx.x * kDotChunk;
    const int64_t x1 = min(n, x0 + kDotChunk);
    const double* a = A + (int64_t)j0 * strideJ + (int64_t)c * ldA;
    const double* uc = u + (int64_t)c * ldu;
    const double* wc = NT == 2 ? w + (int64_t)c * ldw : nullptr;
    double acc[NT][kDotGroup];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int q = 0; q < kDotGroup; ++q) acc[t][q] = 0.0;
    for (int64_t x = x0 + threadIdx.x; x < x1; x += blockDim.x) {
        const double ux = uc[x];
        const double wx = NT == 2 ? wc[x] : 0.0;
#pragma unroll
        for (int q = 0; q < kDotGroup; ++q)
            if (q < nj) {
                const double v = __builtin_nontemporal_load(&a[(int64_t)q * strideJ + x]);
                acc[0][q] += v * ux;
                if (NT == 2) acc[NT - 1][q] += v * wx;
            }
    }
    __shared__ double red[4][NT * kDotGroup];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int q = 0; q < kDotGroup; ++q) {
            double v = acc[t][q];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) red[wave][t * kDotGroup + q] = v;
        }
    __syncthreads();
    if (threadIdx.x < NT * kDotGroup) {
        const int t = threadIdx.x / kDotGroup, q = threadIdx.x - t * kDotGroup;
        if (q < nj)
            partial[((int64_t)(t * J + j0 + q) * nrhs + c) * nchunk + blockIdx.x] =
                (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
    }
}

__global__ void k_dot_final(int np, int nchunk, const double* __restrict__ partial, double* __restrict__ out)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    double s = 0.0;
    for (int k = 0; k < nchunk; ++k) s += partial[(int64_t)p * nchunk + k];
    out[p] = s;
}

// out[c] = sum_j A_j[c] h[j][c]  (the solution update: x += M^-1 V y)
__global__ void k_combine(int J, int nrhs, int64_t n, const double* __restrict__ A, int64_t strideJ, int64_t ldA,
                          const double* __restrict__ h, double* __restrict__ w, int64_t ldw)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * nrhs) return;
    int c = (int)(idx / n);
    int64_t x = idx - (int64_t)c * n;
    double s = 0.0;
    for (int j = 0; j < J; ++j) s += __builtin_nontemporal_load(&A[j * strideJ + c * ldA + x]) * h[j * nrhs + c];
    w[c * ldw + x] = s;
}

// One pass of the delayed reorthogonalisation (basis slots of V: q_0 ..
// q_{j-1} final, u = slot j tentative, w = slot j + 1 = A M^-1 u).  For
// column c with coefficients cf = [s (j), d (j), e, gq, gw]:
//   slot j     <- (u - sum_i s_i q_i) gq          (u reorthogonalised: q_j)
//   slot j + 1 <- (w - sum_i d_i q_i - e u) gw    (next tentative vector)
// gq = gw = 0 zeroes a column that has finished.  Rows are independent, so
// the update is in place.
__global__ __launch_bounds__(256) void k_dcgs2_update(int j, int64_t n, double* V, int64_t strideJ,
                                                      const double* __restrict__ coef)
{
    const int c = blockIdx.y;
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const double* cf = coef + (int64_t)c * (2 * j + 3);
    const double e = cf[2 * j], gq = cf[2 * j + 1], gw = cf[2 * j + 2];
    double* col = V + (int64_t)c * n + x;
    double* uq = col + (int64_t)j * strideJ;
    double* wn = uq + strideJ;
    if (gq == 0.0 && gw == 0.0) {
        *uq = 0.0;
        *wn = 0.0;
        return;
    }
    double a1 = 0.0, a2 = 0.0;
    for (int i = 0; i < j; ++i) {
        const double q = __builtin_nontemporal_load(&col[(int64_t)i * strideJ]);
        a1 += cf[i] * q;
        a2 += cf[j + i] * q;
    }
    const double u = *uq, w = *wn;
    *uq = (u - a1) * gq;
    *wn = (w - a2 - e * u) * gw;
}

// y[c] = alpha[c] * x[c]  (alpha = 0 where scale is not finite or zero)
// (x and y may be the same vectors)
__global__ void k_scale(int nrhs, int64_t n, const double* x, int64_t ldx, const double* __restrict__ inv, double* y,
                        int64_t ldy)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * nrhs) return;
    int c = (int)(idx / n);
    int64_t i = idx - (int64_t)c * n;
    y[c * ldy + i] = x[c * ldx + i] * inv[c];
}

// y = a - b  or  y += b
__global__ void k_axpby(int nrhs, int64_t n, const double* __restrict__ a, int64_t lda, double alpha,
                        const double* __restrict__ b, int64_t ldb, double beta, double* __restrict__ y, int64_t ldy)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * nrhs) return;
    int c = (int)(idx / n);
    int64_t i = idx - (int64_t)c * n;
    y[c * ldy + i] = alpha * a[c * lda + i] + beta * b[c * ldb + i];
}

double* Op::solve_workspace(hipStream_t s, size_t bytes, int purpose)
{
    std::lock_guard<std::mutex> g(solve_mu);
    std::unique_ptr<DevBuf>& b = solve_ws[{s, purpose}];
    if (!b) b.reset(new DevBuf());
    if (b->bytes() < bytes) {
        HM_CHECK_HIP(hipStreamSynchronize(s));
        b->alloc(bytes);
    }
    return b->as<double>();
}

namespace {

struct Krylov {
    Op& op;
    hipStream_t s;
    int nrhs;
    int64_t n;
    int m;
    int pc;
    double *V, *W, *Z, *R, *D, *partial, *hbuf, *coef, *dinv;  // device
    int nchunk;
    std::vector<double> h_host;

    Krylov(Op& o, hipStream_t st, int nr, int restart, int precond) : op(o), s(st), nrhs(nr), m(restart), pc(precond)
    {
        n = 3 * op.ne;
        nchunk = (int)((n + kDotChunk - 1) / kDotChunk);
        const size_t vec = (size_t)nrhs * n;
        const size_t nh = (size_t)2 * (m + 2) * nrhs;  // dot results: two targets, up to m + 2 basis vectors
        const size_t ncoef = (size_t)(2 * m + 3) * nrhs;
        size_t need = sizeof(double) * (vec * (m + 1) + 4 * vec + nh * nchunk + nh + ncoef + nrhs);
        double* p = op.solve_workspace(s, need);
        V = p;
        p += vec * (m + 1);
        W = p;
        p += vec;
        Z = p;
        p += vec;
        R = p;
        p += vec;
        D = p;
        p += vec;
        partial = p;
        p += nh * nchunk;
        hbuf = p;
        p += nh;
        coef = p;
        p += ncoef;
        dinv = p;
        h_host.resize(nh);
    }

    unsigned g1(int64_t total) const { return (unsigned)((total + 255) / 256); }

    // hbuf[(t J + j) nrhs + c] = A_j[c] . u[c] (t = 0) and A_j[c] . w[c] (t = 1, when w is given), j < J;
    // A_j = A + j nrhs n, all vectors [nrhs][n]
    void dots(const double* A, int J, const double* u, const double* w = nullptr)
    {
        const dim3 grid(nchunk, nrhs, (J + kDotGroup - 1) / kDotGroup);
        if (w)
            hipLaunchKernelGGL(k_mdot_partial<2>, grid, dim3(256), 0, s, nrhs, n, A, (int64_t)nrhs * n, n, J, u, n, w,
                               n, partial, nchunk);
        else
            hipLaunchKernelGGL(k_mdot_partial<1>, grid, dim3(256), 0, s, nrhs, n, A, (int64_t)nrhs * n, n, J, u, n,
                               u, n, partial, nchunk);
        const int np = (w ? 2 : 1) * J * nrhs;
        hipLaunchKernelGGL(k_dot_final, dim3((np + 255) / 256), dim3(256), 0, s, np, nchunk, partial, hbuf);
    }
    // copy the first entries * nrhs dot results to the host
    void fetch(int entries)
    {
        HM_CHECK_HIP(
            hipMemcpyAsync(h_host.data(), hbuf, sizeof(double) * entries * nrhs, hipMemcpyDeviceToHost, s));
        HM_CHECK_HIP(hipStreamSynchronize(s));
    }
    void precond(const double* v, double* z)
    {
        if (pc == HM_PC_LEARNED) {
            learned_apply(op, nrhs, v, n, z, n, s);
            return;
        }
        if (pc == HM_PC_LEAF) {
            leaf_pc_apply(op, nrhs, v, n, z, n, s);
            return;
        }
        if (pc == HM_PC_ILU) {
            ilu_pc_apply(op, nrhs, v, n, z, n, s);
            return;
        }
        hipLaunchKernelGGL(k_precond, dim3(g1(op.ne * nrhs)), dim3(256), 0, s, pc, op.ne, nrhs, v, n, z, n,
                           op.d_pc_block.as<double>(), op.d_pc_diag.as<double>());
    }
    void matvec(const Variant& v, const double* x, double* y) { apply(op, v, nrhs, x, n, y, n, true, s); }
};

// Givens least squares per column
struct Ls {
    int m;
    std::vector<double> H;  // (m+1) x m column-major per iteration column
    std::vector<double> cs, sn, g;
    explicit Ls(int mm) : m(mm), H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1, 0.0) {}
    void reset(double beta)
    {
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
    }
    // the residual estimate column j (h[0..j+1]) would give, state unchanged
    double peek(int j, const double* h) const
    {
        // only entry j of the rotated column is needed; each rotation i
        // mixes entries i and i + 1, so carry entry i + 1 forward
        double carry = h[0];
        for (int i = 0; i < j; ++i) carry = -sn[i] * carry + cs[i] * h[i + 1];
        const double r = std::hypot(carry, h[j + 1]);
        return r == 0.0 ? 0.0 : std::fabs(h[j + 1] / r * g[j]);
    }
    // add column j (h[0..j+1]); returns |g[j+1]|
    double push(int j, const double* h)
    {
        double* col = &H[(size_t)j * (m + 1)];
        for (int i = 0; i <= j + 1; ++i) col[i] = h[i];
        for (int i = 0; i < j; ++i) {
            double t = cs[i] * col[i] + sn[i] * col[i + 1];
            col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
            col[i] = t;
        }
        double a = col[j], b = col[j + 1];
        double r = std::hypot(a, b);
        if (r == 0.0) {
            cs[j] = 1.0;
            sn[j] = 0.0;
        } else {
            cs[j] = a / r;
            sn[j] = b / r;
        }
        col[j] = r;
        col[j + 1] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        return std::fabs(g[j + 1]);
    }
    void solve(int k, double* y) const
    {
        for (int i = k - 1; i >= 0; --i) {
            double sum = g[i];
            for (int l = i + 1; l < k; ++l) sum -= H[(size_t)l * (m + 1) + i] * y[l];
            double d = H[(size_t)i * (m + 1) + i];
            y[i] = d != 0.0 ? sum / d : 0.0;
        }
    }
};

struct GmresResult {
    int iterations = 0;
    bool converged = false;
    bool nonfinite = false;  // a NaN or infinity reached the Arnoldi process
};

// Solve A x = b for every column with the operator variant v; x starts at 0.
// Convergence: true residual (same variant) <= tol * bnorm[c], checked at
// restarts and when the Arnoldi estimate says so.
//
// Arnoldi by classical Gram-Schmidt with delayed reorthogonalisation
// (DCGS2: Swirydowicz et al., Numer. Linear Algebra Appl. 2021; Bielich et
// al., Parallel Comput. 2022).  Step j multiplies the tentative vector u
// (slot j: projected once, not yet reorthogonalised) and then, in one pass
// over the basis, takes the dot products of q_0 .. q_{j-1}, u and w = A M^-1 u
// with u and with w.  From them:
//   s = Q^T u, rho^2 = u.u - s.s        reorthogonalise u: q_j = (u - Q s) / rho,
//                                       which finishes column j - 1
//                                       (h += beta s, h_{j,j-1} = beta rho);
//   A M^-1 q_j = (w - Q_{j+1} H s) / rho gives column j and, with the
//   Pythagorean norm, the next tentative vector
//   u' = (w - Q d - e u) / (rho beta').
// One update pass writes q_j and u'.  Each step thus reads the basis twice
// (CGS2 reads it four times) with one host synchronisation.  A column is
// finished with one more dot pass when the step's estimate says the system
// has converged and at the end of a cycle.
GmresResult gmres(Krylov& K, const Variant& v, const double* b, double* x, const std::vector<double>& bnorm,
                  double tol, int max_iter, std::vector<double>& hist, double hist_scale)
{
    const int nrhs = K.nrhs, m = K.m;
    const int64_t n = K.n;
    const int64_t vs = (int64_t)nrhs * n;  // basis slot stride
    hipStream_t s = K.s;
    GmresResult res;
    HM_CHECK_HIP(hipMemsetAsync(x, 0, sizeof(double) * vs, s));
    std::vector<Ls> ls(nrhs, Ls(m));
    // Hessenberg columns before rotation, per right-hand side ((m + 1) x m, column-major)
    std::vector<double> Hf((size_t)nrhs * m * (m + 1));
    auto Hc = [&](int c, int j) { return &Hf[((size_t)c * m + j) * (m + 1)]; };
    std::vector<double> bet(nrhs), inv(nrhs), y((size_t)m * nrhs), coef, p(m + 1), col(m + 1);
    std::vector<int> ncols(nrhs);
    std::vector<char> conv(nrhs, 0), active(nrhs, 0);
    int total = 0;
    bool first = true;
    while (true) {
        // r = b - A x
        if (first) {
            HM_CHECK_HIP(hipMemcpyAsync(K.R, b, sizeof(double) * vs, hipMemcpyDeviceToDevice, s));
        } else {
            K.matvec(v, x, K.W);
            hipLaunchKernelGGL(k_axpby, dim3(K.g1(vs)), dim3(256), 0, s, nrhs, n, b, n, 1.0, K.W, n, -1.0, K.R, n);
        }
        first = false;
        K.dots(K.R, 1, K.R);
        K.fetch(1);
        for (int c = 0; c < nrhs; ++c)
            if (!std::isfinite(K.h_host[c])) res.nonfinite = true;
        if (res.nonfinite) break;
        bool all = true;
        for (int c = 0; c < nrhs; ++c) {
            const double beta = std::sqrt(std::max(0.0, K.h_host[c]));
            conv[c] = beta <= tol * bnorm[c];
            all = all && conv[c];
            ls[c].reset(beta);
            inv[c] = (beta > 0.0 && !conv[c]) ? 1.0 / beta : 0.0;
            active[c] = !conv[c];
            ncols[c] = 0;
            bet[c] = 1.0;
        }
        if (all) {
            res.converged = true;
            break;
        }
        if (total >= max_iter) break;
        std::fill(Hf.begin(), Hf.end(), 0.0);
        HM_CHECK_HIP(hipMemcpyAsync(K.dinv, inv.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_scale, dim3(K.g1(vs)), dim3(256), 0, s, nrhs, n, K.R, n, K.dinv, K.V, n);
        for (int j = 0; j < m && total < max_iter; ++j) {
            double* Vj = K.V + (size_t)j * vs;
            double* Vn = Vj + vs;
            K.precond(Vj, K.Z);
            K.matvec(v, K.Z, Vn);
            ++total;
            K.dots(K.V, j + 2, Vj, Vn);
            K.fetch(2 * (j + 2));
            for (size_t q = 0; q < (size_t)2 * (j + 2) * nrhs; ++q)
                if (!std::isfinite(K.h_host[q])) res.nonfinite = true;
            if (res.nonfinite) {
                res.iterations = total;
                return res;
            }
            const double* G0 = K.h_host.data();                            // basis . u
            const double* G1 = K.h_host.data() + (size_t)(j + 2) * nrhs;   // basis . w
            const size_t nc = (size_t)(2 * j + 3);
            coef.assign(nc * nrhs, 0.0);
            double worst = 0.0;
            bool any = false, all_tentative = true;
            for (int c = 0; c < nrhs; ++c) {
                if (!active[c]) continue;
                auto su = [&](int i) { return G0[(size_t)i * nrhs + c]; };  // q_i . u (u . u at i = j)
                auto sw = [&](int i) { return G1[(size_t)i * nrhs + c]; };  // q_i . w (u . w at j, w . w at j + 1)
                const double a = su(j);
                double ss = 0.0;
                for (int i = 0; i < j; ++i) ss += su(i) * su(i);
                const double rho2 = a - ss;
                const double rho = (a > 0.0 && rho2 > 1e-30 * a) ? std::sqrt(rho2) : 0.0;
                if (j > 0) {
                    double* hp = Hc(c, j - 1);
                    for (int i = 0; i < j; ++i) hp[i] += bet[c] * su(i);
                    hp[j] = bet[c] * rho;
                    const double est = ls[c].push(j - 1, hp);
                    ncols[c] = j;
                    if (est <= tol * bnorm[c] || rho == 0.0) {
                        active[c] = 0;
                        continue;
                    }
                } else if (rho == 0.0) {
                    active[c] = 0;
                    continue;
                }
                // p = H s over the finished columns 0 .. j - 1 (rows 0 .. j)
                std::fill(p.begin(), p.begin() + j + 1, 0.0);
                for (int k = 0; k < j; ++k) {
                    const double* hk = Hc(c, k);
                    for (int i = 0; i <= k + 1; ++i) p[i] += hk[i] * su(k);
                }
                double sz = 0.0;
                for (int i = 0; i < j; ++i) sz += su(i) * sw(i);
                const double qw = (sw(j) - sz) / rho;  // q_j . w
                double* h = Hc(c, j);
                double pq = 0.0, pp = 0.0, hh = 0.0;
                for (int i = 0; i < j; ++i) {
                    h[i] = (sw(i) - p[i]) / rho;
                    pq += p[i] * sw(i);
                }
                h[j] = (qw - p[j]) / rho;
                pq += p[j] * qw;
                for (int i = 0; i <= j; ++i) {
                    pp += p[i] * p[i];
                    hh += h[i] * h[i];
                }
                const double wt2 = (sw(j + 1) - 2.0 * pq + pp) / (rho * rho);  // |A M^-1 q_j|^2
                const double bn = std::sqrt(std::max(wt2 - hh, 1e-24 * wt2));
                double* cf = &coef[(size_t)c * nc];
                const double cj = p[j] + rho * h[j];
                for (int i = 0; i < j; ++i) {
                    cf[i] = su(i);
                    cf[j + i] = p[i] + rho * h[i] - cj * su(i) / rho;
                }
                cf[2 * j] = cj / rho;
                cf[2 * j + 1] = 1.0 / rho;
                if (!(bn > 0.0) || !std::isfinite(bn)) {
                    // A M^-1 q_j lies in the basis: column j is final with a zero subdiagonal
                    h[j + 1] = 0.0;
                    ls[c].push(j, h);
                    ncols[c] = j + 1;
                    active[c] = 0;
                    continue;
                }
                cf[2 * j + 2] = 1.0 / (rho * bn);
                bet[c] = bn;
                h[j + 1] = bn;  // tentative until u' is reorthogonalised
                const double est = ls[c].peek(j, h);
                worst = std::max(worst, est / bnorm[c]);
                any = true;
                all_tentative = all_tentative && est <= tol * bnorm[c];
            }
            HM_CHECK_HIP(hipMemcpyAsync(K.coef, coef.data(), sizeof(double) * coef.size(), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_dcgs2_update, dim3((unsigned)((n + 255) / 256), nrhs), dim3(256), 0, s, j, n, K.V, vs,
                               K.coef);
            if (hist.size() < 1024) hist.push_back(worst * hist_scale);
            if (!any) break;
            const bool last = j + 1 == m || total >= max_iter;
            if (!last && !all_tentative) continue;
            // finish column j: reorthogonalise the tentative vector (slot j + 1)
            K.dots(K.V, j + 2, Vn);
            K.fetch(j + 2);
            for (size_t q = 0; q < (size_t)(j + 2) * nrhs; ++q)
                if (!std::isfinite(K.h_host[q])) res.nonfinite = true;
            if (res.nonfinite) {
                res.iterations = total;
                return res;
            }
            bool remaining = false;
            for (int c = 0; c < nrhs; ++c) {
                if (!active[c]) continue;
                const double* h = Hc(c, j);
                double ss = 0.0;
                for (int i = 0; i <= j; ++i) {
                    const double si = K.h_host[(size_t)i * nrhs + c];
                    col[i] = h[i] + bet[c] * si;
                    ss += si * si;
                }
                col[j + 1] = bet[c] * std::sqrt(std::max(0.0, K.h_host[(size_t)(j + 1) * nrhs + c] - ss));
                const double est = ls[c].peek(j, col.data());
                if (last || est <= tol * bnorm[c]) {
                    std::copy(col.begin(), col.begin() + j + 2, Hc(c, j));
                    ls[c].push(j, col.data());
                    ncols[c] = j + 1;
                    active[c] = 0;
                } else {
                    remaining = true;  // estimate was optimistic: keep going, step j + 1 finishes column j
                }
            }
            if (!remaining) break;
        }
        // x += M^-1 Q y  (columns that had converged before this cycle get y = 0)
        int J = 0;
        std::fill(y.begin(), y.end(), 0.0);
        for (int c = 0; c < nrhs; ++c) {
            if (conv[c] || ncols[c] == 0) continue;
            const int k = ncols[c];
            std::vector<double> yc(k);
            ls[c].solve(k, yc.data());
            for (int i = 0; i < k; ++i) y[(size_t)i * nrhs + c] = yc[i];
            J = std::max(J, k);
        }
        if (J > 0) {
            HM_CHECK_HIP(hipMemcpyAsync(K.hbuf, y.data(), sizeof(double) * J * nrhs, hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_combine, dim3(K.g1(vs)), dim3(256), 0, s, J, nrhs, n, K.V, vs, n, K.hbuf, K.W, n);
            K.precond(K.W, K.Z);
            hipLaunchKernelGGL(k_axpby, dim3(K.g1(vs)), dim3(256), 0, s, nrhs, n, x, n, 1.0, K.Z, n, 1.0, x, n);
        }
    }
    res.iterations = total;
    return res;
}

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

void precond_apply(Op& op, int kind, int nrhs, const double* R, int64_t ldr, double* Z, int64_t ldz, hipStream_t s)
{
    HM_REQUIRE(nrhs >= 1 && nrhs <= kNrhs, HM_EINVAL, "nrhs must be in [1, 16]");
    HM_REQUIRE(kind >= HM_PC_NONE && kind <= HM_PC_ILU, HM_EINVAL, "unknown preconditioner");
    HM_REQUIRE(ldr >= 3 * op.ne && ldz >= 3 * op.ne, HM_EINVAL, "leading dimension below 3N");
    HM_REQUIRE(R && Z, HM_EINVAL, "null vector pointer");
    HM_REQUIRE(kind != HM_PC_LEARNED || op.lp.attached, HM_EINVAL, "no learned correction is attached");
    if (kind == HM_PC_LEARNED) {
        learned_apply(op, nrhs, R, ldr, Z, ldz, s);
    } else if (kind == HM_PC_LEAF) {
        leaf_pc_prepare(op, s);
        leaf_pc_apply(op, nrhs, R, ldr, Z, ldz, s);
    } else if (kind == HM_PC_ILU) {
        // the factors of the last solve's fraction, or of the default 1 %
        ilu_pc_prepare(op, op.ilu.fraction > 0.0 ? op.ilu.fraction : 0.01, s);
        ilu_pc_apply(op, nrhs, R, ldr, Z, ldz, s);
    } else {
        hipLaunchKernelGGL(k_precond, dim3((unsigned)((op.ne * nrhs + 255) / 256)), dim3(256), 0, s, kind, op.ne,
                           nrhs, R, ldr, Z, ldz, op.d_pc_block.as<double>(), op.d_pc_diag.as<double>());
        HM_CHECK_HIP(hipGetLastError());
    }
    HM_CHECK_HIP(hipStreamSynchronize(s));
}

hm_status solve(Op& op, const hm_solve_opts& o, int nrhs, const double* d_B, int64_t ldb, double* d_X, int64_t ldx,
                hm_solve_report* rep, hipStream_t s)
{
    HM_REQUIRE(nrhs >= 1 && nrhs <= kNrhs, HM_EINVAL, "nrhs must be in [1, 16]");
    HM_REQUIRE(o.restart >= 1 && o.restart <= 256, HM_EINVAL, "restart must be in [1, 256]");
    HM_REQUIRE(o.max_iter >= 1, HM_EINVAL, "max_iter must be positive");
    HM_REQUIRE(o.rtol > 0.0 && o.rtol < 1.0, HM_EINVAL, "rtol must be in (0, 1)");
    HM_REQUIRE(o.precond >= HM_PC_NONE && o.precond <= HM_PC_ILU, HM_EINVAL, "unknown preconditioner");
    HM_REQUIRE(ldb >= 3 * op.ne && ldx >= 3 * op.ne, HM_EINVAL, "leading dimension below 3N");
    HM_REQUIRE(d_B && d_X, HM_EINVAL, "null vector pointer");
    HM_REQUIRE(!o.refine || op.ref || op.main.near_prec == HM_F64, HM_EINVAL,
               "refinement needs an FP64 reference copy (keep_f64_reference)");
    double t0 = now_ms();
    Krylov K(op, s, nrhs, o.restart, o.precond);
    const int64_t n = K.n;
    // contiguous copies of B and X ([nrhs][n])
    double* B = K.D;  // reuse D buffer for b
    HM_CHECK_HIP(hipMemcpy2DAsync(B, n * sizeof(double), d_B, ldb * sizeof(double), n * sizeof(double), nrhs,
                                  hipMemcpyDeviceToDevice, s));
    K.dots(B, 1, B);
    K.fetch(1);
    std::vector<double> bnorm(nrhs);
    for (int c = 0; c < nrhs; ++c) bnorm[c] = std::sqrt(std::max(0.0, K.h_host[c]));
    for (int c = 0; c < nrhs; ++c)
        if (bnorm[c] == 0.0) bnorm[c] = 1.0;  // zero right-hand side: x = 0 is exact
    std::vector<double> hist;
    const Variant& ref = op.ref_variant();
    int iters = 0, sweeps = 0;
    bool ok = false, nonfinite = false;
    DevBuf xbuf((size_t)nrhs * n * sizeof(double)), rbuf((size_t)nrhs * n * sizeof(double)),
        dbuf((size_t)nrhs * n * sizeof(double)), tbuf((size_t)nrhs * n * sizeof(double));
    double* X = xbuf.as<double>();
    std::vector<double> relres(nrhs, 0.0);
    auto true_residual = [&](const double* x, double* r) {
        apply(op, ref, nrhs, x, n, tbuf.as<double>(), n, true, s);
        hipLaunchKernelGGL(k_axpby, dim3(K.g1(n * nrhs)), dim3(256), 0, s, nrhs, n, B, n, 1.0, tbuf.as<double>(), n,
                           -1.0, r, n);
        K.dots(r, 1, r);
        K.fetch(1);
        double worst = 0.0;
        for (int c = 0; c < nrhs; ++c) {
            relres[c] = std::sqrt(std::max(0.0, K.h_host[c])) / bnorm[c];
            worst = std::isnan(relres[c]) ? relres[c] : std::max(worst, relres[c]);
        }
        return worst;
    };
    // one complete solve from x = 0 with preconditioner pc
    auto attempt = [&](int pc) {
        K.pc = pc;
        iters = 0;
        sweeps = 0;
        ok = false;
        nonfinite = false;
        hist.clear();
        if (!o.refine) {
            GmresResult g = gmres(K, op.main, B, X, bnorm, o.rtol, o.max_iter, hist, 1.0);
            iters = g.iterations;
            nonfinite = g.nonfinite;
            double r = true_residual(X, rbuf.as<double>());
            nonfinite = nonfinite || !std::isfinite(r);
            ok = !nonfinite && r <= o.rtol;
            return;
        }
        // FP64 iterative refinement: x += A_lp^-1 (b - A_ref x)
        HM_CHECK_HIP(hipMemsetAsync(X, 0, sizeof(double) * nrhs * n, s));
        HM_CHECK_HIP(hipMemcpyAsync(rbuf.get(), B, sizeof(double) * nrhs * n, hipMemcpyDeviceToDevice, s));
        double r = 1.0;
        // A sweep cannot reduce the FP64 residual by more than the
        // low-precision operator's own error allows (about 1e-2 with BF16
        // factors, 1e-5 with FP32), so by default the inner solve stops there.
        const double inner = o.inner_rtol > 0.0 ? o.inner_rtol : (op.main.far_prec == HM_BF16 || op.main.far_prec == HM_BF16_1 ? 1e-2 : 1e-5);
        while (sweeps < o.max_refine && iters < o.max_iter) {
            K.dots(rbuf.as<double>(), 1, rbuf.as<double>());
            K.fetch(1);
            std::vector<double> rn(nrhs);
            for (int c = 0; c < nrhs; ++c) {
                rn[c] = std::sqrt(std::max(0.0, K.h_host[c]));
                if (rn[c] == 0.0) rn[c] = 1.0;
            }
            // solve A d = r; its right-hand side is copied into the Krylov b slot
            HM_CHECK_HIP(hipMemcpyAsync(K.D, rbuf.get(), sizeof(double) * nrhs * n, hipMemcpyDeviceToDevice, s));
            GmresResult g = gmres(K, op.main, K.D, dbuf.as<double>(), rn, inner, o.max_iter - iters, hist, r);
            iters += g.iterations;
            if (g.nonfinite) {
                nonfinite = true;
                break;
            }
            hipLaunchKernelGGL(k_axpby, dim3(K.g1(n * nrhs)), dim3(256), 0, s, nrhs, n, X, n, 1.0, dbuf.as<double>(),
                               n, 1.0, X, n);
            ++sweeps;
            // restore b and form the FP64 residual with the reference operator
            HM_CHECK_HIP(hipMemcpy2DAsync(B, n * sizeof(double), d_B, ldb * sizeof(double), n * sizeof(double), nrhs,
                                          hipMemcpyDeviceToDevice, s));
            r = true_residual(X, rbuf.as<double>());
            if (!std::isfinite(r)) {
                nonfinite = true;
                break;
            }
            if (r <= o.rtol) {
                ok = true;
                break;
            }
        }
        // the Krylov b slot held correction right-hand sides: restore b
        HM_CHECK_HIP(hipMemcpy2DAsync(B, n * sizeof(double), d_B, ldb * sizeof(double), n * sizeof(double), nrhs,
                                      hipMemcpyDeviceToDevice, s));
    };
    // The plain preconditioner under the learned correction (3x3 or leaf
    // block-Jacobi) is its fallback: 3x3 block-Jacobi when no correction is
    // attached for the current tangent, and the attached correction's base
    // run again from x = 0 when the learned solve produced a non-finite
    // value or did not meet the FP64 residual test.
    int pc = o.precond, fallback = HM_FALLBACK_NONE, discarded = 0;
    const double t_pc = now_ms();
    if (pc == HM_PC_LEAF) leaf_pc_prepare(op, s);
    if (pc == HM_PC_ILU) ilu_pc_prepare(op, o.ilu_fraction == 0.0 ? 0.01 : o.ilu_fraction, s);
    const double pc_ms = now_ms() - t_pc;
    if (pc == HM_PC_LEARNED && !op.lp.attached) {
        pc = HM_PC_BLOCK3;
        fallback = HM_FALLBACK_NOT_ATTACHED;
    }
    attempt(pc);
    if (!ok && pc == HM_PC_LEARNED) {
        fallback = nonfinite ? HM_FALLBACK_NONFINITE : HM_FALLBACK_NOT_CONVERGED;
        discarded = iters;
        pc = op.lp.base;
        if (pc == HM_PC_LEAF) leaf_pc_prepare(op, s);
        attempt(pc);
    }
    HM_CHECK_HIP(hipMemcpy2DAsync(d_X, ldx * sizeof(double), X, n * sizeof(double), n * sizeof(double), nrhs,
                                  hipMemcpyDeviceToDevice, s));
    HM_CHECK_HIP(hipStreamSynchronize(s));
    if (rep) {
        std::memset(rep, 0, sizeof(*rep));
        rep->iterations = iters;
        rep->refinements = sweeps;
        rep->converged = ok ? 1 : 0;
        double worst = 0.0;
        for (double r : relres) worst = std::max(worst, r);
        rep->rel_residual = worst;
        rep->solve_ms = now_ms() - t0;
        rep->n_history = (int)std::min<size_t>(hist.size(), 1024);
        rep->precond_used = pc;
        rep->fallback = fallback;
        rep->discarded_iterations = discarded;
        rep->precond_setup_ms = pc_ms;
        if (pc == HM_PC_ILU) {
            rep->precond_nnz = op.ilu.nnz;
            rep->precond_colors = op.ilu.n_colors;
        }
        for (int i = 0; i < rep->n_history; ++i) rep->history[i] = hist[i];
    }
    return ok ? HM_OK : HM_ENOTCONV;
}

}  // namespace hm
