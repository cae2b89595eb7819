// One implicit step of the mechanical problem (paper Sec. 3.1.1,
// "Elasto-plastic solver"): Newton's method on the residual
//   r(dd) = dT'o - dT'(dd) + E dd + I_n dp - eta (dd - dd_prev) / dt
// with the mechanical Jacobian J = E - eta/dt - C^ep.  Each iteration runs
// the interface law from the start-of-step state (end-of-step tractions,
// C^ep and D = C^ep + eta/dt), the FP64 H-matrix product E dd, the residual
// kernel, and a GMRES solve of J y = r on the operator's tangent system;
// then dd -= y.  The residual norm is a two-stage reduction in a fixed
// order, so the iteration is deterministic.
#include "hm_op.hpp"

#include <chrono>
#include <cmath>

namespace hm {
namespace {

constexpr int kNormBlock = 256;
constexpr int kNormPerThread = 8;

__global__ __launch_bounds__(256) void k_mech_residual(int64_t ne, const double* dT0, const double* t_new,
                                                       const double* t_n, const double* Ex, const double* dpress,
                                                       const double* eta_dt, const double* dd, const double* dd_prev,
                                                       double* r)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int64_t k = 3 * e + i;
        double v = (dT0 ? dT0[k] : 0.0) - (t_new[k] - t_n[k]) + Ex[k];
        if (i == 2 && dpress) v += dpress[e];
        if (eta_dt) v -= eta_dt[k] * (dd[k] - (dd_prev ? dd_prev[k] : 0.0));
        r[k] = v;
    }
}

// partial sums of squares: block b covers [b * 2048, (b + 1) * 2048)
__global__ __launch_bounds__(kNormBlock) void k_sumsq_partial(int64_t n, const double* x, double* partial)
{
    __shared__ double red[kNormBlock];
    const int64_t base = (int64_t)blockIdx.x * kNormBlock * kNormPerThread + threadIdx.x;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kNormPerThread; ++j) {
        const int64_t i = base + (int64_t)j * kNormBlock;
        if (i < n) s += x[i] * x[i];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kNormBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sub(int64_t n, const double* y, double* x)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] -= y[i];
}

// partial sums of (dd/dt - dd_prev/dt_prev)^2 and total^2 per block, same layout as k_sumsq_partial
__global__ __launch_bounds__(kNormBlock) void k_lte_partial(int64_t n, const double* dd, double inv_dt,
                                                            const double* dd_prev, double inv_dt_prev,
                                                            const double* total, double* partial)
{
    __shared__ double ra[kNormBlock], rb[kNormBlock];
    const int64_t base = (int64_t)blockIdx.x * kNormBlock * kNormPerThread + threadIdx.x;
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int j = 0; j < kNormPerThread; ++j) {
        const int64_t i = base + (int64_t)j * kNormBlock;
        if (i < n) {
            const double r = dd[i] * inv_dt - (dd_prev ? dd_prev[i] * inv_dt_prev : 0.0);
            sa += r * r;
            sb += total[i] * total[i];
        }
    }
    ra[threadIdx.x] = sa;
    rb[threadIdx.x] = sb;
    __syncthreads();
    for (int w = kNormBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            ra[threadIdx.x] += ra[threadIdx.x + w];
            rb[threadIdx.x] += rb[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = ra[0];
        partial[2 * blockIdx.x + 1] = rb[0];
    }
}

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

hm_status newton_step(Op& op, int n_mat, const hm_interface_material* mats, const int32_t* d_mat_id,
                      const double* d_t, const double* d_dp, const double* d_chi, const double* d_dT0,
                      const double* d_dpress, const double* d_eta_dt, const double* d_dd_prev, double* d_dd,
                      double* d_t_new, double* d_dp_new, double* d_chi_new, const hm_newton_opts& o,
                      hm_newton_report* rep, hipStream_t s)
{
    HM_REQUIRE(o.max_newton >= 0 && o.max_newton <= 63, HM_EINVAL, "max_newton must be in [0, 63]");
    HM_REQUIRE(o.rtol >= 0.0 && o.atol >= 0.0, HM_EINVAL, "tolerances must be >= 0");
    HM_REQUIRE(o.forcing == 0 || o.forcing == 1, HM_EINVAL, "forcing must be 0 or 1");
    HM_REQUIRE(d_t && d_dp && d_chi && d_dd && d_t_new && d_dp_new && d_chi_new, HM_EINVAL,
               "state and increment arrays must not be null");
    HM_REQUIRE(d_t_new != d_t && d_dp_new != d_dp && d_chi_new != d_chi, HM_EINVAL,
               "the start-of-step state is read at every iteration: outputs must be other arrays");
    HM_REQUIRE(op.ref || op.main.near_prec == HM_F64, HM_EINVAL,
               "the residual needs the FP64 operator (build FP64 or with keep_f64_reference)");
    const double t0 = now_ms();
    const int64_t ne = op.ne, n3 = 3 * ne;
    const int64_t nblk = (n3 + kNormBlock * kNormPerThread - 1) / (kNormBlock * kNormPerThread);
    DevBuf ws(sizeof(double) * (3 * n3 + 18 * ne + nblk) + sizeof(int32_t) * ne);
    double* Ex = ws.as<double>();
    double* r = Ex + n3;
    double* y = r + n3;
    double* cep = y + n3;
    double* D = cep + 9 * ne;
    double* partial = D + 9 * ne;
    int32_t* mode = reinterpret_cast<int32_t*>(partial + nblk);
    std::vector<double> hpart(nblk);
    const Variant& v = op.ref_variant();
    const unsigned eblocks = (unsigned)((ne + 255) / 256), vblocks = (unsigned)((n3 + 255) / 256);

    std::vector<double> hist;
    std::vector<int> its;
    double eta_prev = 0.1;
    for (int k = 0;; ++k) {
        interface_update(n_mat, mats, ne, d_mat_id, d_dd, d_t, d_dp, d_chi, d_t_new, d_dp_new, d_chi_new, cep, mode,
                         d_eta_dt, D, s);
        apply(op, v, 1, d_dd, n3, Ex, n3, false, s);
        hipLaunchKernelGGL(k_mech_residual, dim3(eblocks), dim3(256), 0, s, ne, d_dT0, d_t_new, d_t, Ex, d_dpress,
                           d_eta_dt, d_dd, d_dd_prev, r);
        hipLaunchKernelGGL(k_sumsq_partial, dim3((unsigned)nblk), dim3(kNormBlock), 0, s, n3, r, partial);
        HM_CHECK_HIP(hipGetLastError());
        HM_CHECK_HIP(hipMemcpyAsync(hpart.data(), partial, sizeof(double) * nblk, hipMemcpyDeviceToHost, s));
        HM_CHECK_HIP(hipStreamSynchronize(s));
        double ss = 0.0;
        for (double p : hpart) ss += p;
        hist.push_back(std::sqrt(ss));
        const bool done = hist.back() <= std::max(o.rtol * hist.front(), o.atol);
        if (done || k == o.max_newton || !std::isfinite(hist.back())) break;
        tangent_set(op, D, nullptr, s);
        hm_solve_opts lin = o.lin;
        if (o.forcing == 1) {
            // Eisenstat-Walker choice 2 (gamma 0.9, alpha 2) with the usual
            // safeguards: no sudden tightening, no oversolving of the last step
            double eta = 0.1;
            if (k > 0) {
                const double ratio = hist[k] / hist[k - 1];
                eta = 0.9 * ratio * ratio;
                const double keep = 0.9 * eta_prev * eta_prev;
                if (keep > 0.1) eta = std::max(eta, keep);
            }
            eta = std::max(eta, 0.5 * std::max(o.rtol * hist.front(), o.atol) / hist[k]);
            eta = std::max(std::min(eta, 0.1), o.lin.rtol);
            lin.rtol = eta;
            eta_prev = eta;
        }
        hm_solve_report sr{};
        const hm_status st = solve(op, lin, 1, r, n3, y, n3, &sr, s);
        HM_REQUIRE(st == HM_OK || st == HM_ENOTCONV, st, "linear solve failed");
        its.push_back(sr.iterations);
        hipLaunchKernelGGL(k_sub, dim3(vblocks), dim3(256), 0, s, n3, y, d_dd);
        HM_CHECK_HIP(hipGetLastError());
    }
    // leave the operator's tangent at the Jacobian of the returned state
    tangent_set(op, D, nullptr, s);
    const bool converged = hist.back() <= std::max(o.rtol * hist.front(), o.atol);
    if (rep) {
        *rep = hm_newton_report{};
        rep->iterations = (int)its.size();
        rep->converged = converged ? 1 : 0;
        rep->n_history = (int)hist.size();
        for (size_t i = 0; i < hist.size() && i < 64; ++i) rep->residual[i] = hist[i];
        for (size_t i = 0; i < its.size() && i < 64; ++i) rep->gmres_iterations[i] = its[i];
        std::vector<int32_t> hmode(ne);
        HM_CHECK_HIP(hipMemcpyAsync(hmode.data(), mode, sizeof(int32_t) * ne, hipMemcpyDeviceToHost, s));
        HM_CHECK_HIP(hipStreamSynchronize(s));
        for (int32_t m : hmode)
            if (m >= 0 && m < 5) rep->modes[m]++;
        rep->ms = now_ms() - t0;
    }
    return converged ? HM_OK : HM_ENOTCONV;
}

double lte_estimate(int64_t n, const double* d_dd, double dt, const double* d_dd_prev, double dt_prev,
                    const double* d_total, hipStream_t s)
{
    HM_REQUIRE(n >= 1 && d_dd && d_total, HM_EINVAL, "vectors must be non-null and non-empty");
    HM_REQUIRE(dt > 0.0 && (!d_dd_prev || dt_prev > 0.0), HM_EINVAL, "time steps must be positive");
    const int64_t nblk = (n + kNormBlock * kNormPerThread - 1) / (kNormBlock * kNormPerThread);
    DevBuf part(sizeof(double) * 2 * nblk);
    hipLaunchKernelGGL(k_lte_partial, dim3((unsigned)nblk), dim3(kNormBlock), 0, s, n, d_dd, 1.0 / dt, d_dd_prev,
                       d_dd_prev ? 1.0 / dt_prev : 0.0, d_total, part.as<double>());
    HM_CHECK_HIP(hipGetLastError());
    std::vector<double> h(2 * nblk);
    HM_CHECK_HIP(hipMemcpyAsync(h.data(), part.get(), sizeof(double) * 2 * nblk, hipMemcpyDeviceToHost, s));
    HM_CHECK_HIP(hipStreamSynchronize(s));
    double a = 0.0, b = 0.0;
    for (int64_t i = 0; i < nblk; ++i) {
        a += h[2 * i];
        b += h[2 * i + 1];
    }
    HM_REQUIRE(b > 0.0, HM_EINVAL, "the total DD is zero");
    return 0.5 * dt * std::sqrt(a) / std::sqrt(b);
}

}  // namespace hm
