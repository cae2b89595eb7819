// Interface elasto-plastic law of the fault and fracture elements (paper
// Sec. 2.2.2-2.2.3), integrated over one step by an elastic predictor and a
// backward-Euler plastic corrector, with the consistent tangent
// C^ep = dT'/d(delta increment) that enters the mechanical Jacobian
// J = E - eta/dt - C^ep (Sec. 3.1.1).
//
// One thread per element, FP64.  Every function of the return map is written
// once, generic in its scalar type: plain doubles for the scalar consistency
// solves (safeguarded Newton inside a bracket), forward-mode dual numbers for
// derivatives.  The tangent follows from one dual evaluation at the converged
// multipliers (lanes: the three DD increments and the active multipliers)
// and the implicit function theorem on the active consistency equations.
#include "hm_internal.hpp"

#include <cmath>

namespace hm {
namespace {

constexpr int kIfMaxMat = 16;

struct IfMats {
    hm_interface_material m[kIfMaxMat];
};

enum : int32_t { kElastic = 0, kShear = 1, kTensile = 2, kCorner = 3, kOpen = 4, kBadMaterial = -1 };

// ------------------------------------------------------------------ dual numbers

template <int K>
struct Dual {
    double v;
    double d[K];
    __device__ Dual(double x = 0.0) : v(x)
    {
#pragma unroll
        for (int i = 0; i < K; ++i) d[i] = 0.0;
    }
};

template <int K>
__device__ __forceinline__ Dual<K> seeded(double x, int lane)
{
    Dual<K> r(x);
    r.d[lane] = 1.0;
    return r;
}

__device__ __forceinline__ double val(double x) { return x; }
template <int K>
__device__ __forceinline__ double val(const Dual<K>& x) { return x.v; }

template <int K>
__device__ __forceinline__ Dual<K> operator+(const Dual<K>& a, const Dual<K>& b)
{
    Dual<K> r(a.v + b.v);
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator-(const Dual<K>& a, const Dual<K>& b)
{
    Dual<K> r(a.v - b.v);
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator*(const Dual<K>& a, const Dual<K>& b)
{
    Dual<K> r(a.v * b.v);
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator/(const Dual<K>& a, const Dual<K>& b)
{
    Dual<K> r(a.v / b.v);
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator+(const Dual<K>& a, double b) { return a + Dual<K>(b); }
template <int K>
__device__ __forceinline__ Dual<K> operator+(double a, const Dual<K>& b) { return Dual<K>(a) + b; }
template <int K>
__device__ __forceinline__ Dual<K> operator-(const Dual<K>& a, double b) { return a - Dual<K>(b); }
template <int K>
__device__ __forceinline__ Dual<K> operator-(double a, const Dual<K>& b) { return Dual<K>(a) - b; }
template <int K>
__device__ __forceinline__ Dual<K> operator*(const Dual<K>& a, double b)
{
    Dual<K> r(a.v * b);
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = a.d[i] * b;
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator*(double a, const Dual<K>& b) { return b * a; }
template <int K>
__device__ __forceinline__ Dual<K> operator/(const Dual<K>& a, double b) { return a / Dual<K>(b); }

__device__ __forceinline__ double sq(double x) { return sqrt(x); }
template <int K>
__device__ __forceinline__ Dual<K> sq(const Dual<K>& a)
{
    Dual<K> r(sqrt(a.v));
    const double s = r.v > 0.0 ? 0.5 / r.v : 0.0;
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = a.d[i] * s;
    return r;
}

// ------------------------------------------------------------------ the law

// linear weakening W(x / L) = max(0, 1 - x / L); L = 0: fully weakened; L = inf: none
template <class S>
__device__ __forceinline__ S weaken(const S& x, double L)
{
    if (!(L > 0.0)) return S(0.0);
    S r = 1.0 - x / L;
    return val(r) > 0.0 ? r : S(0.0);
}

// running maximum of a magnitude: the new value wins only when strictly larger
template <class S>
__device__ __forceinline__ S grow(double old, const S& nw)
{
    return val(nw) > old ? nw : S(old);
}

template <class S>
__device__ __forceinline__ S friction(const hm_interface_material& m, const S& chi_s)
{
    return m.f_res + (m.f_peak - m.f_res) * weaken(chi_s, m.d_c);
}

template <class S>
__device__ __forceinline__ S coulomb(const hm_interface_material& m, const S& tau, const S& tn, const S* chi)
{
    return tau + friction(m, chi[0]) * tn - m.c_peak * weaken(chi[1], m.w_c);
}

template <class S>
__device__ __forceinline__ S cutoff(const hm_interface_material& m, const S& tn, const S* chi)
{
    return tn - m.sigma_peak * weaken(chi[1], m.w_c);
}

template <class S>
struct EndState {
    S T[3];
    S dp[3];
    S chi[3];
    S tau;
};

// End-of-step traction, inelastic DD and internal variables for given
// multipliers: shear slip lam along tau_tr / |tau_tr|; normal inelastic DD
// lam * psi (Coulomb flow alone, `dilatant`) or nu.
template <class S>
__device__ __forceinline__ EndState<S> end_state(const hm_interface_material& m, const S* Ttr, const double* dps,
                                        const double* chi0, const S& lam, const S& nu, bool dilatant)
{
    EndState<S> e;
    const S q = sq(Ttr[0] * Ttr[0] + Ttr[1] * Ttr[1]);
    S ps1, ps2;
    if (val(lam) == 0.0) {
        ps1 = S(dps[0]);
        ps2 = S(dps[1]);
        e.T[0] = Ttr[0];
        e.T[1] = Ttr[1];
        e.tau = q;
    } else {
        const S s1 = Ttr[0] / q, s2 = Ttr[1] / q;
        ps1 = dps[0] + lam * s1;
        ps2 = dps[1] + lam * s2;
        e.tau = q - m.k_s * lam;
        e.T[0] = e.tau * s1;
        e.T[1] = e.tau * s2;
    }
    const S chi_s = grow(chi0[0], sq(ps1 * ps1 + ps2 * ps2));
    const S psi = m.psi_peak * weaken(chi_s, m.d_c);
    const S dn = dilatant ? lam * psi : nu;
    const S pn = dps[2] + dn;
    e.chi[0] = chi_s;
    e.chi[1] = grow(chi0[1], sq(ps1 * ps1 + ps2 * ps2 + pn * pn));
    e.chi[2] = chi0[2] + lam * psi;
    e.T[2] = Ttr[2] - m.k_n * dn;
    e.dp[0] = ps1;
    e.dp[1] = ps2;
    e.dp[2] = pn;
    return e;
}

// Root of a function decreasing on [0, hi]: 0 if f(0) <= tol, hi if f(hi) >= -tol,
// else safeguarded Newton from the secant point: it stops once a Newton
// correction falls below 1e-12 of the iterate (the next error is below
// rounding), and a bisection step replaces any Newton step that leaves the
// bracket or does not halve the previous step.  fn(x, fx) stores f(x) in fx
// and returns f'(x).
template <class F>
__device__ __forceinline__ double root_dec(F fn, double hi, double tol)
{
    if (!(hi > 0.0)) return 0.0;
    double f0, fh;
    fn(0.0, f0);
    if (f0 <= tol) return 0.0;
    fn(hi, fh);
    if (fh >= -tol) return hi;
    double a = 0.0, b = hi;
    double x = hi * (f0 / (f0 - fh));
    double step_old = hi;
    for (int it = 0; it < 100; ++it) {
        double fx;
        const double dfx = fn(x, fx);
        if (fx == 0.0) return x;
        if (fx > 0.0)
            a = x;
        else
            b = x;
        double xn = dfx < 0.0 ? x - fx / dfx : a;
        double step = fabs(xn - x);
        // a negligible Newton correction: converged (quadratically) to rounding
        if (dfx < 0.0 && step <= 1e-12 * x) return xn;
        if (!(xn > a && xn < b) || 2.0 * step > step_old) {
            xn = 0.5 * (a + b);
            step = 0.5 * (b - a);
        }
        if (step <= 4e-16 * xn || (b - a) <= 8e-16 * b) return xn;
        step_old = step;
        x = xn;
    }
    return x;
}

template <int K>
__device__ __forceinline__ void lift(const double* T, Dual<K>* out)
{
#pragma unroll
    for (int i = 0; i < 3; ++i) out[i] = Dual<K>(T[i]);
}

struct Element {
    double T[3], dp[3], chi[3], cep[9];
    int32_t mode;
};

__device__ __forceinline__ Element update_one(const hm_interface_material& m, const double* dd, const double* T0, const double* dp0,
                              const double* chi0)
{
    Element out;
    double Ttr[3] = {T0[0] + m.k_s * dd[0], T0[1] + m.k_s * dd[1], T0[2] + m.k_n * dd[2]};
    double dps[3] = {dp0[0], dp0[1], dp0[2]};
    // fully damaged (min(chi_t / w_c, 1) = 1): traction-free while the gap is open
    if (weaken(chi0[1], m.w_c) == 0.0) {
        const double g = fmax(0.0, dp0[2] - chi0[2]);
        if (Ttr[2] + m.k_n * g >= 0.0) {
            out.mode = kOpen;
            out.dp[0] = dp0[0] + Ttr[0] / m.k_s;
            out.dp[1] = dp0[1] + Ttr[1] / m.k_s;
            out.dp[2] = dp0[2] + Ttr[2] / m.k_n;
            out.chi[0] = fmax(chi0[0], sqrt(out.dp[0] * out.dp[0] + out.dp[1] * out.dp[1]));
            out.chi[1] = fmax(chi0[1], sqrt(out.dp[0] * out.dp[0] + out.dp[1] * out.dp[1] + out.dp[2] * out.dp[2]));
            out.chi[2] = chi0[2];
#pragma unroll
            for (int i = 0; i < 3; ++i) out.T[i] = 0.0;
#pragma unroll
            for (int i = 0; i < 9; ++i) out.cep[i] = 0.0;
            return out;
        }
        Ttr[2] += m.k_n * g;
        dps[2] = dp0[2] - g;
    }
    const double q = sqrt(Ttr[0] * Ttr[0] + Ttr[1] * Ttr[1]);
    int32_t mode;
    double lam = 0.0, nu = 0.0;
    // tolerance of every surface test: 1e-12 of the trial traction scale, so
    // that states the algorithm puts exactly on a surface (a return ending at
    // zero strength, an element left on its surface without increment) are
    // not decided by the sign of a rounding error
    const double ytol = 1e-12 * (fabs(Ttr[0]) + fabs(Ttr[1]) + fabs(Ttr[2]) + m.c_peak + m.sigma_peak);

    // scalar consistency functions of the single-surface returns and the corner
    auto f_shear = [&](double x, double& fx) -> double {
        Dual<1> T1[3];
        lift(Ttr, T1);
        const EndState<Dual<1>> e = end_state(m, T1, dps, chi0, seeded<1>(x, 0), Dual<1>(0.0), true);
        const Dual<1> r = coulomb(m, e.tau, e.T[2], e.chi);
        fx = r.v;
        return r.d[0];
    };
    auto f_tens = [&](double x, double& fx) -> double {
        Dual<1> T1[3];
        lift(Ttr, T1);
        const EndState<Dual<1>> e = end_state(m, T1, dps, chi0, Dual<1>(0.0), seeded<1>(x, 0), false);
        const Dual<1> r = cutoff(m, e.T[2], e.chi);
        fx = r.v;
        return r.d[0];
    };
    const double nu_hi = fmax(Ttr[2], 0.0) / m.k_n;
    auto nu_of = [&](double l) -> double {
        return root_dec(
            [&](double x, double& fx) -> double {
                Dual<1> T1[3];
                lift(Ttr, T1);
                const EndState<Dual<1>> e = end_state(m, T1, dps, chi0, Dual<1>(l), seeded<1>(x, 0), false);
                const Dual<1> r = cutoff(m, e.T[2], e.chi);
                fx = r.v;
                return r.d[0];
            },
            nu_hi, ytol);
    };
    auto f_corner = [&](double x, double& fx) -> double {
        const double n = nu_of(x);
        Dual<2> T2[3];
        lift(Ttr, T2);
        const EndState<Dual<2>> e = end_state(m, T2, dps, chi0, seeded<2>(x, 0), seeded<2>(n, 1), false);
        const Dual<2> rc = coulomb(m, e.tau, e.T[2], e.chi);
        const Dual<2> rt = cutoff(m, e.T[2], e.chi);
        fx = rc.v;
        const double dn = (n > 0.0 && rt.d[1] != 0.0) ? -rt.d[0] / rt.d[1] : 0.0;
        return rc.d[0] + rc.d[1] * dn;
    };

    const double* c0 = chi0;
    const double fc_tr = coulomb(m, q, Ttr[2], c0), ft_tr = cutoff(m, Ttr[2], c0);
    if (fc_tr <= ytol && ft_tr <= ytol) {
        mode = kElastic;
    } else {
        const double f0 = friction(m, chi0[0]);
        const double w0 = weaken(chi0[1], m.w_c);
        const double cc = m.c_peak * w0, st = m.sigma_peak * w0;
        const double alpha = sqrt(1.0 + f0 * f0) - f0;
        const double h = q - (cc - f0 * st) - alpha * (Ttr[2] - st);
        mode = h > 0.0 ? kShear : kTensile;
        if (mode == kShear) {
            const double lam_hi = q / m.k_s;
            double fh;
            f_shear(lam_hi, fh);
            if (fh > ytol) {
                mode = kCorner;
            } else {
                lam = root_dec(f_shear, lam_hi, ytol);
                const EndState<double> e = end_state(m, Ttr, dps, chi0, lam, 0.0, true);
                if (cutoff(m, e.T[2], e.chi) > ytol) {
                    mode = kCorner;
                    lam = 0.0;
                }
            }
        }
        if (mode == kTensile) {
            nu = root_dec(f_tens, Ttr[2] / m.k_n, ytol);
            const EndState<double> e = end_state(m, Ttr, dps, chi0, 0.0, nu, false);
            if (coulomb(m, e.tau, e.T[2], e.chi) > ytol) {
                mode = kCorner;
                nu = 0.0;
            }
        }
        if (mode == kCorner) {
            lam = root_dec(f_corner, q / m.k_s, ytol);
            nu = nu_of(lam);
        }
    }
    out.mode = mode;

    // active multipliers: those solving a consistency equation
    const bool lam_on = (mode == kShear || mode == kCorner) && lam > 0.0;
    const bool nu_on = (mode == kTensile || mode == kCorner) && nu > 0.0;

    // one dual evaluation: lanes 0-2 the DD increment, 3 lam, 4 nu
    constexpr int L = 5;
    Dual<L> T5[3];
    lift(Ttr, T5);
    T5[0].d[0] = m.k_s;
    T5[1].d[1] = m.k_s;
    T5[2].d[2] = m.k_n;
    Dual<L> lam5(lam), nu5(nu);
    if (lam_on) lam5.d[3] = 1.0;
    if (nu_on) nu5.d[4] = 1.0;
    const EndState<Dual<L>> e = end_state(m, T5, dps, chi0, lam5, nu5, mode == kShear);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        out.T[i] = e.T[i].v;
        out.dp[i] = e.dp[i].v;
        out.chi[i] = e.chi[i].v;
    }
    double cep[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) cep[i][j] = e.T[i].d[j];
    // implicit function theorem on the active consistency equations (Fc for
    // lam, Ft for nu); an inactive multiplier is pinned by an identity row
    const Dual<L> rc = coulomb(m, e.tau, e.T[2], e.chi);
    const Dual<L> rt = cutoff(m, e.T[2], e.chi);
    double a = 1.0, b = 0.0, c = 0.0, d = 1.0;
    if (lam_on) {
        a = rc.d[3];
        b = rc.d[4];
    }
    if (nu_on) {
        c = rt.d[3];
        d = rt.d[4];
    }
    const double det = a * d - b * c;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double r1 = lam_on ? rc.d[j] : 0.0;
        const double r2 = nu_on ? rt.d[j] : 0.0;
        const double yl = -(d * r1 - b * r2) / det;
        const double yn = -(a * r2 - c * r1) / det;
#pragma unroll
        for (int i = 0; i < 3; ++i) cep[i][j] += e.T[i].d[3] * yl + e.T[i].d[4] * yn;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) out.cep[3 * i + j] = cep[i][j];
    return out;
}

__global__ __launch_bounds__(256) void k_interface_update(IfMats mats, int n_mat, int64_t n, const int32_t* mat_id,
                                                          const double* dd, const double* t0, const double* dp0,
                                                          const double* chi0, double* t1, double* dp1, double* chi1,
                                                          double* cep, int32_t* mode, const double* eta_dt,
                                                          double* D)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int id = mat_id ? mat_id[e] : 0;
    double in_dd[3], in_t[3], in_dp[3], in_chi[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        in_dd[i] = dd[3 * e + i];
        in_t[i] = t0[3 * e + i];
        in_dp[i] = dp0[3 * e + i];
        in_chi[i] = chi0[3 * e + i];
    }
    Element r;
    if (id < 0 || id >= n_mat) {
        const double nan = __builtin_nan("");
#pragma unroll
        for (int i = 0; i < 3; ++i) r.T[i] = r.dp[i] = r.chi[i] = nan;
#pragma unroll
        for (int i = 0; i < 9; ++i) r.cep[i] = nan;
        r.mode = kBadMaterial;
    } else {
        r = update_one(mats.m[id], in_dd, in_t, in_dp, in_chi);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        t1[3 * e + i] = r.T[i];
        dp1[3 * e + i] = r.dp[i];
        chi1[3 * e + i] = r.chi[i];
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) cep[9 * e + i] = r.cep[i];
    if (mode) mode[e] = r.mode;
    if (D) {
#pragma unroll
        for (int i = 0; i < 9; ++i) D[9 * e + i] = r.cep[i];
        if (eta_dt)
#pragma unroll
            for (int i = 0; i < 3; ++i) D[9 * e + 4 * i] += eta_dt[3 * e + i];
    }
}

}  // namespace

void interface_update(int n_mat, const hm_interface_material* mats, int64_t n, const int32_t* d_mat_id,
                      const double* d_dd, const double* d_t, const double* d_dp, const double* d_chi, double* d_t_new,
                      double* d_dp_new, double* d_chi_new, double* d_cep, int32_t* d_mode, const double* d_eta_dt,
                      double* d_D, hipStream_t s)
{
    HM_REQUIRE(n_mat >= 1 && n_mat <= kIfMaxMat, HM_EINVAL, "n_mat must be in [1, 16]");
    HM_REQUIRE(mats, HM_EINVAL, "materials are null");
    HM_REQUIRE(n >= 0, HM_EINVAL, "negative element count");
    IfMats pm{};
    for (int i = 0; i < n_mat; ++i) {
        const hm_interface_material& m = mats[i];
        const std::string at = "material " + std::to_string(i) + ": ";
        HM_REQUIRE(std::isfinite(m.k_s) && m.k_s > 0.0 && std::isfinite(m.k_n) && m.k_n > 0.0, HM_EINVAL,
                   at + "stiffnesses must be finite and positive");
        HM_REQUIRE(m.f_res >= 0.0 && m.f_peak >= m.f_res && std::isfinite(m.f_peak), HM_EINVAL,
                   at + "need 0 <= f_res <= f_peak < inf");
        HM_REQUIRE(m.psi_peak >= 0.0 && std::isfinite(m.psi_peak), HM_EINVAL, at + "psi_peak must be >= 0");
        HM_REQUIRE(m.d_c >= 0.0 && m.w_c >= 0.0, HM_EINVAL, at + "critical distances must be >= 0 (inf allowed)");
        HM_REQUIRE(m.c_peak >= 0.0 && m.sigma_peak >= 0.0 && std::isfinite(m.c_peak) && std::isfinite(m.sigma_peak),
                   HM_EINVAL, at + "strengths must be finite and >= 0");
        HM_REQUIRE(m.c_peak >= m.f_peak * m.sigma_peak, HM_EINVAL,
                   at + "the tension cut-off must lie below the Coulomb apex (c_peak >= f_peak sigma_peak)");
        pm.m[i] = m;
    }
    if (n == 0) return;
    HM_REQUIRE(d_dd && d_t && d_dp && d_chi && d_t_new && d_dp_new && d_chi_new && d_cep, HM_EINVAL,
               "state, increment and tangent arrays must not be null");
    const int64_t blocks = (n + 255) / 256;
    HM_REQUIRE(blocks <= 0x7fffffff, HM_EINVAL, "too many elements");
    hipLaunchKernelGGL(k_interface_update, dim3((unsigned)blocks), dim3(256), 0, s, pm, n_mat, n, d_mat_id, d_dd, d_t,
                       d_dp, d_chi, d_t_new, d_dp_new, d_chi_new, d_cep, d_mode, d_eta_dt, d_D);
    HM_CHECK_HIP(hipGetLastError());
}

}  // namespace hm
