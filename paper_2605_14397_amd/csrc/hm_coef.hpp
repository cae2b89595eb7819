// Influence coefficients of the piecewise-constant DD collocation operator.
//
// Paper Sec. 3.1 ("Solid mechanics"): the traction at a collocation point
// (element centroid) due to a uniform DD over a flat element, integrated
// analytically before the limit so the result is regular.
//
// Route taken here: a uniform DD b over a flat polygon produces the same
// stress as the dislocation loop along the polygon boundary with Burgers
// vector b (Volterra).  The loop stress is the Peach-Koehler line integral
//   sig_ac =  (G/4pi) sum_edges [ (J1 x b)_a e_c + (J1 x b)_c e_a ]
//           -(G/(4pi(1-nu))) sum_edges [ -(c_a J1_c + c_c J1_a) + delta_ac (c.J1)
//                                        + 3 c_i J3_iac ]
// with c = b x e for an edge of unit tangent e, r = x - x'(s), R = |r|,
// J1 = int r/R^3 ds and J3 = int r r r / R^5 ds.  Along a straight edge both
// integrals have closed forms in t = s - (x - P0).e and the distance d of x
// to the edge line; they are evaluated below in forms that avoid
// cancellation when x lies near the edge's line outside the edge.  The loop
// runs v0 -> v1 -> ... counter-clockwise about the element normal, with
// b = u+ - u-.
#pragma once

#include <hip/hip_runtime.h>

namespace hm {

struct ElemGeo {
    double v[12];   // up to 4 vertices, xyz each
    double fr[9];   // rows s1, s2, n
    double c[3];    // collocation point (vertex mean)
    int nv;         // 3 or 4
    int pad;
};

__host__ __device__ inline double dot3(const double* a, const double* b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__host__ __device__ inline void cross3(const double* a, const double* b, double* o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// out[a*3 + b] = s_a(recv) . sig(b = e_b(src)) . n(recv), Pa/m.
// kG = G/(4 pi), kN = G/(4 pi (1 - nu)).
__host__ __device__ inline void dd_block(const double* x, const double* fr, const ElemGeo& S, double kG,
                                         double kN, double* out)
{
    const double* n = fr + 6;
    double tr[3][3];  // traction vector (global components) per source basis b
    for (int b = 0; b < 3; ++b)
        for (int k = 0; k < 3; ++k) tr[b][k] = 0.0;

    for (int q = 0; q < S.nv; ++q) {
        const double* P0 = S.v + 3 * q;
        const double* P1 = S.v + 3 * ((q + 1 == S.nv) ? 0 : q + 1);
        double dv[3] = {P1[0] - P0[0], P1[1] - P0[1], P1[2] - P0[2]};
        double L = sqrt(dot3(dv, dv));
        double e[3] = {dv[0] / L, dv[1] / L, dv[2] / L};
        double p[3] = {x[0] - P0[0], x[1] - P0[1], x[2] - P0[2]};
        double p1[3] = {x[0] - P1[0], x[1] - P1[1], x[2] - P1[2]};
        double a = dot3(p, e);
        double rho[3] = {p[0] - a * e[0], p[1] - a * e[1], p[2] - a * e[2]};
        double d2 = dot3(rho, rho);
        double t0 = -a, t1 = L - a;
        double R0 = sqrt(dot3(p, p)), R1 = sqrt(dot3(p1, p1));
        double S0 = t0 / R0, S1 = t1 / R1;
        double sumt = t0 + t1;  // t1 - t0 = L
        double DS, Q;
        if (t0 * t1 > 0.0) {
            // x projects outside the edge: difference forms without cancellation
            DS = L * sumt / (R0 * R1 * (t1 * R0 + t0 * R1));
            Q = (d2 + t1 * t1 + t0 * t0) / (R0 * R1 * (R0 * R1 + t0 * t1));
        } else {
            DS = (S1 - S0) / d2;
            Q = (1.0 - S1 * S0) / d2;
        }
        double dR = L * sumt / (R0 + R1);  // R1 - R0
        // int dt/R^3, int t dt/R^3, int dt/R^5, int t dt/R^5, int t^2 dt/R^5
        double dF0 = DS;
        double dF1 = dR / (R0 * R1);
        double dG0 = DS * (1.0 / (R1 * R1) + 1.0 / (R0 * R0) + Q) * (1.0 / 3.0);
        double dG1 = dR * (R1 * R1 + R1 * R0 + R0 * R0) / (3.0 * R0 * R0 * R0 * R1 * R1 * R1);
        double dG2 = DS * (S1 * S1 + S1 * S0 + S0 * S0) * (1.0 / 3.0);
        // J1 = int r/R^3 with r = rho - t e
        double J1[3] = {rho[0] * dF0 - e[0] * dF1, rho[1] * dF0 - e[1] * dF1, rho[2] * dF0 - e[2] * dF1};
        double en = dot3(e, n), rn = dot3(rho, n), J1n = dot3(J1, n);
        for (int b = 0; b < 3; ++b) {
            const double* bb = S.fr + 3 * b;
            double c[3], W[3];
            cross3(bb, e, c);
            cross3(J1, bb, W);
            double cr = dot3(c, rho), cn = dot3(c, n), Wn = dot3(W, n);
            double g0 = 3.0 * cr * rn * dG0, g1 = 3.0 * cr * dG1, g2 = 3.0 * cr * en * dG2;
            for (int k = 0; k < 3; ++k) {
                double t3 = -(c[k] * J1n + cn * J1[k]) + n[k] * cr * dF0 + rho[k] * g0
                            - (rho[k] * en + e[k] * rn) * g1 + e[k] * g2;
                tr[b][k] += kG * (en * W[k] + e[k] * Wn) - kN * t3;
            }
        }
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) out[3 * a + b] = dot3(fr + 3 * a, tr[b]);
}

}  // namespace hm
