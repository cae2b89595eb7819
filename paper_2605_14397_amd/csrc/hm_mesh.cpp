// Mesh validation and element frames (host).
//
// Paper Sec. 2.2: each discontinuity carries a local orthonormal frame
// (s1, s2, n) with n its normal; Sec. 3.1: the collocation point of a flat
// element is its centroid.  Frame convention: s1 = unit(v1 - v0),
// n = unit((v1 - v0) x (v2 - v0)), s2 = n x s1; collocation point = mean of
// the vertices (the centroid for triangles and rectangles).
#include <cmath>

#include "hm_internal.hpp"

namespace hm {

static double nrm(const double* a) { return std::sqrt(dot3(a, a)); }

void mesh_validate_and_frame(Mesh& m)
{
    HM_REQUIRE(m.nvpe == 3 || m.nvpe == 4, HM_EINVAL, "nv_per_elem must be 3 or 4");
    HM_REQUIRE(m.ne > 0 && m.nv > 0, HM_EINVAL, "empty mesh");
    for (int64_t k = 0; k < m.ne * m.nvpe; ++k)
        HM_REQUIRE(m.conn[k] >= 0 && m.conn[k] < m.nv, HM_EINVAL,
                   "connectivity id out of range at entry " + std::to_string(k));
    m.cent.assign(3 * m.ne, 0.0);
    m.frame.assign(9 * m.ne, 0.0);
    m.area.assign(m.ne, 0.0);
    m.geo.resize(m.ne);
    for (int64_t e = 0; e < m.ne; ++e) {
        ElemGeo g;
        std::memset(&g, 0, sizeof(g));
        g.nv = m.nvpe;
        for (int q = 0; q < m.nvpe; ++q)
            for (int k = 0; k < 3; ++k) g.v[3 * q + k] = m.xyz[3 * m.conn[e * m.nvpe + q] + k];
        double e1[3], e2[3], nn[3];
        for (int k = 0; k < 3; ++k) {
            e1[k] = g.v[3 + k] - g.v[k];
            e2[k] = g.v[6 + k] - g.v[k];
        }
        cross3(e1, e2, nn);
        double diam = 0.0;
        for (int a = 0; a < m.nvpe; ++a)
            for (int b = a + 1; b < m.nvpe; ++b) {
                double d[3] = {g.v[3 * b] - g.v[3 * a], g.v[3 * b + 1] - g.v[3 * a + 1], g.v[3 * b + 2] - g.v[3 * a + 2]};
                diam = std::fmax(diam, nrm(d));
            }
        double l1 = nrm(e1), ln = nrm(nn);
        HM_REQUIRE(diam > 0.0 && 0.5 * ln >= 1e-12 * diam * diam, HM_EBADMESH,
                   "degenerate element " + std::to_string(e));
        for (int k = 0; k < 3; ++k) {
            g.fr[k] = e1[k] / l1;
            g.fr[6 + k] = nn[k] / ln;
        }
        cross3(g.fr + 6, g.fr, g.fr + 3);
        double area = 0.5 * ln;
        if (m.nvpe == 4) {
            // planar rectangle: v2 = v1 + v3 - v0 and (v1 - v0) orthogonal to (v3 - v0)
            double e3[3], dev[3];
            for (int k = 0; k < 3; ++k) {
                e3[k] = g.v[9 + k] - g.v[k];
                dev[k] = g.v[6 + k] - (g.v[3 + k] + g.v[9 + k] - g.v[k]);
            }
            HM_REQUIRE(nrm(dev) <= 1e-10 * diam && std::fabs(dot3(e1, e3)) <= 1e-10 * diam * diam, HM_EBADMESH,
                       "element " + std::to_string(e) + " is not a planar rectangle");
            area = l1 * nrm(e3);
        }
        for (int k = 0; k < 3; ++k) {
            double s = 0.0;
            for (int q = 0; q < m.nvpe; ++q) s += g.v[3 * q + k];
            g.c[k] = s / m.nvpe;
        }
        m.geo[e] = g;
        for (int k = 0; k < 3; ++k) m.cent[3 * e + k] = g.c[k];
        for (int k = 0; k < 9; ++k) m.frame[9 * e + k] = g.fr[k];
        m.area[e] = area;
    }
}

}  // namespace hm
