// Cluster tree and block cluster tree (host).
//
// Paper Sec. 3.1 (hierarchical matrices): far-field interactions are kept
// as low-rank approximations and near-field ones in full.  The paper gives
// no tree details; the choices here are:
//   * cluster tree: recursive bisection of the element collocation points
//     at the median along the longest axis of their bounding box, down to
//     at most leaf_size elements (ties broken by element id);
//   * a pair of clusters (t, s) is admissible when
//       min(diam t, diam s) <= eta * dist(t, s),  dist > 0,
//     with axis-aligned bounding boxes of the elements' vertices, the box
//     diagonal as diameter and the box-to-box distance;
//   * admissible pairs become low-rank blocks, inadmissible pairs of leaves
//     dense blocks, other pairs are split (only the non-leaf side when one
//     side is a leaf).
#include <algorithm>
#include <cmath>
#include <numeric>

#include "hm_internal.hpp"

namespace hm {

namespace {

struct Builder {
    const Mesh& m;
    Plan& p;
    std::vector<double> ebmin, ebmax;  // per element vertex bbox

    Builder(const Mesh& mesh, Plan& plan) : m(mesh), p(plan)
    {
        ebmin.resize(3 * m.ne);
        ebmax.resize(3 * m.ne);
        for (int64_t e = 0; e < m.ne; ++e)
            for (int k = 0; k < 3; ++k) {
                double lo = 1e300, hi = -1e300;
                for (int q = 0; q < m.nvpe; ++q) {
                    double v = m.geo[e].v[3 * q + k];
                    lo = std::fmin(lo, v);
                    hi = std::fmax(hi, v);
                }
                ebmin[3 * e + k] = lo;
                ebmax[3 * e + k] = hi;
            }
    }

    int build(int64_t begin, int64_t end, int level)
    {
        int id = (int)p.nodes.size();
        p.nodes.emplace_back();
        Cluster c;
        c.begin = begin;
        c.end = end;
        c.level = level;
        double cmin[3] = {1e300, 1e300, 1e300}, cmax[3] = {-1e300, -1e300, -1e300};
        for (int k = 0; k < 3; ++k) {
            c.bmin[k] = 1e300;
            c.bmax[k] = -1e300;
        }
        for (int64_t q = begin; q < end; ++q) {
            int64_t e = p.perm[q];
            for (int k = 0; k < 3; ++k) {
                c.bmin[k] = std::fmin(c.bmin[k], ebmin[3 * e + k]);
                c.bmax[k] = std::fmax(c.bmax[k], ebmax[3 * e + k]);
                cmin[k] = std::fmin(cmin[k], m.cent[3 * e + k]);
                cmax[k] = std::fmax(cmax[k], m.cent[3 * e + k]);
            }
        }
        p.depth = std::max(p.depth, level);
        if (end - begin > p.leaf_size) {
            int axis = 0;
            for (int k = 1; k < 3; ++k)
                if (cmax[k] - cmin[k] > cmax[axis] - cmin[axis]) axis = k;
            auto first = p.perm.begin() + begin, last = p.perm.begin() + end;
            std::sort(first, last, [&](int64_t a, int64_t b) {
                double ka = m.cent[3 * a + axis], kb = m.cent[3 * b + axis];
                return ka < kb || (ka == kb && a < b);
            });
            int64_t mid = begin + (end - begin) / 2;
            p.nodes[id] = c;
            int l = build(begin, mid, level + 1);
            int r = build(mid, end, level + 1);
            p.nodes[id].child[0] = l;
            p.nodes[id].child[1] = r;
        } else {
            c.leaf_id = (int)p.leaves.size();
            p.leaves.push_back(id);
            p.nodes[id] = c;
        }
        return id;
    }

    static double diam(const Cluster& c)
    {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += (c.bmax[k] - c.bmin[k]) * (c.bmax[k] - c.bmin[k]);
        return std::sqrt(s);
    }

    static double dist(const Cluster& a, const Cluster& b)
    {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) {
            double g = std::fmax(0.0, std::fmax(a.bmin[k] - b.bmax[k], b.bmin[k] - a.bmax[k]));
            s += g * g;
        }
        return std::sqrt(s);
    }

    bool admissible(int t, int s) const
    {
        const Cluster& a = p.nodes[t];
        const Cluster& b = p.nodes[s];
        double d = dist(a, b);
        return d > 0.0 && std::fmin(diam(a), diam(b)) <= p.eta * d;
    }

    void blocks(int t, int s)
    {
        if (admissible(t, s)) {
            p.lowrank.emplace_back(t, s);
            return;
        }
        const Cluster& a = p.nodes[t];
        const Cluster& b = p.nodes[s];
        if (a.is_leaf() && b.is_leaf()) {
            p.dense.emplace_back(t, s);
        } else if (a.is_leaf()) {
            blocks(t, b.child[0]);
            blocks(t, b.child[1]);
        } else if (b.is_leaf()) {
            blocks(a.child[0], s);
            blocks(a.child[1], s);
        } else {
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) blocks(a.child[i], b.child[j]);
        }
    }

    // Planarity of every cluster: a leaf is planar when every element's
    // normal is parallel to the first one's and every vertex lies within
    // plane_tol of its plane; an inner node when both children lie in one
    // plane.
    void planes(int id)
    {
        Cluster& c = p.nodes[id];
        const double ptol = p.plane_tol;
        if (c.is_leaf()) {
            const int64_t e0 = p.perm[c.begin];
            const double* n0 = &m.frame[9 * e0 + 6];
            double d0 = 0.0;
            for (int k = 0; k < 3; ++k) d0 += n0[k] * m.cent[3 * e0 + k];
            bool ok = true;
            for (int64_t q = c.begin; q < c.end && ok; ++q) {
                const int64_t e = p.perm[q];
                const double* ne = &m.frame[9 * e + 6];
                if (std::fabs(ne[0] * n0[0] + ne[1] * n0[1] + ne[2] * n0[2]) < 1.0 - 1e-12) ok = false;
                for (int v = 0; v < m.nvpe && ok; ++v) {
                    const double* x = &m.geo[e].v[3 * v];
                    if (std::fabs(n0[0] * x[0] + n0[1] * x[1] + n0[2] * x[2] - d0) > ptol) ok = false;
                }
            }
            c.planar = ok;
            for (int k = 0; k < 3; ++k) c.pn[k] = n0[k];
            c.pd = d0;
            return;
        }
        planes(c.child[0]);
        planes(c.child[1]);
        const Cluster& a = p.nodes[c.child[0]];
        const Cluster& b = p.nodes[c.child[1]];
        c.planar = a.planar && b.planar && same_plane(a, b, ptol);
        for (int k = 0; k < 3; ++k) c.pn[k] = a.pn[k];
        c.pd = a.pd;
    }

    static bool same_plane(const Cluster& a, const Cluster& b, double ptol)
    {
        const double dot = a.pn[0] * b.pn[0] + a.pn[1] * b.pn[1] + a.pn[2] * b.pn[2];
        if (std::fabs(dot) < 1.0 - 1e-12) return false;
        return std::fabs(a.pd - (dot > 0 ? b.pd : -b.pd)) <= ptol;
    }

    void leaf_ranges(int id)
    {
        Cluster& c = p.nodes[id];
        if (c.is_leaf()) {
            c.first_leaf = c.leaf_id;
            c.n_leaves = 1;
            return;
        }
        leaf_ranges(c.child[0]);
        leaf_ranges(c.child[1]);
        c.first_leaf = p.nodes[c.child[0]].first_leaf;
        c.n_leaves = p.nodes[c.child[0]].n_leaves + p.nodes[c.child[1]].n_leaves;
    }
};

}  // namespace

// Replace the (admissible) pair (t, s) by the blocks of its children,
// chosen with the same rules as the initial block tree.
void split_block(Plan& p, int t, int s, std::vector<std::pair<int, int>>& lowrank,
                 std::vector<std::pair<int, int>>& dense)
{
    const Cluster& a = p.nodes[t];
    const Cluster& b = p.nodes[s];
    std::vector<std::pair<int, int>> kids;
    if (a.is_leaf() && b.is_leaf()) {
        dense.emplace_back(t, s);
        return;
    } else if (a.is_leaf()) {
        kids = {{t, b.child[0]}, {t, b.child[1]}};
    } else if (b.is_leaf()) {
        kids = {{a.child[0], s}, {a.child[1], s}};
    } else {
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) kids.emplace_back(a.child[i], b.child[j]);
    }
    for (auto& k : kids) {
        const Cluster& ka = p.nodes[k.first];
        const Cluster& kb = p.nodes[k.second];
        double d = Builder::dist(ka, kb);
        if (d > 0.0 && std::fmin(Builder::diam(ka), Builder::diam(kb)) <= p.eta * d)
            lowrank.push_back(k);
        else if (ka.is_leaf() && kb.is_leaf())
            dense.push_back(k);
        else
            split_block(p, k.first, k.second, lowrank, dense);
    }
}

bool coplanar_pair(const Plan& p, int t, int s)
{
    const Cluster& a = p.nodes[t];
    const Cluster& b = p.nodes[s];
    return a.planar && b.planar && Builder::same_plane(a, b, p.plane_tol);
}

void sort_blocks(Plan& p)
{
    auto by_target = [&](const std::pair<int, int>& x, const std::pair<int, int>& y) {
        const Cluster &a = p.nodes[x.first], &b = p.nodes[y.first];
        if (a.begin != b.begin) return a.begin < b.begin;
        if (a.end != b.end) return a.end > b.end;
        return p.nodes[x.second].begin < p.nodes[y.second].begin;
    };
    std::sort(p.dense.begin(), p.dense.end(), by_target);
    std::sort(p.lowrank.begin(), p.lowrank.end(), by_target);
}

Plan make_plan(const Mesh& m, int leaf_size, double eta)
{
    HM_REQUIRE(leaf_size >= 1 && leaf_size <= 64, HM_EINVAL, "leaf_size must be in [1, 64]");
    HM_REQUIRE(eta > 0.0 && std::isfinite(eta), HM_EINVAL, "eta must be positive");
    Plan p;
    p.leaf_size = leaf_size;
    p.eta = eta;
    p.perm.resize(m.ne);
    std::iota(p.perm.begin(), p.perm.end(), 0);
    Builder b(m, p);
    p.nodes.reserve(4 * (m.ne / std::max(1, leaf_size / 2) + 1));
    b.build(0, m.ne, 0);
    b.leaf_ranges(0);
    p.plane_tol = 1e-10 * Builder::diam(p.nodes[0]);
    b.planes(0);
    b.blocks(0, 0);
    p.iperm.resize(m.ne);
    for (int64_t q = 0; q < m.ne; ++q) p.iperm[p.perm[q]] = q;
    sort_blocks(p);
    return p;
}

}  // namespace hm
