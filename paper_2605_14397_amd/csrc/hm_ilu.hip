// The paper's sparse approximation of A11 and its incomplete LU
// factorisation, as a preconditioner of the A11 solves (Sec. 3.3.1,
// solution of the Jacobian system: the second choice of the approximate
// A11, C^ep plus a fraction p of the largest near-field entries of E,
// applied through an ILU factorisation).
//
//   1. Threshold: the near field is every entry of E in the dense
//      (inadmissible) leaf blocks of the operator.  Its coefficients are
//      evaluated on the GPU (FP64, the operator's own closed forms) and the
//      k-th largest magnitude key is found by four 12-bit histogram passes
//      over a 48-bit key of |a| (the IEEE bit pattern without its last 15
//      bits), k = ceil(p x entries); entries whose key reaches it are kept.
//   2. Pattern: the kept entries (gathered on the GPU), minus D = eta/dt +
//      C^ep on every 3x3 diagonal block; an inactive element keeps an
//      identity row and no coupling.  The host colours the elements
//      greedily (increasing id, smallest colour free among lower-id
//      neighbours) and sorts each row by elimination order: elements by
//      (colour, id), DOFs s1, s2, n.
//   3. ILU(0) on the GPU, one launch per colour: an element's three rows
//      only meet rows of earlier colours or its own earlier rows, so the
//      elements of a colour are factorised concurrently, one thread each.
//   4. Application: forward (unit L) and backward (U) substitution, one
//      launch per colour each, one thread per (element, column).
// Everything is FP64.  Rows keep the operator's original DOF numbering;
// only the order of entries inside a row follows the elimination order.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>

#include "hm_op.hpp"

namespace hm {

namespace {

constexpr int kKeyShift = 15;   // key = bits(|a|) >> 15: 48 bits
constexpr int kBinBits = 12;
constexpr int kBins = 1 << kBinBits;

// one dense block in cluster positions, and the first pair of each tile
struct NearDesc {
    int64_t t_begin, s_begin;
    int32_t m, n;
};
struct NearTile {
    int32_t block, first;   // block index, first element pair (of m n) of this tile of 256
};

__device__ inline uint64_t mag_key(double a)
{
    return (uint64_t)__double_as_longlong(fabs(a)) >> kKeyShift;
}

// pass q of the threshold search: histogram bits [47 - 12 q, 36 - 12 q] of
// the keys whose higher bits equal `prefix` (all keys for q = 0)
__global__ void k_near_hist(const ElemGeo* __restrict__ geo, const NearDesc* __restrict__ descs,
                            const NearTile* __restrict__ tiles, double kG, double kN, int pass, uint64_t prefix,
                            unsigned long long* __restrict__ hist)
{
    __shared__ unsigned int h[kBins];
    for (int i = threadIdx.x; i < kBins; i += blockDim.x) h[i] = 0u;
    __syncthreads();
    const NearTile T = tiles[blockIdx.x];
    const NearDesc D = descs[T.block];
    const int p = T.first + (int)threadIdx.x;
    if (p < D.m * D.n) {
        const int i = p / D.n, j = p - i * D.n;
        const ElemGeo& R = geo[D.t_begin + i];
        double blk[9];
        dd_block(R.c, R.fr, geo[D.s_begin + j], kG, kN, blk);
        const int hi_shift = 48 - kBinBits * pass;   // bits above this pass's field
        const int shift = hi_shift - kBinBits;
        for (int q = 0; q < 9; ++q) {
            const uint64_t key = mag_key(blk[q]);
            if (pass > 0 && (key >> hi_shift) != prefix) continue;
            atomicAdd(&h[(key >> shift) & (kBins - 1)], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kBins; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], (unsigned long long)h[i]);
}

// kept entries (key >= kth) appended as (row DOF, column DOF, value) in the
// original numbering; slots by an atomic counter (the host sorts them)
struct Coo {
    int64_t row, col;
    double v;
};

__global__ void k_near_gather(const ElemGeo* __restrict__ geo, const int64_t* __restrict__ perm,
                              const NearDesc* __restrict__ descs, const NearTile* __restrict__ tiles, double kG,
                              double kN, uint64_t kth, unsigned long long cap, unsigned long long* __restrict__ count,
                              Coo* __restrict__ out)
{
    const NearTile T = tiles[blockIdx.x];
    const NearDesc D = descs[T.block];
    const int p = T.first + (int)threadIdx.x;
    if (p >= D.m * D.n) return;
    const int i = p / D.n, j = p - i * D.n;
    const ElemGeo& R = geo[D.t_begin + i];
    double blk[9];
    dd_block(R.c, R.fr, geo[D.s_begin + j], kG, kN, blk);
    const int64_t er = perm[D.t_begin + i], ec = perm[D.s_begin + j];
    for (int q = 0; q < 9; ++q) {
        if (mag_key(blk[q]) < kth) continue;
        const unsigned long long slot = atomicAdd(count, 1ull);
        if (slot < cap) out[slot] = Coo{3 * er + q / 3, 3 * ec + q % 3, blk[q]};
    }
}

__device__ inline int64_t elim_key(const int32_t* __restrict__ pos, int32_t col)
{
    return 3 * (int64_t)pos[col / 3] + col % 3;
}

// ILU(0) of the rows of the elements of one colour (one thread per element):
// row i, for each k < i of its L part in elimination order: a_ik /= u_kk,
// then a_ij -= a_ik u_kj over the positions j > k present in both rows.
__global__ void k_ilu_factor(const int32_t* __restrict__ elems, int n, const int32_t* __restrict__ pos,
                             const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                             const int64_t* __restrict__ diag, double* __restrict__ val, int* __restrict__ status)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int e = elems[t];
    for (int a = 0; a < 3; ++a) {
        const int64_t i = 3 * (int64_t)e + a;
        const int64_t rb = rowptr[i], re = rowptr[i + 1], di = diag[i];
        for (int64_t x = rb; x < di; ++x) {
            const int32_t k = col[x];
            const double ukk = val[diag[k]];
            const double lik = val[x] / ukk;
            val[x] = lik;
            // merge row k's upper part (after its diagonal) with row i after x
            int64_t y = diag[k] + 1;
            const int64_t ye = rowptr[k + 1];
            int64_t z = x + 1;
            if (y >= ye || z >= re) continue;
            int64_t ky = elim_key(pos, col[y]), kz = elim_key(pos, col[z]);
            while (true) {
                if (ky == kz) {
                    val[z] -= lik * val[y];
                    if (++y >= ye || ++z >= re) break;
                    ky = elim_key(pos, col[y]);
                    kz = elim_key(pos, col[z]);
                } else if (ky < kz) {
                    if (++y >= ye) break;
                    ky = elim_key(pos, col[y]);
                } else {
                    if (++z >= re) break;
                    kz = elim_key(pos, col[z]);
                }
            }
        }
        const double piv = val[di];
        if (!(fabs(piv) > 0.0) || !isfinite(piv)) atomicExch(status, 1);
    }
}

// z = L^-1 r on the rows of one colour (unit L; earlier colours final)
__global__ void k_ilu_forward(const int32_t* __restrict__ elems, int n, int nrhs, const int64_t* __restrict__ rowptr,
                              const int32_t* __restrict__ col, const int64_t* __restrict__ diag,
                              const double* __restrict__ val, const double* __restrict__ r, int64_t ldr,
                              double* __restrict__ z, int64_t ldz)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nrhs) return;
    const int c = t % nrhs;
    const int e = elems[t / nrhs];
    const double* rc = r + (int64_t)c * ldr;
    double* zc = z + (int64_t)c * ldz;
    for (int a = 0; a < 3; ++a) {
        const int64_t i = 3 * (int64_t)e + a;
        double s = rc[i];
        for (int64_t x = rowptr[i]; x < diag[i]; ++x) s -= val[x] * zc[col[x]];
        zc[i] = s;
    }
}

// z = U^-1 z on the rows of one colour (later colours final)
__global__ void k_ilu_backward(const int32_t* __restrict__ elems, int n, int nrhs, const int64_t* __restrict__ rowptr,
                               const int32_t* __restrict__ col, const int64_t* __restrict__ diag,
                               const double* __restrict__ val, double* __restrict__ z, int64_t ldz)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nrhs) return;
    const int c = t % nrhs;
    const int e = elems[t / nrhs];
    double* zc = z + (int64_t)c * ldz;
    for (int a = 2; a >= 0; --a) {
        const int64_t i = 3 * (int64_t)e + a;
        double s = zc[i];
        const int64_t di = diag[i];
        for (int64_t x = di + 1; x < rowptr[i + 1]; ++x) s -= val[x] * zc[col[x]];
        zc[i] = s / val[di];
    }
}

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

void ilu_pc_prepare(Op& op, double fraction, hipStream_t s)
{
    HM_REQUIRE(fraction > 0.0 && fraction <= 1.0, HM_EINVAL, "ILU fraction must be in (0, 1]");
    std::lock_guard<std::mutex> guard(op.pc_mu);
    IluPc& F = op.ilu;
    if (F.current && F.fraction == fraction) return;
    const double t0 = now_ms();
    F.current = false;
    const int64_t ne = op.ne, nd = 3 * ne;
    HM_REQUIRE(nd < (int64_t)1 << 31, HM_EUNSUPPORTED, "ILU preconditioner: more than 2^31 DOFs");
    double G, kG, kN;
    moduli(op.young, op.nu, G, kG, kN);
    // ---- near-field blocks and their tiles ----
    const Plan& p = op.plan;
    std::vector<NearDesc> descs;
    std::vector<NearTile> tiles;
    int64_t near_entries = 0;
    for (const auto& b : p.dense) {
        const Cluster& t = p.nodes[b.first];
        const Cluster& sc = p.nodes[b.second];
        const int32_t m = (int32_t)t.size(), n = (int32_t)sc.size();
        const int32_t id = (int32_t)descs.size();
        descs.push_back(NearDesc{t.begin, sc.begin, m, n});
        for (int32_t f = 0; f < m * n; f += 256) tiles.push_back(NearTile{id, f});
        near_entries += 9 * (int64_t)m * n;
    }
    DevBuf d_descs, d_tiles;
    upload(d_descs, descs, s);
    upload(d_tiles, tiles, s);
    // ---- threshold: k-th largest key by four 12-bit histogram passes ----
    const int64_t k = std::max<int64_t>(1, (int64_t)std::ceil(fraction * (double)near_entries));
    DevBuf d_hist(kBins * sizeof(unsigned long long));
    std::vector<unsigned long long> hist(kBins);
    uint64_t prefix = 0;
    int64_t above = 0;   // kept keys strictly above the current prefix range
    for (int pass = 0; pass < 4; ++pass) {
        HM_CHECK_HIP(hipMemsetAsync(d_hist.get(), 0, d_hist.bytes(), s));
        for (size_t t0b = 0; t0b < tiles.size(); t0b += (1u << 30)) {
            const unsigned nb = (unsigned)std::min<size_t>(tiles.size() - t0b, (size_t)1 << 30);
            hipLaunchKernelGGL(k_near_hist, dim3(nb), dim3(256), 0, s, op.d_geo.as<ElemGeo>(),
                               d_descs.as<NearDesc>(), d_tiles.as<NearTile>() + t0b, kG, kN, pass, prefix,
                               d_hist.as<unsigned long long>());
        }
        HM_CHECK_HIP(hipGetLastError());
        HM_CHECK_HIP(hipMemcpyAsync(hist.data(), d_hist.get(), d_hist.bytes(), hipMemcpyDeviceToHost, s));
        HM_CHECK_HIP(hipStreamSynchronize(s));
        // walk down from the largest bin to the one holding the k-th key
        int bin = kBins - 1;
        for (; bin > 0; --bin) {
            if (above + (int64_t)hist[bin] >= k) break;
            above += (int64_t)hist[bin];
        }
        prefix = (prefix << kBinBits) | (uint64_t)bin;
    }
    const uint64_t kth = prefix;   // 48-bit key of the k-th largest magnitude
    // ---- gather the kept entries ----
    // count them: everything above plus every key equal to kth
    const int64_t n_keep = above + (int64_t)hist[kth & (kBins - 1)];
    DevBuf d_coo((size_t)std::max<int64_t>(1, n_keep) * sizeof(Coo)), d_cnt(sizeof(unsigned long long));
    HM_CHECK_HIP(hipMemsetAsync(d_cnt.get(), 0, d_cnt.bytes(), s));
    for (size_t t0b = 0; t0b < tiles.size(); t0b += (1u << 30)) {
        const unsigned nb = (unsigned)std::min<size_t>(tiles.size() - t0b, (size_t)1 << 30);
        hipLaunchKernelGGL(k_near_gather, dim3(nb), dim3(256), 0, s, op.d_geo.as<ElemGeo>(), op.d_perm.as<int64_t>(),
                           d_descs.as<NearDesc>(), d_tiles.as<NearTile>() + t0b, kG, kN, kth,
                           (unsigned long long)n_keep, d_cnt.as<unsigned long long>(), d_coo.as<Coo>());
    }
    HM_CHECK_HIP(hipGetLastError());
    unsigned long long got = 0;
    std::vector<Coo> coo((size_t)n_keep);
    HM_CHECK_HIP(hipMemcpyAsync(&got, d_cnt.get(), sizeof(got), hipMemcpyDeviceToHost, s));
    if (n_keep > 0)
        HM_CHECK_HIP(hipMemcpyAsync(coo.data(), d_coo.get(), n_keep * sizeof(Coo), hipMemcpyDeviceToHost, s));
    std::vector<double> D(op.has_D ? 9 * ne : 0);
    std::vector<uint8_t> mask(op.has_mask ? ne : 0);
    if (op.has_D) HM_CHECK_HIP(hipMemcpyAsync(D.data(), op.d_D.get(), D.size() * 8, hipMemcpyDeviceToHost, s));
    if (op.has_mask) HM_CHECK_HIP(hipMemcpyAsync(mask.data(), op.d_mask.get(), ne, hipMemcpyDeviceToHost, s));
    HM_CHECK_HIP(hipStreamSynchronize(s));
    HM_REQUIRE((int64_t)got == n_keep, HM_EINTERNAL, "ILU: kept-entry count differs between passes");
    auto active = [&](int64_t e) { return mask.empty() || mask[e] != 0; };
    // ---- pattern: kept entries between active elements, plus the diagonal blocks ----
    std::vector<Coo> ent;
    ent.reserve(coo.size() + 9 * ne);
    for (const Coo& c : coo)
        if (active(c.row / 3) && active(c.col / 3)) ent.push_back(c);
    for (int64_t e = 0; e < ne; ++e)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double v = 0.0;
                if (!active(e))
                    v = a == b ? 1.0 : 0.0;
                else if (op.has_D)
                    v = -D[9 * e + 3 * a + b];
                if (!active(e) && a != b) continue;
                ent.push_back(Coo{3 * e + a, 3 * e + b, v});
            }
    // element graph (both directions) and greedy colouring in increasing id
    std::vector<std::vector<int32_t>> adj(ne);
    for (const Coo& c : ent) {
        const int64_t e = c.row / 3, f = c.col / 3;
        if (e == f) continue;
        adj[e].push_back((int32_t)f);
        adj[f].push_back((int32_t)e);
    }
    std::vector<int32_t> colour(ne, -1);
    int n_colors = 0;
    {
        std::vector<int64_t> seen;   // seen[c] == e: colour c held by a lower-id neighbour of e
        for (int64_t e = 0; e < ne; ++e) {
            for (int32_t f : adj[e])
                if (f < e) {
                    const int32_t c = colour[f];
                    if ((size_t)c >= seen.size()) seen.resize(c + 1, -1);
                    seen[c] = e;
                }
            int32_t c = 0;
            while ((size_t)c < seen.size() && seen[c] == e) ++c;
            colour[e] = c;
            n_colors = std::max(n_colors, c + 1);
        }
    }
    std::vector<int32_t> order(ne), pos(ne);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return colour[a] < colour[b]; });
    for (int64_t q = 0; q < ne; ++q) pos[order[q]] = (int32_t)q;
    std::vector<int64_t> color_begin(n_colors + 1, 0);
    for (int64_t e = 0; e < ne; ++e) color_begin[colour[e] + 1]++;
    for (int c = 0; c < n_colors; ++c) color_begin[c + 1] += color_begin[c];
    // rows sorted by elimination order, duplicates (kept diagonal-block entries and -D) summed
    auto ekey = [&](int64_t d) { return 3 * (int64_t)pos[d / 3] + d % 3; };
    std::sort(ent.begin(), ent.end(), [&](const Coo& a, const Coo& b) {
        return a.row != b.row ? a.row < b.row : ekey(a.col) < ekey(b.col);
    });
    std::vector<int64_t> rowptr(nd + 1, 0), diag(nd, -1);
    std::vector<int32_t> col;
    std::vector<double> val;
    col.reserve(ent.size());
    val.reserve(ent.size());
    for (size_t q = 0; q < ent.size(); ++q) {
        if (!col.empty() && q > 0 && ent[q].row == ent[q - 1].row && ent[q].col == ent[q - 1].col) {
            val.back() += ent[q].v;
            continue;
        }
        rowptr[ent[q].row + 1]++;
        if (ent[q].col == ent[q].row) diag[ent[q].row] = (int64_t)col.size();
        col.push_back((int32_t)ent[q].col);
        val.push_back(ent[q].v);
    }
    for (int64_t i = 0; i < nd; ++i) rowptr[i + 1] += rowptr[i];
    for (int64_t i = 0; i < nd; ++i) HM_REQUIRE(diag[i] >= 0, HM_EINTERNAL, "ILU: row without a diagonal entry");
    // ---- upload and factorise colour by colour ----
    upload(F.order, order, s);
    upload(F.pos, pos, s);
    upload(F.rowptr, rowptr, s);
    upload(F.col, col, s);
    upload(F.diag, diag, s);
    upload(F.val, val, s);
    DevBuf d_status(sizeof(int));
    HM_CHECK_HIP(hipMemsetAsync(d_status.get(), 0, sizeof(int), s));
    for (int c = 0; c < n_colors; ++c) {
        const int n = (int)(color_begin[c + 1] - color_begin[c]);
        hipLaunchKernelGGL(k_ilu_factor, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s,
                           F.order.as<int32_t>() + color_begin[c], n, F.pos.as<int32_t>(), F.rowptr.as<int64_t>(),
                           F.col.as<int32_t>(), F.diag.as<int64_t>(), F.val.as<double>(), d_status.as<int>());
    }
    HM_CHECK_HIP(hipGetLastError());
    int status = 0;
    HM_CHECK_HIP(hipMemcpyAsync(&status, d_status.get(), sizeof(int), hipMemcpyDeviceToHost, s));
    HM_CHECK_HIP(hipStreamSynchronize(s));
    HM_REQUIRE(status == 0, HM_EINVAL, "ILU(0) of the approximate tangent met a zero or non-finite pivot");
    F.color_begin = color_begin;
    F.n_colors = n_colors;
    F.nnz = (int64_t)col.size();
    F.n_kept = n_keep;
    F.near_entries = near_entries;
    F.threshold_key = kth;
    F.fraction = fraction;
    F.setup_ms = now_ms() - t0;
    F.current = true;
}

void ilu_pc_apply(const Op& op, int nrhs, const double* r, int64_t ldr, double* z, int64_t ldz, hipStream_t s)
{
    const IluPc& F = op.ilu;
    HM_REQUIRE(F.current, HM_EINTERNAL, "ILU preconditioner not prepared");
    for (int c = 0; c < F.n_colors; ++c) {
        const int n = (int)(F.color_begin[c + 1] - F.color_begin[c]);
        hipLaunchKernelGGL(k_ilu_forward, dim3((unsigned)((n * nrhs + 255) / 256)), dim3(256), 0, s,
                           F.order.as<int32_t>() + F.color_begin[c], n, nrhs, F.rowptr.as<int64_t>(),
                           F.col.as<int32_t>(), F.diag.as<int64_t>(), F.val.as<double>(), r, ldr, z, ldz);
    }
    for (int c = F.n_colors - 1; c >= 0; --c) {
        const int n = (int)(F.color_begin[c + 1] - F.color_begin[c]);
        hipLaunchKernelGGL(k_ilu_backward, dim3((unsigned)((n * nrhs + 255) / 256)), dim3(256), 0, s,
                           F.order.as<int32_t>() + F.color_begin[c], n, nrhs, F.rowptr.as<int64_t>(),
                           F.col.as<int32_t>(), F.diag.as<int64_t>(), F.val.as<double>(), z, ldz);
    }
    HM_CHECK_HIP(hipGetLastError());
}

}  // namespace hm
