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
//      Steps 1-2 depend on E, p and the active mask only and are kept
//      across tangents; a new D refreshes the values (E's part minus D on
//      the diagonal blocks) and redoes step 3.
//   3. ILU(0) on the GPU, one launch per colour: an element's three rows
//      only meet rows of earlier colours or its own earlier rows, so the
//      elements of a colour are factorised concurrently, one thread each.
//   4. Application: forward (unit L) and backward (U) substitution, one
//      launch per colour each, on a DOF-major copy of the vectors (16
//      lanes per element, one per column).
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

// The substitutions run on a DOF-major copy of the vectors: column c of
// DOF i at zt[16 i + c], so the 16 columns of a neighbour are one 128-byte
// line and one row entry (value, column) serves 16 lanes.
constexpr int kCols = 16;

// r [nrhs][ldr] -> zt [n][16] (columns >= nrhs zero), through an LDS tile
// of 64 DOFs so both sides are read and written contiguously
__global__ void k_ilu_to_dof_major(int64_t n, int nrhs, const double* __restrict__ r, int64_t ldr,
                                   double* __restrict__ zt)
{
    __shared__ double tile[64][kCols + 1];
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    for (int q = threadIdx.x; q < 64 * kCols; q += blockDim.x) {
        const int c = q / 64, i = q % 64;
        tile[i][c] = (c < nrhs && i0 + i < n) ? r[(int64_t)c * ldr + i0 + i] : 0.0;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 64 * kCols; q += blockDim.x) {
        const int i = q / kCols, c = q % kCols;
        if (i0 + i < n) zt[(i0 + i) * kCols + c] = tile[i][c];
    }
}

__global__ void k_ilu_from_dof_major(int64_t n, int nrhs, const double* __restrict__ zt, double* __restrict__ z,
                                     int64_t ldz)
{
    __shared__ double tile[64][kCols + 1];
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    for (int q = threadIdx.x; q < 64 * kCols; q += blockDim.x) {
        const int i = q / kCols, c = q % kCols;
        if (i0 + i < n) tile[i][c] = zt[(i0 + i) * kCols + c];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 64 * kCols; q += blockDim.x) {
        const int c = q / 64, i = q % 64;
        if (c < nrhs && i0 + i < n) z[(int64_t)c * ldz + i0 + i] = tile[i][c];
    }
}

// forward substitution (unit L) on the elements of one colour, in place in
// zt: 16 elements per workgroup, lane c of an element's 16 lanes = column c
__global__ void k_ilu_forward(const int32_t* __restrict__ elems, int n, const int64_t* __restrict__ rowptr,
                              const int32_t* __restrict__ col, const int64_t* __restrict__ diag,
                              const double* __restrict__ val, double* __restrict__ zt)
{
    const int slot = blockIdx.x * (blockDim.x / kCols) + threadIdx.x / kCols;
    const int c = threadIdx.x % kCols;
    if (slot >= n) return;
    const int e = elems[slot];
    for (int a = 0; a < 3; ++a) {
        const int64_t i = 3 * (int64_t)e + a;
        double s = zt[i * kCols + c];
        for (int64_t x = rowptr[i]; x < diag[i]; ++x) s -= val[x] * zt[(int64_t)col[x] * kCols + c];
        zt[i * kCols + c] = s;
    }
}

// backward substitution (U) on the elements of one colour, in place in zt
__global__ void k_ilu_backward(const int32_t* __restrict__ elems, int n, const int64_t* __restrict__ rowptr,
                               const int32_t* __restrict__ col, const int64_t* __restrict__ diag,
                               const double* __restrict__ val, double* __restrict__ zt)
{
    const int slot = blockIdx.x * (blockDim.x / kCols) + threadIdx.x / kCols;
    const int c = threadIdx.x % kCols;
    if (slot >= n) return;
    const int e = elems[slot];
    for (int a = 2; a >= 0; --a) {
        const int64_t i = 3 * (int64_t)e + a;
        const int64_t di = diag[i];
        double s = zt[i * kCols + c];
        for (int64_t x = di + 1; x < rowptr[i + 1]; ++x) s -= val[x] * zt[(int64_t)col[x] * kCols + c];
        zt[i * kCols + c] = s / val[di];
    }
}

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// The structure of the approximation for (fraction, active mask): the kept
// entries of E, the pattern, its colouring and elimination order, the CSR
// rows with E's part of the values (val0) and, per element, where its
// 3x3 diagonal block sits in them (dpos).  D does not enter: a new tangent
// with the same mask only refreshes the values.
void ilu_structure(Op& op, double fraction, const std::vector<uint8_t>& mask, hipStream_t s)
{
    IluPc& F = op.ilu;
    F.structure = false;
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
                if (!active(e) && a != b) continue;
                ent.push_back(Coo{3 * e + a, 3 * e + b, active(e) ? 0.0 : 1.0});
            }
    // element graph in both directions (CSR by a counting sort; duplicates kept)
    std::vector<int64_t> gptr(ne + 1, 0);
    for (const Coo& c : ent) {
        const int64_t e = c.row / 3, f = c.col / 3;
        if (e == f) continue;
        gptr[e + 1]++;
        gptr[f + 1]++;
    }
    for (int64_t e = 0; e < ne; ++e) gptr[e + 1] += gptr[e];
    std::vector<int32_t> gadj(gptr[ne]);
    {
        std::vector<int64_t> at(gptr.begin(), gptr.end() - 1);
        for (const Coo& c : ent) {
            const int64_t e = c.row / 3, f = c.col / 3;
            if (e == f) continue;
            gadj[at[e]++] = (int32_t)f;
            gadj[at[f]++] = (int32_t)e;
        }
    }
    // greedy colouring in increasing id
    std::vector<int32_t> colour(ne, -1);
    int n_colors = 0;
    {
        std::vector<int64_t> seen;   // seen[c] == e: colour c held by a lower-id neighbour of e
        for (int64_t e = 0; e < ne; ++e) {
            for (int64_t q = gptr[e]; q < gptr[e + 1]; ++q) {
                const int32_t f = gadj[q];
                if (f >= e) continue;
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
    // rows: bucket the entries by row, sort each row by elimination order,
    // sum duplicates (kept diagonal-block entries and -D)
    std::vector<int64_t> bptr(nd + 1, 0);
    for (const Coo& c : ent) bptr[c.row + 1]++;
    for (int64_t i = 0; i < nd; ++i) bptr[i + 1] += bptr[i];
    std::vector<std::pair<int64_t, double>> bucket(ent.size());   // (elimination key, value)
    std::vector<int32_t> bcol(ent.size());
    {
        std::vector<int64_t> at(bptr.begin(), bptr.end() - 1);
        for (const Coo& c : ent) {
            const int64_t q = at[c.row]++;
            bucket[q] = {3 * (int64_t)pos[c.col / 3] + c.col % 3, c.v};
            bcol[q] = (int32_t)c.col;
        }
    }
    std::vector<int64_t>().swap(gptr);
    std::vector<int32_t>().swap(gadj);
    std::vector<int64_t> rowptr(nd + 1, 0), diag(nd, -1);
    std::vector<int32_t> col;
    std::vector<double> val;
    col.reserve(ent.size());
    val.reserve(ent.size());
    std::vector<int64_t> idx;
    for (int64_t i = 0; i < nd; ++i) {
        const int64_t b = bptr[i], e = bptr[i + 1];
        idx.resize(e - b);
        std::iota(idx.begin(), idx.end(), b);
        std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) { return bucket[x].first < bucket[y].first; });
        const int64_t ikey = 3 * (int64_t)pos[i / 3] + i % 3;
        for (size_t q = 0; q < idx.size(); ++q) {
            const int64_t x = idx[q];
            if (q > 0 && bucket[x].first == bucket[idx[q - 1]].first) {
                val.back() += bucket[x].second;
                continue;
            }
            if (bucket[x].first == ikey) diag[i] = (int64_t)col.size();
            col.push_back(bcol[x]);
            val.push_back(bucket[x].second);
        }
        rowptr[i + 1] = (int64_t)col.size();
    }
    for (int64_t i = 0; i < nd; ++i) HM_REQUIRE(diag[i] >= 0, HM_EINTERNAL, "ILU: row without a diagonal entry");
    // where each active element's diagonal block sits in its three rows
    std::vector<int64_t> dpos(9 * ne, -1);
    for (int64_t e = 0; e < ne; ++e) {
        if (!active(e)) continue;
        for (int a = 0; a < 3; ++a) {
            const int64_t i = 3 * e + a;
            for (int64_t x = rowptr[i]; x < rowptr[i + 1]; ++x)
                if (col[x] / 3 == e) dpos[9 * e + 3 * a + col[x] % 3] = x;
        }
    }
    upload(F.order, order, s);
    upload(F.pos, pos, s);
    upload(F.rowptr, rowptr, s);
    upload(F.col, col, s);
    upload(F.diag, diag, s);
    upload(F.val0, val, s);
    upload(F.dpos, dpos, s);
    F.val.alloc(val.size() * sizeof(double));
    HM_CHECK_HIP(hipStreamSynchronize(s));
    F.color_begin = color_begin;
    F.n_colors = n_colors;
    F.nnz = (int64_t)col.size();
    F.n_kept = n_keep;
    F.near_entries = near_entries;
    F.threshold_key = kth;
    F.fraction = fraction;
    F.structure = true;
}

// val = val0 - D on the diagonal blocks of active elements (one thread per element)
__global__ void k_ilu_values(int64_t ne, const int64_t* __restrict__ dpos, const double* __restrict__ D,
                             double* __restrict__ val)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    for (int q = 0; q < 9; ++q) {
        const int64_t x = dpos[9 * e + q];
        if (x >= 0) val[x] -= D[9 * e + q];
    }
}

void ilu_pc_prepare(Op& op, double fraction, hipStream_t s)
{
    HM_REQUIRE(fraction > 0.0 && fraction <= 1.0, HM_EINVAL, "ILU fraction must be in (0, 1]");
    std::lock_guard<std::mutex> guard(op.pc_mu);
    IluPc& F = op.ilu;
    if (F.current && F.fraction == fraction) return;
    const double t0 = now_ms();
    F.current = false;
    const int64_t ne = op.ne;
    // the structure is kept while the fraction and the active mask stay the same
    std::vector<uint8_t> mask(op.has_mask ? ne : 0);
    if (op.has_mask) HM_CHECK_HIP(hipMemcpyAsync(mask.data(), op.d_mask.get(), ne, hipMemcpyDeviceToHost, s));
    HM_CHECK_HIP(hipStreamSynchronize(s));
    uint64_t key = 1469598103934665603ull ^ (uint64_t)op.has_mask;   // FNV-1a of the mask
    for (uint8_t b : mask) key = (key ^ (uint64_t)(b != 0)) * 1099511628211ull;
    if (!F.structure || F.fraction != fraction || F.mask_key != key) {
        ilu_structure(op, fraction, mask, s);
        F.mask_key = key;
    }
    // numeric factorisation of val0 - D, colour by colour
    HM_CHECK_HIP(hipMemcpyAsync(F.val.get(), F.val0.get(), F.nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (op.has_D)
        hipLaunchKernelGGL(k_ilu_values, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, ne,
                           F.dpos.as<int64_t>(), op.d_D.as<double>(), F.val.as<double>());
    DevBuf d_status(sizeof(int));
    HM_CHECK_HIP(hipMemsetAsync(d_status.get(), 0, sizeof(int), s));
    for (int c = 0; c < F.n_colors; ++c) {
        const int n = (int)(F.color_begin[c + 1] - F.color_begin[c]);
        hipLaunchKernelGGL(k_ilu_factor, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s,
                           F.order.as<int32_t>() + F.color_begin[c], n, F.pos.as<int32_t>(), F.rowptr.as<int64_t>(),
                           F.col.as<int32_t>(), F.diag.as<int64_t>(), F.val.as<double>(), d_status.as<int>());
    }
    HM_CHECK_HIP(hipGetLastError());
    int status = 0;
    HM_CHECK_HIP(hipMemcpyAsync(&status, d_status.get(), sizeof(int), hipMemcpyDeviceToHost, s));
    HM_CHECK_HIP(hipStreamSynchronize(s));
    HM_REQUIRE(status == 0, HM_EINVAL, "ILU(0) of the approximate tangent met a zero or non-finite pivot");
    F.setup_ms = now_ms() - t0;
    F.current = true;
}

void ilu_pc_apply(Op& op, int nrhs, const double* r, int64_t ldr, double* z, int64_t ldz, hipStream_t s)
{
    const IluPc& F = op.ilu;
    HM_REQUIRE(F.current, HM_EINTERNAL, "ILU preconditioner not prepared");
    HM_REQUIRE(nrhs >= 1 && nrhs <= kCols, HM_EINVAL, "nrhs must be in [1, 16]");
    const int64_t n = 3 * op.ne;
    double* zt = op.solve_workspace(s, (size_t)n * kCols * sizeof(double), kWsIlu);
    const unsigned tiles = (unsigned)((n + 63) / 64);
    hipLaunchKernelGGL(k_ilu_to_dof_major, dim3(tiles), dim3(256), 0, s, n, nrhs, r, ldr, zt);
    for (int c = 0; c < F.n_colors; ++c) {
        const int m = (int)(F.color_begin[c + 1] - F.color_begin[c]);
        hipLaunchKernelGGL(k_ilu_forward, dim3((unsigned)((m + 15) / 16)), dim3(256), 0, s,
                           F.order.as<int32_t>() + F.color_begin[c], m, F.rowptr.as<int64_t>(), F.col.as<int32_t>(),
                           F.diag.as<int64_t>(), F.val.as<double>(), zt);
    }
    for (int c = F.n_colors - 1; c >= 0; --c) {
        const int m = (int)(F.color_begin[c + 1] - F.color_begin[c]);
        hipLaunchKernelGGL(k_ilu_backward, dim3((unsigned)((m + 15) / 16)), dim3(256), 0, s,
                           F.order.as<int32_t>() + F.color_begin[c], m, F.rowptr.as<int64_t>(), F.col.as<int32_t>(),
                           F.diag.as<int64_t>(), F.val.as<double>(), zt);
    }
    hipLaunchKernelGGL(k_ilu_from_dof_major, dim3(tiles), dim3(256), 0, s, n, nrhs, zt, z, ldz);
    HM_CHECK_HIP(hipGetLastError());
}

}  // namespace hm
