// H-matrix product Y = E X (paper Sec. 3.1: the hierarchical matrix brings
// the product E . delta from O(n^2) to O(n log n); it sits inside the
// Krylov solve of the tangent system, Sec. 3.3.1).
//
// Structure of one product (all stages are HIP kernels on one stream):
//   gather   X (FP64, element order) -> per-leaf fragment chunks (working
//            precisions; BF16 as a hi/lo pair), inactive elements zeroed
//   phase A  for every low-rank block b: T_b = V_b^T X_sigma   (MFMA)
//   reduce   T_b = sum of phase-A partials in a fixed order
//   phase B  for every target leaf t: Y_t = sum D X_sigma + sum U_b[t] T_b
//            (MFMA), one workgroup owns the leaf: no atomics, fixed order
//   scatter  Y -> FP64 element order, + FP64 self blocks (mixed forms),
//            tangent epilogue y = E x - D x, identity on inactive elements
// The matrix streams from HBM once per product; X and T chunks are small
// and re-read from cache.
#include <type_traits>

#include "hm_op.hpp"
#include "hm_util.hpp"

namespace hm {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// ---- per storage type: 16-byte granule and MFMA step ----
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

template <class T>
struct Mma;

template <>
struct Mma<double> {
    static constexpr int w = 2;
    // two 16x16x4 FP64 products: k = 2g + t
    template <class A>
    __device__ static A run(u4 ra, u4 rb, u4, A c)
    {
        d2 a = __builtin_bit_cast(d2, ra), b = __builtin_bit_cast(d2, rb);
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], c, 0, 0, 0);
        return c;
    }
};

template <>
struct Mma<float> {
    static constexpr int w = 4;
    // four 16x16x4 FP32 products: k = 4g + t
    template <class A>
    __device__ static A run(u4 ra, u4 rb, u4, A c)
    {
        f4 a = __builtin_bit_cast(f4, ra), b = __builtin_bit_cast(f4, rb);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], c, 0, 0, 0);
        return c;
    }
};

template <>
struct Mma<uint16_t> {
    static constexpr int w = 8;
    // one 16x16x32 BF16 product per half of the split in-vector (hi + lo)
    template <class A>
    __device__ static A run(u4 ra, u4 rbh, u4 rbl, A c)
    {
        bf8 a = __builtin_bit_cast(bf8, ra);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf8, rbh), c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf8, rbl), c, 0, 0, 0);
        return c;
    }
};

// BF16 in-vectors without a lo half (one product per k-step)
struct bf16s {
    uint16_t bits;
};

template <>
struct Mma<bf16s> {
    static constexpr int w = 8;
    template <class A>
    __device__ static A run(u4 ra, u4 rb, u4, A c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, ra), __builtin_bit_cast(bf8, rb), c, 0,
                                                        0, 0);
    }
};

template <class A>
struct AccScalar;
// Row of the 16x16 result held by (lane, register v); the column is lane % 16.
// FP32 results hold four consecutive rows per lane group, FP64 results hold
// rows interleaved by lane group (checked with integer-valued inputs).
template <>
struct AccScalar<f4> {
    typedef float type;
    __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <>
struct AccScalar<d4> {
    typedef double type;
    __device__ static int row(int lane, int v) { return 4 * v + (lane >> 4); }
};

// Workgroups are dealt to the 8 XCDs round-robin: workgroup bid runs on
// XCD bid & 7 as that XCD's (bid >> 3)-th.  Each XCD takes its own
// contiguous task range (neighbouring leaves share one L2), per = tasks per
// workgroup.
__device__ inline int xcd_task(int bid, const XcdSplit& sp, int per, int sub)
{
    const int x = bid & 7;
    const int t = sp.begin[x] + per * (bid >> 3) + sub;
    return t < sp.begin[x + 1] ? t : -1;
}

__host__ inline unsigned xcd_grid(const XcdSplit& sp, int per)
{
    int m = 0;
    for (int x = 0; x < 8; ++x) m = std::max(m, (sp.begin[x + 1] - sp.begin[x] + per - 1) / per);
    return 8u * (unsigned)m;
}

// Queue-driven launches (merged batches): as many workgroups as fit on the
// chip at once; workgroup b belongs to XCD b & 7 and works on that XCD's
// range.  The first tasks of a range go one to each of its wavefronts
// (phase A) or workgroups (phase B) by index; the rest are claimed through
// the range's counter, the claim of the next task in flight while the
// current one runs.  A wavefront or workgroup whose range is empty claims
// from the other ranges.  Claims are taken in range order; every task runs
// exactly once.
__device__ inline int claim_wave(int* q, int lane)
{
    int t = 0;
    if (lane == 0) t = atomicAdd(q, 1);
    return __builtin_amdgcn_readfirstlane(t);
}

// true when the range's counter has reached `left` claims (a plain read)
__device__ inline bool range_done(const int* q, int left)
{
    return __builtin_amdgcn_readfirstlane(__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >= left;
}

// Workgroups of a queue-driven launch: as many as are resident at once
// (registers and LDS of the kernel's build, compute units of the device), a
// multiple of 8, at least 8.  Callers cap it by what the tasks can use.
static unsigned queue_grid(const void* kernel)
{
    int dev = 0, cus = 0, per_cu = 0;
    HM_CHECK_HIP(hipGetDevice(&dev));
    HM_CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HM_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0));
    const int64_t g = (int64_t)std::max(1, per_cu) * std::max(1, cus);
    return (unsigned)std::max<int64_t>(8, g / 8 * 8);
}

// Buffers of one operand pair: A panels and the in-vector chunks they read.
struct Side {
    const char* A;     // panel storage
    const char* Bhi;   // in-vector chunks (X or T), hi part
    const char* Blo;   // lo part (BF16 split) or null
    int es, w;         // element bytes, elements per 16-byte granule
};

// One unit of work: k-step ks of one panel, all its row tiles.  A unit past
// the end of a task is "empty": its loads go through zero-size buffer
// resources and return zeros, so every loop iteration issues the same loads
// and the compiler can keep the next unit's loads in flight while the
// current one is multiplied.
struct Unit {
    const char* a;     // first granule of the k-step
    const char* bh;    // the k-step's in-vector granules (lane 0)
    const char* bl;
    int gg;            // granules in this k-step (1..4)
    int far;
    int valid;
};

// Walks the flattened sequence of (panel, k-step) units of a task.
struct Cursor {
    const PanelRef* items;
    int n_items, item, base, nks;
    PanelRef P;
    __device__ void init(const PanelRef* it, int n, int kstep_near, int kstep_far)
    {
        items = it;
        n_items = n;
        item = 0;
        base = 0;
        if (n > 0) {
            P = items[0];
            nks = (P.cols + (P.far ? kstep_far : kstep_near) - 1) / (P.far ? kstep_far : kstep_near);
        }
    }
    // position on unit u (u never decreases); false past the end
    __device__ bool seek(int u, int kstep_near, int kstep_far)
    {
        while (item < n_items && u >= base + nks) {
            base += nks;
            ++item;
            if (item < n_items) {
                P = items[item];
                const int ks = P.far ? kstep_far : kstep_near;
                nks = (P.cols + ks - 1) / ks;
            }
        }
        return item < n_items;
    }
};

__device__ inline Unit make_unit(const Cursor& c, bool valid, int u, int rows, const Side& nearS, const Side& farS)
{
    Unit x;
    x.valid = valid ? 1 : 0;
    if (!valid) {
        x.a = nearS.A;
        x.bh = nearS.Bhi;
        x.bl = nullptr;
        x.gg = 4;
        x.far = 0;
        return x;
    }
    const Side& S = c.P.far ? farS : nearS;
    const int ks = u - c.base;
    const int Gr = (c.P.cols + S.w - 1) / S.w;
    x.gg = min(4, Gr - 4 * ks);
    x.a = S.A + (int64_t)c.P.a_off * S.es + (int64_t)ks * rows * 64;
    const int64_t boff = (int64_t)c.P.b_off * S.es + (int64_t)ks * 64 * 16;
    x.bh = S.Bhi + boff;
    x.bl = S.Blo ? S.Blo + boff : nullptr;
    x.far = c.P.far;
    return x;
}

// Loads of all R row tiles of one unit through a raw buffer resource over
// the unit's chunk: the row-tile offset is a scalar, lanes outside the
// panel get an out-of-range offset and read zero (raw buffer range check).
__device__ inline __amdgpu_buffer_rsrc_t chunk_rsrc(const char* base, uint32_t bytes)
{
    // the base and size are wave-uniform by construction; say so explicitly
    const uint64_t b = reinterpret_cast<uint64_t>(base);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    char* p = reinterpret_cast<char*>(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)__builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}

// Cache policy of the panel loads: every panel byte is read once per
// product, so the loads are marked non-temporal (they stream past the
// caches that keep the X and T chunks, which are re-read).
constexpr int kPanelAux = 2;

// Tiles r0 .. r0 + R - 1 of the unit's panel (rows rows, Rf = ceil(rows / 16)
// tiles; the last may be partial); tiles at or past Rf read zero.
template <int R, bool LO>
__device__ __attribute__((always_inline)) inline void load_unit(const Unit& x, int rows, int r0, int lane, u4 (&a)[R],
                                                                 u4& bh, u4& bl)
{
    const int g = lane >> 4, i = lane & 15;
    const uint32_t kOut = 0x80000000u;
    const int gg = __builtin_amdgcn_readfirstlane(x.gg);
    const int Rf = __builtin_amdgcn_readfirstlane((rows + 15) >> 4);
    r0 = __builtin_amdgcn_readfirstlane(r0);
    const bool gok = g < gg;
    const int rr_last = rows - 16 * (Rf - 1);
    const uint32_t vfull = gok ? 16u * (uint32_t)(16 * g + i) : kOut;
    const uint32_t vlast = (gok && i < rr_last) ? 16u * (uint32_t)(g * rr_last + i) : kOut;
    const __amdgpu_buffer_rsrc_t rs = chunk_rsrc(x.a, x.valid ? (uint32_t)(rows * gg * 16) : 0u);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int t = r0 + r;
        a[r] = __builtin_bit_cast(u4, __builtin_amdgcn_raw_buffer_load_b128(
                                          rs, t < Rf - 1 ? vfull : (t == Rf - 1 ? vlast : kOut), t * 256 * gg,
                                          kPanelAux));
    }
    // the in-vector k-step: 64 granules, one per lane
    const __amdgpu_buffer_rsrc_t rb = chunk_rsrc(x.bh, x.valid ? 1024u : 0u);
    bh = __builtin_bit_cast(u4, __builtin_amdgcn_raw_buffer_load_b128(rb, 16u * (uint32_t)lane, 0, 0));
    if constexpr (LO) {
        const __amdgpu_buffer_rsrc_t rl = chunk_rsrc(x.bl ? x.bl : x.bh, (x.valid && x.bl) ? 1024u : 0u);
        bl = __builtin_bit_cast(u4, __builtin_amdgcn_raw_buffer_load_b128(rl, 16u * (uint32_t)lane, 0, 0));
    } else {
        bl = u4{0, 0, 0, 0};  // no lo part in this form (only BF16 in-vectors are split)
    }
}

// Every launch (phase A and B) is compiled for its tasks' own row-tile
// count, so all R tiles are multiplied (a partial last tile reads zeros).
template <int R, class NT, class FT, class ACC>
__device__ __attribute__((always_inline)) inline void mma_unit(int far, const u4 (&a)[R], u4 bh, u4 bl,
                                                                ACC (&acc)[R])
{
    if constexpr (std::is_same<NT, FT>::value) {
        // one element type: no branch (keeps the loop straight for the wait counters)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = Mma<NT>::run(a[r], bh, bl, acc[r]);
        return;
    }
    if (far) {
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = Mma<FT>::run(a[r], bh, bl, acc[r]);
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = Mma<NT>::run(a[r], bh, bl, acc[r]);
    }
}

// Accumulate this wave's units u0, u0 + step, ... of one task.  The loads
// of the next units are in flight while the current one is multiplied: two
// units ahead for up to 4 row tiles, one unit ahead for more (register
// budget).  Loads are issued unconditionally (empty units past the end), so
// the control flow around them is static.
template <int R, class NT, class FT, class ACC>
__device__ __attribute__((always_inline)) inline void stream_units(const PanelRef* items, int n_items, int rows,
                                                                    int r0, const Side& nearS, const Side& farS,
                                                                    int u0, int step, int lane, ACC (&acc)[R])
{
    // only BF16 in-vectors carry a lo part
    constexpr bool kLo = std::is_same<FT, uint16_t>::value;
    const int ksn = 4 * nearS.w, ksf = 4 * farS.w;
    Cursor c;
    c.init(items, n_items, ksn, ksf);
    int u = u0;
    if (!c.seek(u, ksn, ksf)) return;
    if constexpr (R <= 4) {
        u4 a0[R], a1[R], a2[R], b0h, b0l, b1h, b1l, b2h, b2l;
        Unit x0 = make_unit(c, true, u, rows, nearS, farS);
        load_unit<R, kLo>(x0, rows, r0, lane, a0, b0h, b0l);
        bool vb = c.seek(u + step, ksn, ksf);
        Unit x1 = make_unit(c, vb, u + step, rows, nearS, farS);
        load_unit<R, kLo>(x1, rows, r0, lane, a1, b1h, b1l);
        while (true) {
            const bool vc = c.seek(u + 2 * step, ksn, ksf);
            const Unit x2 = make_unit(c, vc, u + 2 * step, rows, nearS, farS);
            load_unit<R, kLo>(x2, rows, r0, lane, a2, b2h, b2l);
            mma_unit<R, NT, FT, ACC>(x0.far, a0, b0h, b0l, acc);
            if (!vb) break;
            const bool vd = c.seek(u + 3 * step, ksn, ksf);
            x0 = make_unit(c, vd, u + 3 * step, rows, nearS, farS);
            load_unit<R, kLo>(x0, rows, r0, lane, a0, b0h, b0l);
            mma_unit<R, NT, FT, ACC>(x1.far, a1, b1h, b1l, acc);
            if (!vc) break;
            const bool ve = c.seek(u + 4 * step, ksn, ksf);
            x1 = make_unit(c, ve, u + 4 * step, rows, nearS, farS);
            load_unit<R, kLo>(x1, rows, r0, lane, a1, b1h, b1l);
            mma_unit<R, NT, FT, ACC>(x2.far, a2, b2h, b2l, acc);
            if (!vd) break;
            // a0 now holds unit u + 3 step, a1 unit u + 4 step
            u += 3 * step;
            vb = ve;
        }
    } else {
        u4 a0[R], a1[R], b0h, b0l, b1h, b1l;
        Unit x0 = make_unit(c, true, u, rows, nearS, farS);
        load_unit<R, kLo>(x0, rows, r0, lane, a0, b0h, b0l);
        while (true) {
            const bool v1 = c.seek(u + step, ksn, ksf);
            const Unit x1 = make_unit(c, v1, u + step, rows, nearS, farS);
            load_unit<R, kLo>(x1, rows, r0, lane, a1, b1h, b1l);
            mma_unit<R, NT, FT, ACC>(x0.far, a0, b0h, b0l, acc);
            if (!v1) break;
            const bool v2 = c.seek(u + 2 * step, ksn, ksf);
            x0 = make_unit(c, v2, u + 2 * step, rows, nearS, farS);
            load_unit<R, kLo>(x0, rows, r0, lane, a0, b0h, b0l);
            mma_unit<R, NT, FT, ACC>(x1.far, a1, b1h, b1l, acc);
            if (!v2) break;
            u += 2 * step;
        }
    }
}

// Sum the four waves' accumulators in a fixed order; wave 0 writes the
// window's rows 16 (r0 + r) + i below rows.
template <int R, class ACC, class S>
__device__ __attribute__((always_inline)) inline void reduce_and_store(ACC (&acc)[R], int rows, int r0,
                                                                        S* __restrict__ out, int64_t row0, S* red,
                                                                        int wave, int lane)
{
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (wave > 0)
            for (int v = 0; v < 4; ++v) red[(wave - 1) * 256 + lane * 4 + v] = acc[r][v];
        __syncthreads();
        if (wave == 0) {
            for (int v = 0; v < 4; ++v) {
                S s = acc[r][v] + red[lane * 4 + v];
                s += red[256 + lane * 4 + v];
                s += red[512 + lane * 4 + v];
                int row = 16 * (r0 + r) + AccScalar<ACC>::row(lane, v);
                if (row < rows) out[(row0 + row) * kNrhs + (lane & 15)] = s;
            }
        }
        __syncthreads();
    }
}

template <class NT, class FT>
struct Sides {
    Side nearS, farS;
};

// ------------------------------------------------------------------
// phase A: one wavefront per task; T partial = sum of its V^T sub-panels x X
// ------------------------------------------------------------------
// T value -> far-precision fragment entry (BF16 as a hi/lo pair)
template <class FT, class S>
__device__ inline void store_t(FT* __restrict__ thi, FT* __restrict__ tlo, int64_t off, S v)
{
    if constexpr (std::is_same<FT, uint16_t>::value) {
        float f = (float)v;
        uint16_t h = f32_to_bf16_bits(f);
        thi[off] = h;
        tlo[off] = f32_to_bf16_bits(f - bf16_bits_to_f32(h));
    } else if constexpr (std::is_same<FT, bf16s>::value) {
        thi[off] = bf16s{f32_to_bf16_bits((float)v)};
    } else {
        thi[off] = (FT)v;
    }
}

template <int R, class NT, class FT, class ACC>
__device__ void phaseA_wave(const TaskA& T, const PanelRef* items, const MemberT* __restrict__ members,
                            const Side& farS, typename AccScalar<ACC>::type* __restrict__ tpart,
                            FT* __restrict__ thi, FT* __restrict__ tlo, int lane)
{
    ACC acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = ACC{0, 0, 0, 0};
    stream_units<R, NT, FT, ACC>(items + T.item_begin, T.n_items, T.rows, T.r0, farS, farS, 0, 1, lane, acc);
    // only the window's own tiles (r0 .. r0 + R - 1 below ceil(K / 16)) are
    // written; rows past the stacked K hold zeros and belong to no member
    const int Rf = __builtin_amdgcn_readfirstlane((T.rows + 15) >> 4);
    if (T.direct) {
        // the task covers every source leaf: each member's rows go to its
        // own T chunk (a member's T rows past its rank stay zero)
        for (int j = 0; j < T.n_mem; ++j) {
            const MemberT M = members[T.mem_begin + j];
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (T.r0 + r < Rf)
                    for (int v = 0; v < 4; ++v) {
                        const int q = 16 * (T.r0 + r) + AccScalar<ACC>::row(lane, v) - M.lo;
                        if (q >= 0 && q < M.rows)
                            store_t<FT>(thi, tlo, M.t_off + bfrag_offset(Mma<FT>::w, q, lane & 15), acc[r][v]);
                    }
        }
        return;
    }
    auto* out = tpart + T.out_off;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (T.r0 + r < Rf)
            for (int v = 0; v < 4; ++v)
                out[(16 * (T.r0 + r) + AccScalar<ACC>::row(lane, v)) * kNrhs + (lane & 15)] = acc[r][v];
}

// Phase A runs one launch for every task, one wavefront per task; the
// window height (1 to 4 row tiles) is compiled per case and picked per task
// (wave-uniform).
template <class FT, class ACC>
__device__ __attribute__((always_inline)) inline void phaseA_task(const TaskA T, const PanelRef* items,
                                                                   const MemberT* members, const Bases* bases,
                                                                   int lane)
{
    typedef typename AccScalar<ACC>::type S;
    const Bases B = bases[T.op];
    const Side farS{reinterpret_cast<const char*>(B.farA), reinterpret_cast<const char*>(B.xfhi),
                    reinterpret_cast<const char*>(B.xflo), (int)sizeof(FT), Mma<FT>::w};
    S* tp = static_cast<S*>(B.tpart);
    FT* th = static_cast<FT*>(B.thi);
    FT* tl = static_cast<FT*>(B.tlo);
    switch (__builtin_amdgcn_readfirstlane(window_tiles(T.rows, T.r0))) {
        case 1: phaseA_wave<1, FT, FT, ACC>(T, items, members, farS, tp, th, tl, lane); break;
        case 2: phaseA_wave<2, FT, FT, ACC>(T, items, members, farS, tp, th, tl, lane); break;
        case 3: phaseA_wave<3, FT, FT, ACC>(T, items, members, farS, tp, th, tl, lane); break;
        default: phaseA_wave<4, FT, FT, ACC>(T, items, members, farS, tp, th, tl, lane); break;
    }
}

// One workgroup per four tasks (one per wavefront) in XCD-range order: the
// hardware deals the workgroups out as slots free up.
template <class FT, class ACC>
__global__ __launch_bounds__(256) void k_phaseA(const TaskA* __restrict__ tasks, XcdSplit sp,
                                                const PanelRef* __restrict__ items,
                                                const MemberT* __restrict__ members, const Bases* __restrict__ bases)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int t = xcd_task(blockIdx.x, sp, 4, wave);
    if (t < 0) return;
    phaseA_task<FT, ACC>(tasks[t], items, members, bases, lane);
}

// The resident workgroups work through the XCD ranges' queues, one task
// per wavefront at a time.
template <class FT, class ACC>
__global__ __launch_bounds__(256) void k_phaseA_q(const TaskA* __restrict__ tasks, XcdSplit sp,
                                                  const PanelRef* __restrict__ items,
                                                  const MemberT* __restrict__ members,
                                                  const Bases* __restrict__ bases, int* __restrict__ queue)
{
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int home = blockIdx.x & 7;
    const int nstatic = (gridDim.x >> 3) * 4, mine = (blockIdx.x >> 3) * 4 + wave;
    for (int j = 0; j < 8; ++j) {
        const int x = (home + j) & 7;
        const int first = sp.begin[x], n = sp.begin[x + 1] - first;
        int* q = queue + x * kQueueStride;
        int t = mine;
        if (j > 0) {
            if (range_done(q, n - nstatic)) continue;
            t = nstatic + claim_wave(q, lane);
        }
        while (t < n) {
            const int next = nstatic + claim_wave(q, lane);
            phaseA_task<FT, ACC>(tasks[first + t], items, members, bases, lane);
            t = next;
        }
    }
}

// ------------------------------------------------------------------
// reduce phase-A partials into T fragment chunks (far precision)
// ------------------------------------------------------------------
template <class FT, class S>
__global__ void k_reduceT(const ReduceDesc* __restrict__ rd, const Bases* __restrict__ bases)
{
    const ReduceDesc D = rd[blockIdx.x];
    const Bases B = bases[D.op];
    const S* tpart = static_cast<const S*>(B.tpart);
    FT* thi = static_cast<FT*>(B.thi);
    FT* tlo = static_cast<FT*>(B.tlo);
    const int Kp = (int)round_up(D.rank, kChunkAlign);
    const int64_t slot = D.slot_stride;
    constexpr int w = Mma<FT>::w;
    for (int e = threadIdx.x; e < Kp * kNrhs; e += blockDim.x) {
        const int row = e / kNrhs, c = e - row * kNrhs;
        S v = 0;
        if (row < D.rank) {
            // the loads of eight slots go out together; the sum keeps slot order
            const S* src = tpart + D.slot_begin + (int64_t)row * kNrhs + c;
            int s = 0;
            for (; s + 8 <= D.n_slots; s += 8) {
                S t[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) t[q] = src[(int64_t)(s + q) * slot];
#pragma unroll
                for (int q = 0; q < 8; ++q) v += t[q];
            }
            for (; s < D.n_slots; ++s) v += src[(int64_t)s * slot];
        }
        store_t<FT>(thi, tlo, D.t_off + bfrag_offset(w, row, c), v);
    }
}

// ------------------------------------------------------------------
// phase B: one workgroup per target leaf, its four waves share the units
// ------------------------------------------------------------------
template <int R, class NT, class FT, class ACC>
__device__ void phaseB_task(const TaskB& T, const PanelRef* items, const Side& nearS, const Side& farS,
                            typename AccScalar<ACC>::type* __restrict__ Y, typename AccScalar<ACC>::type* red,
                            int wave, int lane)
{
    ACC acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = ACC{0, 0, 0, 0};
    stream_units<R, NT, FT, ACC>(items + T.item_begin, T.n_items, T.rows, T.r0, nearS, farS, wave, 4, lane, acc);
    reduce_and_store<R, ACC>(acc, T.rows, T.r0, Y, T.y_off, red, wave, lane);
}

// Phase B runs one launch for every task, one workgroup per task (its four
// waves share the units); the window height (1 to WMAX row tiles) is
// compiled per case and picked per task.  Task lists whose windows are at
// most 4 tiles high launch the WMAX = 4 build, whose smaller register
// footprint keeps more waves per SIMD resident.
template <class NT, class FT, class ACC, int WMAX>
__device__ __attribute__((always_inline)) inline void phaseB_one(const TaskB T, const PanelRef* items,
                                                                  const Bases* bases,
                                                                  typename AccScalar<ACC>::type* red, int wave,
                                                                  int lane)
{
    typedef typename AccScalar<ACC>::type S;
    const Bases B = bases[T.op];
    const Side nearS{reinterpret_cast<const char*>(B.nearA), reinterpret_cast<const char*>(B.xnear), nullptr,
                     (int)sizeof(NT), Mma<NT>::w};
    const Side farS{reinterpret_cast<const char*>(B.farA), reinterpret_cast<const char*>(B.thi),
                    reinterpret_cast<const char*>(B.tlo), (int)sizeof(FT), Mma<FT>::w};
    S* y = static_cast<S*>(B.y);
    switch (__builtin_amdgcn_readfirstlane(T.nt)) {
        case 1: phaseB_task<1, NT, FT, ACC>(T, items, nearS, farS, y, red, wave, lane); break;
        case 2: phaseB_task<2, NT, FT, ACC>(T, items, nearS, farS, y, red, wave, lane); break;
        case 3: phaseB_task<3, NT, FT, ACC>(T, items, nearS, farS, y, red, wave, lane); break;
        default:
            if constexpr (WMAX == 4) {
                phaseB_task<4, NT, FT, ACC>(T, items, nearS, farS, y, red, wave, lane);
            } else {
                switch (__builtin_amdgcn_readfirstlane(T.nt)) {
                    case 4: phaseB_task<4, NT, FT, ACC>(T, items, nearS, farS, y, red, wave, lane); break;
                    case 5: phaseB_task<5, NT, FT, ACC>(T, items, nearS, farS, y, red, wave, lane); break;
                    case 6: phaseB_task<6, NT, FT, ACC>(T, items, nearS, farS, y, red, wave, lane); break;
                    case 7: phaseB_task<7, NT, FT, ACC>(T, items, nearS, farS, y, red, wave, lane); break;
                    default: phaseB_task<8, NT, FT, ACC>(T, items, nearS, farS, y, red, wave, lane); break;
                }
            }
            break;
    }
}

// One workgroup per task in XCD-range order.
template <class NT, class FT, class ACC, int WMAX>
__global__ __launch_bounds__(256) void k_phaseB(const TaskB* __restrict__ tasks, XcdSplit sp,
                                                const PanelRef* __restrict__ items, const Bases* __restrict__ bases)
{
    typedef typename AccScalar<ACC>::type S;
    __shared__ S red[3 * 256];
    const int t = xcd_task(blockIdx.x, sp, 1, 0);
    if (t < 0) return;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    phaseB_one<NT, FT, ACC, WMAX>(tasks[t], items, bases, red, wave, lane);
}

// The resident workgroups work through the XCD ranges' queues, one task
// per workgroup at a time.
template <class NT, class FT, class ACC, int WMAX>
__global__ __launch_bounds__(256) void k_phaseB_q(const TaskB* __restrict__ tasks, XcdSplit sp,
                                                  const PanelRef* __restrict__ items,
                                                  const Bases* __restrict__ bases, int* __restrict__ queue)
{
    typedef typename AccScalar<ACC>::type S;
    __shared__ S red[3 * 256];
    __shared__ int claimed;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int home = blockIdx.x & 7;
    const int nstatic = gridDim.x >> 3, mine = blockIdx.x >> 3;
    for (int j = 0; j < 8; ++j) {
        const int x = (home + j) & 7;
        const int first = sp.begin[x], n = sp.begin[x + 1] - first;
        int* q = queue + (8 + x) * kQueueStride;
        // thread 0 decides for the whole workgroup
        if (threadIdx.x == 0)
            claimed = j == 0 ? mine : range_done(q, n - nstatic) ? n : nstatic + atomicAdd(q, 1);
        __syncthreads();
        int t = __builtin_amdgcn_readfirstlane(claimed);
        __syncthreads();
        while (t < n) {
            int next = 0;
            if (threadIdx.x == 0) next = nstatic + atomicAdd(q, 1);
            phaseB_one<NT, FT, ACC, WMAX>(tasks[first + t], items, bases, red, wave, lane);
            if (threadIdx.x == 0) claimed = next;
            __syncthreads();
            t = __builtin_amdgcn_readfirstlane(claimed);
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------
// gather / scatter: one workgroup per leaf, through an LDS tile of the
// leaf's chunk (dofs x 16 columns), so the fragment-ordered chunk is read or
// written in memory order and the FP64 vectors element by element
// ------------------------------------------------------------------
// The workgroup's segment: the last one whose first leaf is at or below b.
__device__ inline int segment_of(const Segment* __restrict__ segs, int nseg, int b)
{
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].leaf0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// dof q of a chunk and column c at fragment offset o (inverse of bfrag_offset)
template <int W>
__device__ inline void frag_dof(int64_t o, int& q, int& c)
{
    const int t = (int)(o % W);
    const int64_t r = o / W;
    c = (int)(r % kNrhs);
    q = (int)(r / kNrhs) * W + t;
}

template <class NT, class FT>
__device__ inline void gather_leaf(const Segment& S, const Bases& B, int nrhs, int l)
{
    __shared__ double xs[kLeafDofMax][kNrhs + 1];
    const LeafIo L = S.leaves[l];
    const int m = L.m;
    const int n_off = (int)chunk_n_off(m), len = (int)chunk_len(m);
    // the chunk's padding rows (past the shear and past the normal dofs) are zero
    for (int idx = threadIdx.x; idx < len * kNrhs; idx += blockDim.x) {
        const int q = idx / kNrhs;
        if ((q >= 2 * m && q < n_off) || q >= n_off + m) xs[q][idx % kNrhs] = 0.0;
    }
    // lane i takes element i, wave w columns 4w .. 4w + 3 (256 threads, at
    // most 64 elements): one index load, then its twelve values in flight
    // together (columns past nrhs read column nrhs - 1 and store zeros)
    const int i = threadIdx.x & 63, c0 = 4 * (threadIdx.x >> 6);
    if (i < m) {
        const int64_t e = S.perm[L.begin + i];
        const bool act = !S.mask || S.mask[e];
        double v[4][3];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double* x = S.X + (int64_t)min(c0 + k, nrhs - 1) * S.ldx + 3 * e;
#pragma unroll
            for (int a = 0; a < 3; ++a) v[k][a] = x[a];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool on = act && c0 + k < nrhs;
            xs[2 * i][c0 + k] = on ? v[k][0] : 0.0;
            xs[2 * i + 1][c0 + k] = on ? v[k][1] : 0.0;
            xs[n_off + i][c0 + k] = on ? v[k][2] : 0.0;
        }
    }
    __syncthreads();
    const int64_t base = L.xoff * kNrhs;
    NT* xnear = static_cast<NT*>(B.xnear);
    for (int64_t o = threadIdx.x; o < (int64_t)len * kNrhs; o += blockDim.x) {
        int q, c;
        frag_dof<Mma<NT>::w>(o, q, c);
        xnear[base + o] = cvt<NT>(xs[q][c]);
    }
    if (B.xfhi != B.xnear) {
        FT* xfhi = static_cast<FT*>(B.xfhi);
        FT* xflo = static_cast<FT*>(B.xflo);
        for (int64_t o = threadIdx.x; o < (int64_t)len * kNrhs; o += blockDim.x) {
            int q, c;
            frag_dof<Mma<FT>::w>(o, q, c);
            store_t<FT>(xfhi, xflo, base + o, xs[q][c]);
        }
    }
}

// the product's first kernel also clears the claim counters of a
// queue-driven launch
__device__ inline void clear_queue(int* __restrict__ queue)
{
    if (queue && blockIdx.x == 0 && threadIdx.x < kQueueInts / kQueueStride) queue[threadIdx.x * kQueueStride] = 0;
}

template <class NT, class FT>
__global__ __launch_bounds__(256) void k_gather1(Segment S, const Bases* __restrict__ bases, int nrhs,
                                                 int* __restrict__ queue)
{
    clear_queue(queue);
    gather_leaf<NT, FT>(S, bases[S.op], nrhs, blockIdx.x);
}

template <class NT, class FT>
__global__ __launch_bounds__(256) void k_gatherN(const Segment* __restrict__ segs, int nseg,
                                                 const Bases* __restrict__ bases, int nrhs, int* __restrict__ queue)
{
    clear_queue(queue);
    const Segment S = segs[segment_of(segs, nseg, blockIdx.x)];
    gather_leaf<NT, FT>(S, bases[S.op], nrhs, blockIdx.x - S.leaf0);
}

template <class S_t>
__device__ inline void scatter_leaf(const Segment& S, const Bases& B, int nrhs, int l)
{
    __shared__ S_t ys[kLeafDofMax][kNrhs + 1];
    const LeafIo L = S.leaves[l];
    const int m = L.m;
    const int n_off = (int)chunk_n_off(m), len = (int)chunk_len(m);
    // lane i takes element i, wave w columns 4w .. 4w + 3 (as in the gather):
    // the element's index, self and tangent blocks are loaded once and the
    // vector values of its four columns go out together, before the leaf's
    // output rows are staged in LDS, so both are in flight at once
    const int i = threadIdx.x & 63, c0 = 4 * (threadIdx.x >> 6);
    const bool act = i < m && c0 < nrhs;
    int64_t e = 0;
    double x[4][3] = {}, prev[4][3] = {}, sf[9] = {}, dm[9] = {};
    bool passive = false, with_d = false;
    if (act) {
        e = S.perm[L.begin + i];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int c = min(c0 + k, nrhs - 1);
#pragma unroll
            for (int a = 0; a < 3; ++a) x[k][a] = S.X[c * S.ldx + 3 * e + a];
            if (S.accumulate)
#pragma unroll
                for (int a = 0; a < 3; ++a) prev[k][a] = S.Y[c * S.ldy + 3 * e + a];
        }
        if (S.self)
#pragma unroll
            for (int q = 0; q < 9; ++q) sf[q] = S.self[9 * e + q];
        passive = S.tangent && S.mask && !S.mask[e];
        with_d = S.tangent && !passive && S.D;
        if (with_d)
#pragma unroll
            for (int q = 0; q < 9; ++q) dm[q] = S.D[9 * e + q];
    }
    const S_t* Y = static_cast<const S_t*>(B.y) + L.xoff * kNrhs;
    for (int idx = threadIdx.x; idx < len * kNrhs; idx += blockDim.x) ys[idx / kNrhs][idx % kNrhs] = Y[idx];
    __syncthreads();
    if (!act) return;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = c0 + k;
        if (c >= nrhs) break;
        double y[3];
        for (int a = 0; a < 3; ++a) y[a] = (double)ys[a < 2 ? 2 * i + a : n_off + i][c];
        if (S.self)
            for (int a = 0; a < 3; ++a)
                y[a] += sf[3 * a] * x[k][0] + sf[3 * a + 1] * x[k][1] + sf[3 * a + 2] * x[k][2];
        if (passive) {
            for (int a = 0; a < 3; ++a) y[a] = x[k][a];
        } else if (with_d) {
            for (int a = 0; a < 3; ++a)
                y[a] -= dm[3 * a] * x[k][0] + dm[3 * a + 1] * x[k][1] + dm[3 * a + 2] * x[k][2];
        }
        double* out = S.Y + c * S.ldy + 3 * e;
        for (int a = 0; a < 3; ++a) out[a] = S.accumulate ? prev[k][a] + y[a] : y[a];
    }
}

template <class S_t>
__global__ __launch_bounds__(256) void k_scatter1(Segment S, const Bases* __restrict__ bases, int nrhs)
{
    scatter_leaf<S_t>(S, bases[S.op], nrhs, blockIdx.x);
}

template <class S_t>
__global__ __launch_bounds__(256) void k_scatterN(const Segment* __restrict__ segs, int nseg,
                                                  const Bases* __restrict__ bases, int nrhs)
{
    const Segment S = segs[segment_of(segs, nseg, blockIdx.x)];
    scatter_leaf<S_t>(S, bases[S.op], nrhs, blockIdx.x - S.leaf0);
}

// ------------------------------------------------------------------
// host driver
// ------------------------------------------------------------------
// ------------------------------------------------------------------
// workspaces
// ------------------------------------------------------------------
WsLayout Variant::ws_layout() const
{
    WsLayout w;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t off = at;
        at = (size_t)round_up((int64_t)(at + bytes), 256);
        return off;
    };
    const size_t tfrag = (size_t)std::max<int64_t>(1, tfrag_elems);
    w.xn = take((size_t)xel * prec_bytes(near_prec));
    w.xfh = far_is_near() ? w.xn : take((size_t)xel * prec_bytes(far_prec));
    w.xfl = far_prec == HM_BF16 ? take((size_t)xel * prec_bytes(far_prec)) : 0;
    w.tph = take(tfrag * prec_bytes(far_prec));
    w.tpl = far_prec == HM_BF16 ? take(tfrag * prec_bytes(far_prec)) : 0;
    w.zero_end = at;
    const int acc_bytes = acc_f64() ? 8 : 4;
    w.tpart = take((size_t)std::max<int64_t>(1, tpart_elems) * acc_bytes);
    w.y = take((size_t)xel * acc_bytes);
    w.bases = take(sizeof(Bases));
    w.total = at;
    return w;
}

Bases Variant::host_bases(void* block) const
{
    const WsLayout w = ws_layout();
    char* p = static_cast<char*>(block);
    Bases b;
    b.nearA = near_a.get();
    b.farA = far_a.get();
    b.xnear = p + w.xn;
    b.xfhi = p + w.xfh;
    b.xflo = far_prec == HM_BF16 ? p + w.xfl : nullptr;
    b.thi = p + w.tph;
    b.tlo = far_prec == HM_BF16 ? p + w.tpl : nullptr;
    b.tpart = p + w.tpart;
    b.y = p + w.y;
    return b;
}

__global__ void k_zero16(uint4* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void k_set_bases(Bases b, Bases* __restrict__ dst)
{
    if (threadIdx.x == 0) *dst = b;
}

void Variant::prepare_block(void* block, hipStream_t s) const
{
    const WsLayout w = ws_layout();
    const int64_t words = (int64_t)(w.zero_end / 16);
    if (words > 0) {
        const unsigned grid = (unsigned)std::min<int64_t>((words + 255) / 256, 4096);
        hipLaunchKernelGGL(k_zero16, dim3(grid), dim3(64 * 4), 0, s, static_cast<uint4*>(block), words);
    }
    hipLaunchKernelGGL(k_set_bases, dim3(1), dim3(64), 0, s, host_bases(block),
                       reinterpret_cast<Bases*>(static_cast<char*>(block) + w.bases));
    HM_CHECK_HIP(hipGetLastError());
}

std::unique_ptr<ApplyWs> Variant::new_workspace(hipStream_t s) const
{
    std::unique_ptr<ApplyWs> ws(new ApplyWs());
    ws->block.alloc(ws_layout().total);
    prepare_block(ws->block.get(), s);
    ws->gen = gen;
    return ws;
}

void* Variant::workspace(hipStream_t s) const
{
    std::lock_guard<std::mutex> g(ws_mu);
    std::unique_ptr<ApplyWs>& w = ws_pool[s];
    if (!w) {
        w = new_workspace(s);
    } else if (w->gen != gen) {
        // the task lists changed: the partial-slot section may have grown
        if (w->block.bytes() < ws_layout().total) {
            HM_CHECK_HIP(hipStreamSynchronize(s));
            w->block.alloc(ws_layout().total);
        }
        prepare_block(w->block.get(), s);
        w->gen = gen;
    }
    return w->block.get();
}

LaunchSet launch_set(const Variant& v, void* block)
{
    LaunchSet L;
    L.near_prec = v.near_prec;
    L.far_prec = v.far_prec;
    L.bases = reinterpret_cast<const Bases*>(static_cast<const char*>(block) + v.ws_layout().bases);
    L.tasksA = v.tasksA.as<TaskA>();
    L.nTasksA = v.nTasksA;
    L.splitA = v.splitA;
    L.splitB = v.splitB;
    L.itemsA = v.itemsA.as<PanelRef>();
    L.membersA = v.membersA.as<MemberT>();
    L.reduce = v.reduce.as<ReduceDesc>();
    L.nReduce = v.nReduce;
    L.tasksB = v.tasksB.as<TaskB>();
    L.nTasksB = v.nTasksB;
    L.itemsB = v.itemsB.as<PanelRef>();
    L.maxNtB = v.maxNtB;
    return L;
}

Segment make_segment(const Op& op, const Variant& v, const double* X, int64_t ldx, double* Y, int64_t ldy,
                     bool tangent, int op_index, bool accumulate)
{
    Segment g;
    g.accumulate = accumulate ? 1 : 0;
    g.pad = 0;
    g.ne = op.ne;
    g.ldx = ldx;
    g.ldy = ldy;
    g.X = X;
    g.Y = Y;
    g.perm = op.d_perm.as<int64_t>();
    g.leaves = op.d_leaf_io.as<LeafIo>();
    g.nleaf = (int32_t)op.plan.leaves.size();
    g.leaf0 = 0;
    g.self = v.self_separate ? op.d_self.as<double>() : nullptr;
    g.D = (tangent && op.has_D) ? op.d_D.as<double>() : nullptr;
    g.mask = (tangent && op.has_mask) ? op.d_mask.as<uint8_t>() : nullptr;
    g.op = op_index;
    g.tangent = tangent ? 1 : 0;
    return g;
}

template <class NT, class FT, class ACC>
static void launch_t(const LaunchSet& L, int nrhs, const Segment* segs_dev, const Segment* seg1, int nseg,
                     int64_t total_leaves, hipStream_t s, hipEvent_t* ev)
{
    typedef typename AccScalar<ACC>::type S;
    auto mark = [&](int i) {
        if (ev) HM_CHECK_HIP(hipEventRecord(ev[i], s));
    };
    static const unsigned gridA = queue_grid(reinterpret_cast<const void*>(&k_phaseA_q<FT, ACC>));
    static const unsigned gridB4 = queue_grid(reinterpret_cast<const void*>(&k_phaseB_q<NT, FT, ACC, 4>));
    static const unsigned gridB8 = queue_grid(reinterpret_cast<const void*>(&k_phaseB_q<NT, FT, ACC, 8>));
    mark(0);
    if (nseg == 1 && seg1)
        hipLaunchKernelGGL((k_gather1<NT, FT>), dim3((unsigned)total_leaves), dim3(256), 0, s, *seg1, L.bases, nrhs,
                           L.queue);
    else
        hipLaunchKernelGGL((k_gatherN<NT, FT>), dim3((unsigned)total_leaves), dim3(256), 0, s, segs_dev, nseg,
                           L.bases, nrhs, L.queue);
    mark(1);
    if (L.nTasksA > 0 && L.queue)
        hipLaunchKernelGGL((k_phaseA_q<FT, ACC>), dim3(std::min<unsigned>(gridA, 8u * ((L.nTasksA + 31) / 32))),
                           dim3(256), 0, s, L.tasksA, L.splitA, L.itemsA, L.membersA, L.bases, L.queue);
    else if (L.nTasksA > 0)
        hipLaunchKernelGGL((k_phaseA<FT, ACC>), dim3(xcd_grid(L.splitA, 4)), dim3(256), 0, s, L.tasksA, L.splitA,
                           L.itemsA, L.membersA, L.bases);
    mark(2);
    if (L.nReduce > 0)
        hipLaunchKernelGGL((k_reduceT<FT, S>), dim3(L.nReduce), dim3(256), 0, s, L.reduce, L.bases);
    mark(3);
    if (L.nTasksB > 0) {
        const bool w4 = L.maxNtB <= 4;
        const unsigned gq = std::min<unsigned>(w4 ? gridB4 : gridB8, 8u * ((L.nTasksB + 7) / 8));
        const unsigned gg = xcd_grid(L.splitB, 1);
        if (L.queue && w4)
            hipLaunchKernelGGL((k_phaseB_q<NT, FT, ACC, 4>), dim3(gq), dim3(256), 0, s, L.tasksB, L.splitB, L.itemsB,
                               L.bases, L.queue);
        else if (L.queue)
            hipLaunchKernelGGL((k_phaseB_q<NT, FT, ACC, 8>), dim3(gq), dim3(256), 0, s, L.tasksB, L.splitB, L.itemsB,
                               L.bases, L.queue);
        else if (w4)
            hipLaunchKernelGGL((k_phaseB<NT, FT, ACC, 4>), dim3(gg), dim3(256), 0, s, L.tasksB, L.splitB, L.itemsB,
                               L.bases);
        else
            hipLaunchKernelGGL((k_phaseB<NT, FT, ACC, 8>), dim3(gg), dim3(256), 0, s, L.tasksB, L.splitB, L.itemsB,
                               L.bases);
    }
    mark(4);
    if (nseg == 1 && seg1)
        hipLaunchKernelGGL((k_scatter1<S>), dim3((unsigned)total_leaves), dim3(256), 0, s, *seg1, L.bases, nrhs);
    else
        hipLaunchKernelGGL((k_scatterN<S>), dim3((unsigned)total_leaves), dim3(256), 0, s, segs_dev, nseg, L.bases,
                           nrhs);
    mark(5);
    HM_CHECK_HIP(hipGetLastError());
}

int phaseA_resident_waves(int near_prec, int far_prec)
{
    const void* k = near_prec == HM_F64   ? reinterpret_cast<const void*>(&k_phaseA<double, d4>)
                    : far_prec == HM_F32  ? reinterpret_cast<const void*>(&k_phaseA<float, f4>)
                    : far_prec == HM_BF16 ? reinterpret_cast<const void*>(&k_phaseA<uint16_t, f4>)
                                          : reinterpret_cast<const void*>(&k_phaseA<bf16s, f4>);
    int dev = 0, cus = 0, per_cu = 0;
    HM_CHECK_HIP(hipGetDevice(&dev));
    HM_CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HM_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, 0));
    return std::max(1, per_cu) * std::max(1, cus) * 4;
}

void launch_product(const LaunchSet& L, int nrhs, const Segment* segs_dev, const Segment* seg1, int nseg,
                    int64_t total_leaves, hipStream_t s, hipEvent_t* ev)
{
    HM_REQUIRE(nrhs >= 1 && nrhs <= kNrhs, HM_EINVAL, "nrhs must be in [1, 16]");
    if (L.near_prec == HM_F64)
        launch_t<double, double, d4>(L, nrhs, segs_dev, seg1, nseg, total_leaves, s, ev);
    else if (L.far_prec == HM_F32)
        launch_t<float, float, f4>(L, nrhs, segs_dev, seg1, nseg, total_leaves, s, ev);
    else if (L.far_prec == HM_BF16)
        launch_t<float, uint16_t, f4>(L, nrhs, segs_dev, seg1, nseg, total_leaves, s, ev);
    else
        launch_t<float, bf16s, f4>(L, nrhs, segs_dev, seg1, nseg, total_leaves, s, ev);
}

void apply(const Op& op, const Variant& v, int nrhs, const double* X, int64_t ldx, double* Y, int64_t ldy,
           bool tangent, hipStream_t s, hipEvent_t* ev, bool accumulate)
{
    HM_REQUIRE(nrhs >= 1 && nrhs <= kNrhs, HM_EINVAL, "nrhs must be in [1, 16]");
    HM_REQUIRE(ldx >= 3 * op.ne && ldy >= 3 * op.ne, HM_EINVAL, "leading dimension below 3N");
    HM_REQUIRE(X && Y, HM_EINVAL, "null vector pointer");
    const Segment g = make_segment(op, v, X, ldx, Y, ldy, tangent, 0, accumulate);
    launch_product(launch_set(v, v.workspace(s)), nrhs, nullptr, &g, 1, g.nleaf, s, ev);
}

void apply_in(const Op& op, const Variant& v, void* block, int nrhs, const double* X, int64_t ldx, double* Y,
              int64_t ldy, bool tangent, hipStream_t s, bool accumulate)
{
    HM_REQUIRE(nrhs >= 1 && nrhs <= kNrhs, HM_EINVAL, "nrhs must be in [1, 16]");
    HM_REQUIRE(ldx >= 3 * op.ne && ldy >= 3 * op.ne, HM_EINVAL, "leading dimension below 3N");
    HM_REQUIRE(X && Y && block, HM_EINVAL, "null pointer");
    HM_REQUIRE(((uintptr_t)block & 255) == 0, HM_EINVAL, "workspace block not 256-byte aligned");
    v.prepare_block(block, s);
    const Segment g = make_segment(op, v, X, ldx, Y, ldy, tangent, 0, accumulate);
    launch_product(launch_set(v, block), nrhs, nullptr, &g, 1, g.nleaf, s, nullptr);
}

// ------------------------------------------------------------------
// tangent terms and block-Jacobi preconditioner
// ------------------------------------------------------------------
// pc_block[e] = (E_ee - D_e)^-1 (3x3, FP64) on active elements, identity on
// inactive ones; pc_diag[3e + a] = 1 / (E_ee - D_e)_aa (point Jacobi).
__global__ void k_precond_setup(int64_t ne, const double* __restrict__ self, const double* __restrict__ Dt,
                                const uint8_t* __restrict__ mask, double* __restrict__ pcb, double* __restrict__ pcd)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    double A[9];
    for (int k = 0; k < 9; ++k) A[k] = self[9 * e + k] - (Dt ? Dt[9 * e + k] : 0.0);
    if (mask && !mask[e]) {
        for (int k = 0; k < 9; ++k) A[k] = (k % 4 == 0) ? 1.0 : 0.0;
    }
    double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8], c02 = A[3] * A[7] - A[4] * A[6];
    double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    double inv = 1.0 / det;
    double B[9] = {c00 * inv,
                   (A[2] * A[7] - A[1] * A[8]) * inv,
                   (A[1] * A[5] - A[2] * A[4]) * inv,
                   c01 * inv,
                   (A[0] * A[8] - A[2] * A[6]) * inv,
                   (A[2] * A[3] - A[0] * A[5]) * inv,
                   c02 * inv,
                   (A[1] * A[6] - A[0] * A[7]) * inv,
                   (A[0] * A[4] - A[1] * A[3]) * inv};
    for (int k = 0; k < 9; ++k) pcb[9 * e + k] = B[k];
    for (int a = 0; a < 3; ++a) pcd[3 * e + a] = 1.0 / A[4 * a];
}

void tangent_set(Op& op, const double* d_D, const uint8_t* d_mask, hipStream_t s)
{
    const int64_t ne = op.ne;
    if (d_D) {
        op.d_D.alloc(9 * ne * sizeof(double));
        HM_CHECK_HIP(hipMemcpyAsync(op.d_D.get(), d_D, 9 * ne * sizeof(double), hipMemcpyDeviceToDevice, s));
        op.has_D = true;
    } else {
        op.d_D.release();
        op.has_D = false;
    }
    if (d_mask) {
        op.d_mask.alloc(ne);
        HM_CHECK_HIP(hipMemcpyAsync(op.d_mask.get(), d_mask, ne, hipMemcpyDeviceToDevice, s));
        op.has_mask = true;
    } else {
        op.d_mask.release();
        op.has_mask = false;
    }
    // the learned correction was predicted for the previous tangent
    op.lp.features_current = false;
    op.lp.attached = false;
    op.leaf_pc_current = false;
    op.ilu.current = false;
    if (!op.d_pc_block.get()) op.d_pc_block.alloc(9 * ne * sizeof(double));
    if (!op.d_pc_diag.get()) op.d_pc_diag.alloc(3 * ne * sizeof(double));
    hipLaunchKernelGGL(k_precond_setup, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, ne,
                       op.d_self.as<double>(), op.has_D ? op.d_D.as<double>() : nullptr,
                       op.has_mask ? op.d_mask.as<uint8_t>() : nullptr, op.d_pc_block.as<double>(),
                       op.d_pc_diag.as<double>());
    HM_CHECK_HIP(hipGetLastError());
    HM_CHECK_HIP(hipStreamSynchronize(s));
}

}  // namespace hm
