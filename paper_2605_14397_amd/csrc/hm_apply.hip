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
#include "hm_op.hpp"
#include "hm_util.hpp"

namespace hm {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// ---- per storage type: 16-byte granule and MFMA step ----
template <class T>
struct Mma;

template <>
struct Mma<double> {
    static constexpr int w = 2;
    typedef d2 vec;
    // two 16x16x4 FP64 products: k = 2g + t
    template <class A>
    __device__ static A run(vec a, vec b, vec, A c)
    {
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], c, 0, 0, 0);
        return c;
    }
};

template <>
struct Mma<float> {
    static constexpr int w = 4;
    typedef f4 vec;
    // four 16x16x4 FP32 products: k = 4g + t
    template <class A>
    __device__ static A run(vec a, vec b, vec, A c)
    {
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
    typedef bf8 vec;
    // one 16x16x32 BF16 product per half of the split in-vector (hi + lo)
    template <class A>
    __device__ static A run(vec a, vec bhi, vec blo, A c)
    {
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bhi, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, blo, c, 0, 0, 0);
        return c;
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

template <class V, class T>
__device__ inline V load16(const T* p)
{
    return *reinterpret_cast<const V*>(p);
}

template <class V>
__device__ inline V zero16()
{
    V z;
    __builtin_memset(&z, 0, sizeof(V));
    return z;
}

// Workgroups are dealt to the 8 XCDs round-robin; give each XCD a
// contiguous range of tasks so neighbouring leaves share one L2.
__device__ inline int xcd_task(int bid, int grid, int ntasks)
{
    int per = grid >> 3;
    int t = (bid & 7) * per + (bid >> 3);
    return t < ntasks ? t : -1;
}

// Stream one panel's k-steps owned by this wave into the accumulators.
template <class ST, class ACC>
__device__ __attribute__((always_inline)) inline void run_panel(const PanelRef& P, const ST* __restrict__ A, const ST* __restrict__ Bhi,
                                 const ST* __restrict__ Blo, int R, int wave, int lane, int& unit,
                                 ACC (&acc)[kRowTilesMax])
{
    typedef typename Mma<ST>::vec vec;
    constexpr int w = Mma<ST>::w;
    constexpr int kstep = 4 * w;
    const int nks = (P.cols + kstep - 1) / kstep;
    const int Gr = (P.cols + w - 1) / w;
    const int g = lane >> 4, i = lane & 15;
    int ks = (wave - unit) & 3;
    const ST* Ap = A + P.a_off;
    for (; ks < nks; ks += 4) {
        const int gg = min(4, Gr - 4 * ks);
        const int64_t boff = P.b_off + ((int64_t)ks * 64 + lane) * w;
        vec bhi = load16<vec>(Bhi + boff);
        vec blo = Blo ? load16<vec>(Blo + boff) : zero16<vec>();
        vec a[kRowTilesMax];
#pragma unroll
        for (int r = 0; r < kRowTilesMax; ++r) {
            if (r < R) {
                const int rr = min(16, P.rows - 16 * r);
                const bool ok = (i < rr) && (g < gg);
                const int64_t off = (int64_t)r * 16 * Gr * w + (int64_t)ks * rr * 4 * w + (int64_t)(g * rr + i) * w;
                a[r] = ok ? load16<vec>(Ap + off) : zero16<vec>();
            }
        }
#pragma unroll
        for (int r = 0; r < kRowTilesMax; ++r)
            if (r < R) acc[r] = Mma<ST>::run(a[r], bhi, blo, acc[r]);
    }
    unit += nks;
}

// Sum the four waves' accumulators in a fixed order; wave 0 writes rows < rows.
template <class ACC, class S>
__device__ __attribute__((always_inline)) inline void reduce_and_store(ACC (&acc)[kRowTilesMax], int R, int rows, S* __restrict__ out,
                                        int64_t row0, S* red, int wave, int lane)
{
#pragma unroll
    for (int r = 0; r < kRowTilesMax; ++r) {
        if (r >= R) break;
        if (wave > 0)
            for (int v = 0; v < 4; ++v) red[(wave - 1) * 256 + lane * 4 + v] = acc[r][v];
        __syncthreads();
        if (wave == 0) {
            for (int v = 0; v < 4; ++v) {
                S s = acc[r][v] + red[lane * 4 + v];
                s += red[256 + lane * 4 + v];
                s += red[512 + lane * 4 + v];
                int row = 16 * r + AccScalar<ACC>::row(lane, v);
                if (row < rows) out[(row0 + row) * kNrhs + (lane & 15)] = s;
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------
// phase A: T partial = sum over this task's V^T sub-panels of V^T X
// ------------------------------------------------------------------
template <class FT, class ACC>
__global__ __launch_bounds__(256) void k_phaseA(const TaskA* __restrict__ tasks, int ntasks,
                                                const PanelRef* __restrict__ items, const FT* __restrict__ farA,
                                                const FT* __restrict__ xhi, const FT* __restrict__ xlo,
                                                typename AccScalar<ACC>::type* __restrict__ tpart)
{
    typedef typename AccScalar<ACC>::type S;
    __shared__ S red[3 * 256];
    const int bid = blockIdx.x;
    if (bid >= ntasks) return;
    const TaskA T = tasks[bid];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    ACC acc[kRowTilesMax];
#pragma unroll
    for (int r = 0; r < kRowTilesMax; ++r) acc[r] = ACC{0, 0, 0, 0};
    const int R = (T.rows + 15) >> 4;
    int unit = 0;
    for (int it = 0; it < T.n_items; ++it) {
        const PanelRef P = items[T.item_begin + it];
        run_panel<FT, ACC>(P, farA, xhi, xlo, R, wave, lane, unit, acc);
    }
    reduce_and_store<ACC, S>(acc, R, 16 * R, tpart + T.out_off, 0, red, wave, lane);
}

// ------------------------------------------------------------------
// reduce phase-A partials into T fragment chunks (far precision)
// ------------------------------------------------------------------
template <class FT, class S>
__global__ void k_reduceT(const ReduceDesc* __restrict__ rd, const S* __restrict__ tpart, FT* __restrict__ thi,
                          FT* __restrict__ tlo)
{
    const ReduceDesc D = rd[blockIdx.x];
    const int Kp = (int)round_up(D.rank, kChunkAlign);
    const int64_t slot = (int64_t)((D.rank + 15) / 16) * 16 * kNrhs;
    constexpr int w = Mma<FT>::w;
    for (int e = threadIdx.x; e < Kp * kNrhs; e += blockDim.x) {
        const int row = e / kNrhs, c = e - row * kNrhs;
        S v = 0;
        if (row < D.rank)
            for (int s = 0; s < D.n_slots; ++s) v += tpart[D.slot_begin + s * slot + (int64_t)row * kNrhs + c];
        const int64_t off = D.t_off + bfrag_offset(w, row, c);
        if constexpr (sizeof(FT) == 2) {
            float f = (float)v;
            uint16_t h = f32_to_bf16_bits(f);
            thi[off] = h;
            tlo[off] = f32_to_bf16_bits(f - bf16_bits_to_f32(h));
        } else {
            thi[off] = (FT)v;
        }
    }
}

// ------------------------------------------------------------------
// phase B: one workgroup per target leaf
// ------------------------------------------------------------------
template <class NT, class FT, class ACC>
__global__ __launch_bounds__(256) void k_phaseB(const TaskB* __restrict__ tasks, int ntasks,
                                                const PanelRef* __restrict__ items, const NT* __restrict__ nearA,
                                                const FT* __restrict__ farA, const NT* __restrict__ xnear,
                                                const FT* __restrict__ thi, const FT* __restrict__ tlo,
                                                typename AccScalar<ACC>::type* __restrict__ Y)
{
    typedef typename AccScalar<ACC>::type S;
    __shared__ S red[3 * 256];
    const int t = xcd_task(blockIdx.x, gridDim.x, ntasks);
    if (t < 0) return;
    const TaskB T = tasks[t];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    ACC acc[kRowTilesMax];
#pragma unroll
    for (int r = 0; r < kRowTilesMax; ++r) acc[r] = ACC{0, 0, 0, 0};
    const int R = (T.rows + 15) >> 4;
    int unit = 0;
    for (int it = 0; it < T.n_items; ++it) {
        const PanelRef P = items[T.item_begin + it];
        if (P.far)
            run_panel<FT, ACC>(P, farA, thi, tlo, R, wave, lane, unit, acc);
        else
            run_panel<NT, ACC>(P, nearA, xnear, nullptr, R, wave, lane, unit, acc);
    }
    reduce_and_store<ACC, S>(acc, R, T.rows, Y, T.y_off, red, wave, lane);
}

// ------------------------------------------------------------------
// gather / scatter
// ------------------------------------------------------------------
template <class NT, class FT>
__global__ void k_gather(int64_t ne, int nrhs, const double* __restrict__ X, int64_t ldx,
                         const uint8_t* __restrict__ mask, const int64_t* __restrict__ xslot,
                         const int32_t* __restrict__ xloc, NT* __restrict__ xnear, FT* __restrict__ xfhi,
                         FT* __restrict__ xflo)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ne * kNrhs) return;
    const int c = (int)(idx / ne);
    const int64_t e = idx - (int64_t)c * ne;
    const bool on = c < nrhs && (!mask || mask[e]);
    const int64_t base = xslot[e] * kNrhs;
    const int q0 = xloc[e];
    for (int a = 0; a < 3; ++a) {
        const double x = on ? X[c * ldx + 3 * e + a] : 0.0;
        xnear[base + bfrag_offset(Mma<NT>::w, q0 + a, c)] = cvt<NT>(x);
        if (xfhi) {
            const int64_t off = base + bfrag_offset(Mma<FT>::w, q0 + a, c);
            if constexpr (sizeof(FT) == 2) {
                float f = (float)x;
                uint16_t h = f32_to_bf16_bits(f);
                xfhi[off] = h;
                xflo[off] = f32_to_bf16_bits(f - bf16_bits_to_f32(h));
            } else {
                xfhi[off] = cvt<FT>(x);
            }
        }
    }
}

template <class S>
__global__ void k_scatter(int64_t ne, int nrhs, const S* __restrict__ Y, const int64_t* __restrict__ xslot,
                          const int32_t* __restrict__ xloc, const double* __restrict__ X, int64_t ldx,
                          double* __restrict__ Yout, int64_t ldy, const double* __restrict__ self,
                          const double* __restrict__ Dt, const uint8_t* __restrict__ mask, int tangent)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ne * nrhs) return;
    const int c = (int)(idx / ne);
    const int64_t e = idx - (int64_t)c * ne;
    const int64_t row = xslot[e] + xloc[e];
    double y[3], x[3];
    for (int a = 0; a < 3; ++a) {
        y[a] = (double)Y[(row + a) * kNrhs + c];
        x[a] = X[c * ldx + 3 * e + a];
    }
    if (self)
        for (int a = 0; a < 3; ++a)
            y[a] += self[9 * e + 3 * a] * x[0] + self[9 * e + 3 * a + 1] * x[1] + self[9 * e + 3 * a + 2] * x[2];
    if (tangent) {
        if (mask && !mask[e]) {
            for (int a = 0; a < 3; ++a) y[a] = x[a];
        } else if (Dt) {
            for (int a = 0; a < 3; ++a)
                y[a] -= Dt[9 * e + 3 * a] * x[0] + Dt[9 * e + 3 * a + 1] * x[1] + Dt[9 * e + 3 * a + 2] * x[2];
        }
    }
    for (int a = 0; a < 3; ++a) Yout[c * ldy + 3 * e + a] = y[a];
}

// ------------------------------------------------------------------
// host driver
// ------------------------------------------------------------------
template <class NT, class FT, class ACC>
static void apply_t(const Op& op, const Variant& v, int nrhs, const double* X, int64_t ldx, double* Y, int64_t ldy,
                    bool tangent, hipStream_t s)
{
    typedef typename AccScalar<ACC>::type S;
    const int64_t ne = op.ne;
    const uint8_t* mask = (tangent && op.has_mask) ? op.d_mask.as<uint8_t>() : nullptr;
    const bool sep = !v.far_is_near();
    FT* xfhi = sep ? v.xf_far_hi.as<FT>() : nullptr;
    FT* xflo = (sep && v.far_prec == HM_BF16) ? v.xf_far_lo.as<FT>() : nullptr;
    {
        int64_t n = ne * kNrhs;
        hipLaunchKernelGGL((k_gather<NT, FT>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ne, nrhs, X, ldx,
                           mask, op.d_xslot.as<int64_t>(), op.d_xloc.as<int32_t>(), v.xf_near.as<NT>(), xfhi, xflo);
    }
    const FT* xa_hi = sep ? xfhi : reinterpret_cast<const FT*>(v.xf_near.get());
    const FT* xa_lo = xflo;
    if (v.nTasksA > 0) {
        hipLaunchKernelGGL((k_phaseA<FT, ACC>), dim3(v.nTasksA), dim3(256), 0, s, v.tasksA.as<TaskA>(), v.nTasksA,
                           v.itemsA.as<PanelRef>(), v.far_a.as<FT>(), xa_hi, xa_lo, v.tpart.as<S>());
        hipLaunchKernelGGL((k_reduceT<FT, S>), dim3(v.nReduce), dim3(256), 0, s, v.reduce.as<ReduceDesc>(),
                           v.tpart.as<S>(), v.tf_hi.as<FT>(), v.far_prec == HM_BF16 ? v.tf_lo.as<FT>() : nullptr);
    }
    {
        int grid = (int)round_up(v.nTasksB, 8);
        hipLaunchKernelGGL((k_phaseB<NT, FT, ACC>), dim3(grid), dim3(256), 0, s, v.tasksB.as<TaskB>(), v.nTasksB,
                           v.itemsB.as<PanelRef>(), v.near_a.as<NT>(), v.far_a.as<FT>(), v.xf_near.as<NT>(),
                           v.tf_hi.as<FT>(), v.far_prec == HM_BF16 ? v.tf_lo.as<FT>() : nullptr, v.y.as<S>());
    }
    {
        int64_t n = ne * nrhs;
        const double* Dt = (tangent && op.has_D) ? op.d_D.as<double>() : nullptr;
        hipLaunchKernelGGL((k_scatter<S>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ne, nrhs, v.y.as<S>(),
                           op.d_xslot.as<int64_t>(), op.d_xloc.as<int32_t>(), X, ldx, Y, ldy,
                           v.self_separate ? op.d_self.as<double>() : nullptr, Dt, mask, tangent ? 1 : 0);
    }
    HM_CHECK_HIP(hipGetLastError());
}

void apply(const Op& op, const Variant& v, int nrhs, const double* X, int64_t ldx, double* Y, int64_t ldy,
           bool tangent, hipStream_t s)
{
    HM_REQUIRE(nrhs >= 1 && nrhs <= kNrhs, HM_EINVAL, "nrhs must be in [1, 16]");
    HM_REQUIRE(ldx >= 3 * op.ne && ldy >= 3 * op.ne, HM_EINVAL, "leading dimension below 3N");
    HM_REQUIRE(X && Y, HM_EINVAL, "null vector pointer");
    if (v.near_prec == HM_F64)
        apply_t<double, double, d4>(op, v, nrhs, X, ldx, Y, ldy, tangent, s);
    else if (v.far_prec == HM_F32)
        apply_t<float, float, f4>(op, v, nrhs, X, ldx, Y, ldy, tangent, s);
    else
        apply_t<float, uint16_t, f4>(op, v, nrhs, X, ldx, Y, ldy, tangent, s);
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
