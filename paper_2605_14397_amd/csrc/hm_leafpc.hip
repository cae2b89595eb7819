// Leaf block-Jacobi preconditioner of the tangent system (paper Sec. 3.3.1:
// the A11 systems are solved iteratively with a cheap preconditioner built
// from A11 itself; here M is the block diagonal of A11 over the cluster-tree
// leaves, each block inverted exactly in FP64).
//
// For leaf l with elements e_1 .. e_m (cluster order) the block is the
// 3m x 3m restriction of A11 = E - D: E from the collocation coefficients,
// D subtracted on the 3x3 diagonal blocks of active elements, identity rows
// and columns for inactive elements (as in the product).  The inverse is
// formed once per tangent state and stored column-major; applying M^-1 to
// 16 right-hand sides streams it once.
#include "hm_op.hpp"

namespace hm {

namespace {

constexpr int kGjSide = 32;                       // 32 x 32 threads per leaf block
constexpr int kGjSlots = kLeafDofMax / kGjSide;   // entries per thread along each axis
constexpr double kSingular = 1e-13;               // relative pivot threshold

static_assert(kLeafDofMax % kGjSide == 0, "leaf dofs must tile the thread grid");

}  // namespace

// One workgroup of 1024 threads per leaf.  Thread t = 32 tj + ti holds the
// entries (ti + 32 r, tj + 32 c) of the block in registers.  Gauss-Jordan
// elimination in place, column by column, with partial pivoting and no row
// interchanges: the pivot of column k is the largest |a(i, k)| over rows not
// yet used as pivots, p_k.  Each step sets row p to r_j = a(p, j) / piv
// (1 / piv at j = k) and, with column k first zeroed, subtracts a(i, k) r_j
// from every other row (so column k becomes -a(i, k) / piv); row p is
// written, never formed as a difference.  At the end A^-1 (s(q), p_l) =
// X (q, l), where s(q) is the step at which row q was the pivot.  The step
// loop is unrolled over the register slot of column k, so every register
// access has a constant index; row p_k is published through LDS by its
// owners.  Input: E rows of the block, row-major; output: A^-1, column-major,
// same place.  A pivot below 1e-13 of the block's largest term |E_ij| +
// |D_ij| (a numerically singular block) sets *status.
__global__ __launch_bounds__(1024) void k_leaf_invert(const LeafPc* __restrict__ desc,
                                                      const int64_t* __restrict__ perm,
                                                      const double* __restrict__ D,
                                                      const uint8_t* __restrict__ mask, double* __restrict__ blocks,
                                                      int* __restrict__ status)
{
    const LeafPc L = desc[blockIdx.x];
    const int n = 3 * L.m;
    const int ti = threadIdx.x & (kGjSide - 1), tj = threadIdx.x / kGjSide;
    double* A = blocks + L.off;
    __shared__ double rowp[kLeafDofMax], colk[kLeafDofMax];
    __shared__ int pk[kLeafDofMax], stepof[kLeafDofMax];
    __shared__ uint8_t used[kLeafDofMax];
    __shared__ int64_t eid[kLeafDofMax / 3];
    __shared__ uint8_t act[kLeafDofMax / 3];
    __shared__ int s_piv;
    __shared__ double s_amax[kGjSide];
    if (threadIdx.x < L.m) {
        const int64_t e = perm[L.begin + threadIdx.x];
        eid[threadIdx.x] = e;
        act[threadIdx.x] = mask ? mask[e] : 1;
    }
    if (threadIdx.x < kLeafDofMax) {
        used[threadIdx.x] = 0;
        pk[threadIdx.x] = threadIdx.x;      // in-range defaults (replaced step by step)
        stepof[threadIdx.x] = threadIdx.x;
    }
    __syncthreads();

    double a[kGjSlots][kGjSlots];
    double scale = 0.0;  // largest |E_ij| + |D_ij|: the size of the terms, not of their difference
#pragma unroll
    for (int r = 0; r < kGjSlots; ++r)
#pragma unroll
        for (int c = 0; c < kGjSlots; ++c) {
            const int i = ti + kGjSide * r, j = tj + kGjSide * c;
            double v = i == j ? 1.0 : 0.0;
            if (i < n && j < n) {
                const int ei = i / 3, ej = j / 3;
                if (act[ei] && act[ej]) {
                    v = A[(int64_t)i * n + j];
                    double t = fabs(v);
                    if (ei == ej && D) {
                        const double d = D[eid[ei] * 9 + (i % 3) * 3 + (j % 3)];
                        v -= d;
                        t += fabs(d);
                    }
                    scale = fmax(scale, t);
                } else {
                    scale = fmax(scale, fabs(v));
                }
            }
            a[r][c] = v;
        }
    // pivots below kSingular of the largest term count as zero
    {
        double m = scale;
        for (int off = kGjSide / 2; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
        if (ti == 0) s_amax[tj] = m;
        __syncthreads();
        if (threadIdx.x < kGjSide) {
            double v = s_amax[threadIdx.x];
            for (int off = kGjSide / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
            if (threadIdx.x == 0) s_amax[0] = v;
        }
        __syncthreads();
    }
    const double tiny = kSingular * s_amax[0];

#pragma unroll
    for (int kr = 0; kr < kGjSlots; ++kr)
        for (int kt = 0; kt < kGjSide; ++kt) {
            const int k = kGjSide * kr + kt;
            if (k >= n) break;
            // pivot among unused rows, held by the 32 threads of column group kt
            if (tj == kt) {
                double best = -1.0;
                int bi = n;
#pragma unroll
                for (int r = 0; r < kGjSlots; ++r) {
                    const int i = ti + kGjSide * r;
                    const double v = fabs(a[r][kr]);
                    if (i < n && !used[i] && v > best) {
                        best = v;
                        bi = i;
                    }
                }
                for (int off = kGjSide / 2; off > 0; off >>= 1) {
                    const double ob = __shfl_xor(best, off);
                    const int oi = __shfl_xor(bi, off);
                    if (ob > best || (ob == best && oi < bi)) {
                        best = ob;
                        bi = oi;
                    }
                }
                if (ti == 0) {
                    if (!(best > tiny) || bi >= n) {
                        *status = 1;
                        bi = k;  // keep the indices in range; the result is discarded
                    }
                    s_piv = bi;
                    used[bi] = 1;
                    pk[k] = bi;
                    stepof[bi] = k;
                }
            }
            __syncthreads();
            const int p = s_piv;
            const int pr = p / kGjSide, pt = p % kGjSide;
            // publish row p and column k
            if (ti == pt) {
#pragma unroll
                for (int q = 0; q < kGjSlots; ++q)
                    if (q == pr)
#pragma unroll
                        for (int c = 0; c < kGjSlots; ++c) rowp[tj + kGjSide * c] = a[q][c];
            }
            if (tj == kt)
#pragma unroll
                for (int r = 0; r < kGjSlots; ++r) colk[ti + kGjSide * r] = a[r][kr];
            __syncthreads();
            if (tj == kt)
#pragma unroll
                for (int r = 0; r < kGjSlots; ++r) a[r][kr] = 0.0;
            const double piv = rowp[k], inv = 1.0 / piv;
            double rr[kGjSlots];
#pragma unroll
            for (int c = 0; c < kGjSlots; ++c) {
                const int j = tj + kGjSide * c;
                rr[c] = j == k ? inv : rowp[j] * inv;
            }
#pragma unroll
            for (int r = 0; r < kGjSlots; ++r) {
                const int i = ti + kGjSide * r;
                const bool isp = i == p;
                const double cr = isp ? 0.0 : colk[i];
#pragma unroll
                for (int c = 0; c < kGjSlots; ++c) a[r][c] = isp ? rr[c] : a[r][c] - cr * rr[c];
            }
            __syncthreads();
        }
    // A^-1 (s(q), p_l) = X (q, l), stored column-major
#pragma unroll
    for (int r = 0; r < kGjSlots; ++r)
#pragma unroll
        for (int c = 0; c < kGjSlots; ++c) {
            const int q = ti + kGjSide * r, l = tj + kGjSide * c;
            if (q < n && l < n) A[(int64_t)pk[l] * n + stepof[q]] = a[r][c];
        }
}

// z = M^-1 r: one workgroup per leaf; the leaf's rows of r (all columns)
// are staged in LDS, thread i forms row i of the block times them (the
// column-major inverse is read coalesced, once).
__global__ __launch_bounds__(256) void k_leaf_apply(const LeafPc* __restrict__ desc, const int64_t* __restrict__ perm,
                                                    const double* __restrict__ inv, int nrhs,
                                                    const double* __restrict__ r, int64_t ldr, double* __restrict__ z,
                                                    int64_t ldz)
{
    const LeafPc L = desc[blockIdx.x];
    const int n = 3 * L.m;
    __shared__ double rl[kLeafDofMax * kNrhs];
    __shared__ int64_t eid[kLeafDofMax / 3];
    if (threadIdx.x < L.m) eid[threadIdx.x] = perm[L.begin + threadIdx.x];
    __syncthreads();
    for (int e = threadIdx.x; e < n * kNrhs; e += blockDim.x) {
        const int c = e / n, j = e - c * n;
        rl[j * kNrhs + c] = c < nrhs ? r[c * ldr + 3 * eid[j / 3] + j % 3] : 0.0;
    }
    __syncthreads();
    const double* Ai = inv + L.off;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double acc[kNrhs];
#pragma unroll
        for (int c = 0; c < kNrhs; ++c) acc[c] = 0.0;
#pragma unroll 4
        for (int j = 0; j < n; ++j) {
            const double aij = __builtin_nontemporal_load(&Ai[(int64_t)j * n + i]);  // streamed once
#pragma unroll
            for (int c = 0; c < kNrhs; ++c) acc[c] += aij * rl[j * kNrhs + c];
        }
        const int64_t dof = 3 * eid[i / 3] + i % 3;
        for (int c = 0; c < nrhs; ++c) z[c * ldz + dof] = acc[c];
    }
}

void leaf_pc_prepare(Op& op, hipStream_t s)
{
    // concurrent solves on several streams: the first forms the inverses
    // (and waits for them), the others find them current
    std::lock_guard<std::mutex> g(op.pc_mu);
    if (op.leaf_pc_current) return;
    const int nleaf = (int)op.plan.leaves.size();
    if (!op.d_leaf_inv.get()) op.d_leaf_inv.alloc((size_t)std::max<int64_t>(1, op.leaf_inv_elems) * sizeof(double));
    leaf_blocks_coef(op, op.d_leaf_inv.as<double>(), s);
    DevBuf status(sizeof(int));
    HM_CHECK_HIP(hipMemsetAsync(status.get(), 0, sizeof(int), s));
    hipLaunchKernelGGL(k_leaf_invert, dim3((unsigned)nleaf), dim3(kGjSide * kGjSide), 0, s,
                       op.d_leaf_desc.as<LeafPc>(), op.d_perm.as<int64_t>(),
                       op.has_D ? op.d_D.as<double>() : nullptr, op.has_mask ? op.d_mask.as<uint8_t>() : nullptr,
                       op.d_leaf_inv.as<double>(), status.as<int>());
    HM_CHECK_HIP(hipGetLastError());
    int h = 0;
    HM_CHECK_HIP(hipMemcpyAsync(&h, status.get(), sizeof(int), hipMemcpyDeviceToHost, s));
    HM_CHECK_HIP(hipStreamSynchronize(s));
    HM_REQUIRE(h == 0, HM_EINVAL, "a diagonal leaf block of the tangent operator is singular; use HM_PC_BLOCK3");
    op.leaf_pc_current = true;
}

void leaf_pc_apply(const Op& op, int nrhs, const double* r, int64_t ldr, double* z, int64_t ldz, hipStream_t s)
{
    HM_REQUIRE(op.leaf_pc_current, HM_EINTERNAL, "leaf preconditioner not prepared");
    hipLaunchKernelGGL(k_leaf_apply, dim3((unsigned)op.plan.leaves.size()), dim3(256), 0, s,
                       op.d_leaf_desc.as<LeafPc>(), op.d_perm.as<int64_t>(), op.d_leaf_inv.as<double>(), nrhs, r, ldr,
                       z, ldz);
    HM_CHECK_HIP(hipGetLastError());
}

}  // namespace hm
