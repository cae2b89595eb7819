// Operator build: influence coefficients of dense leaves, adaptive cross
// approximation (ACA) of admissible blocks, packing into the apply layout.
//
// Paper Sec. 3.1: E is stored as a hierarchical matrix whose far-field
// blocks are low-rank and near-field blocks full.  Everything that touches
// coefficients runs in FP64 on the GPU; low precisions appear only when the
// finished factors are packed.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>

#include "hm_op.hpp"
#include "hm_util.hpp"

namespace hm {

// ------------------------------------------------------------------
// coefficient kernels
// ------------------------------------------------------------------
__global__ void k_kernel_block(const ElemGeo* __restrict__ geo, const int64_t* __restrict__ rows,
                               const int64_t* __restrict__ cols, int64_t nr, int64_t nc, double kG, double kN,
                               double* __restrict__ out)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nr * nc) return;
    int64_t r = p / nc, c = p - r * nc;
    const ElemGeo& R = geo[rows[r]];
    double x[3] = {R.c[0], R.c[1], R.c[2]};
    double fr[9];
    for (int k = 0; k < 9; ++k) fr[k] = R.fr[k];
    double blk[9];
    dd_block(x, fr, geo[cols[c]], kG, kN, blk);
    for (int k = 0; k < 9; ++k) out[p * 9 + k] = blk[k];
}

struct DenseDesc {
    int64_t t_begin, s_begin;  // cluster positions
    int64_t out_off;           // FP64 row-major [3m][3n]
    int32_t m, n;
};

// one thread per element pair of one dense leaf block (blockIdx.y)
__global__ void k_dense_coef(const ElemGeo* __restrict__ geo, const DenseDesc* __restrict__ descs, double kG,
                             double kN, double* __restrict__ out)
{
    const DenseDesc D = descs[blockIdx.y];
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= D.m * D.n) return;
    int i = p / D.n, j = p - i * D.n;
    const ElemGeo& R = geo[D.t_begin + i];
    double x[3] = {R.c[0], R.c[1], R.c[2]};
    double fr[9];
    for (int k = 0; k < 9; ++k) fr[k] = R.fr[k];
    double blk[9];
    dd_block(x, fr, geo[D.s_begin + j], kG, kN, blk);
    int64_t ld = 3 * (int64_t)D.n;
    double* o = out + D.out_off + (3 * (int64_t)i) * ld + 3 * j;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) o[a * ld + b] = blk[3 * a + b];
}

// ------------------------------------------------------------------
// adaptive cross approximation, element-block partial pivoting, FP64
// ------------------------------------------------------------------
// The block approximated holds components ca .. ca + NC - 1 of every
// element (NC = 3: the full 3x3 coupling; NC = 2 / 1: the shear / normal
// part of a coplanar block).  Each step evaluates the residual of one
// element row (NC DOF rows) and of the best element column (NC DOF
// columns).  The NC x NC pivot block is then eliminated by up to NC scalar
// cross steps with complete pivoting, so the rank grows by 1..NC per step
// and the components of an element are always sampled together.  Stop when
// the update of a step has ||U_k V_k^T||_F <= tol ||S_k||_F on two
// consecutive steps.
constexpr int kAcaThreads = 256;     // workgroup of a block below kAcaBig elements on both sides
constexpr int kAcaThreadsBig = 512;  // the larger blocks (a whole CU at the kernel's register use)
constexpr int kAcaBig = 512;
constexpr int kAcaMaxRank = 192;

struct AcaDesc {
    int64_t t_begin, s_begin;    // cluster positions
    int64_t u_off, v_off;        // workspace: U [kmax][NC m], V [kmax][NC n]
    int64_t rrow_off, rcol_off;  // scratch: Rrow [NC][NC n], Rcol [NC m][NC]
    int64_t flag_off;            // bytes: row used [m], column used [n]
    int32_t m, n, first_row, kmax;
    int32_t ca, pad;             // first component of the part
};

__device__ inline void wave_argmax(double& v, int& i)
{
    for (int off = 32; off > 0; off >>= 1) {
        double v2 = __shfl_xor(v, off);
        int i2 = __shfl_xor(i, off);
        if (v2 > v || (v2 == v && i2 >= 0 && (i < 0 || i2 < i))) {
            v = v2;
            i = i2;
        }
    }
}

// block-wide argmax (ties -> smaller index); all threads get the result
template <int NT>
__device__ inline void block_argmax(double& v, int& i, double* s_v, int* s_i)
{
    wave_argmax(v, i);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        s_v[w] = v;
        s_i[w] = i;
    }
    __syncthreads();
    v = s_v[0];
    i = s_i[0];
    for (int q = 1; q < NT / 64; ++q) {
        double v2 = s_v[q];
        int i2 = s_i[q];
        if (v2 > v || (v2 == v && i2 >= 0 && (i < 0 || i2 < i))) {
            v = v2;
            i = i2;
        }
    }
    __syncthreads();
}

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// out[q] = A[q] . b for q < nq; A rows of length L with stride L.
// Deterministic: fixed per-thread order, fixed shuffle tree, fixed wave order.
template <int NT>
__device__ void block_dots(const double* A, const double* b, int64_t L, int nq, double* out, double* s_red)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int q0 = 0; q0 < nq; q0 += 8) {
        double acc[8];
        for (int t = 0; t < 8; ++t) acc[t] = 0.0;
        for (int64_t x = threadIdx.x; x < L; x += NT) {
            double bx = b[x];
            for (int t = 0; t < 8; ++t)
                if (q0 + t < nq) acc[t] += A[(int64_t)(q0 + t) * L + x] * bx;
        }
        for (int t = 0; t < 8; ++t) {
            double s = wave_sum(acc[t]);
            if (lane == 0) s_red[w * 8 + t] = s;
        }
        __syncthreads();
        if (threadIdx.x < 8 && q0 + (int)threadIdx.x < nq) {
            double s = 0.0;
            for (int ww = 0; ww < NT / 64; ++ww) s += s_red[ww * 8 + threadIdx.x];
            out[q0 + threadIdx.x] = s;
        }
        __syncthreads();
    }
}

template <int NC, int NT>
__global__ __launch_bounds__(NT) void k_aca(const ElemGeo* __restrict__ geo, const AcaDesc* __restrict__ descs,
                                                     double kG, double kN, double tol, double* __restrict__ ws,
                                                     uint8_t* __restrict__ flags, int* __restrict__ out_rank,
                                                     int* __restrict__ out_status)
{
    const AcaDesc D = descs[blockIdx.x];
    const int ca = D.ca;
    const int64_t m3 = NC * (int64_t)D.m, n3 = NC * (int64_t)D.n;
    double* U = ws + D.u_off;
    double* V = ws + D.v_off;
    double* Rrow = ws + D.rrow_off;
    double* Rcol = ws + D.rcol_off;
    uint8_t* rowused = flags + D.flag_off;
    uint8_t* colused = rowused + D.m;

    __shared__ double s_piv[NC * kAcaMaxRank];   // U rows of the pivot element, then V rows
    __shared__ double s_red[NT / 64 * 8];
    __shared__ int s_ired[NT / 64];
    __shared__ double s_uu[NC][kAcaMaxRank], s_vv[NC][kAcaMaxRank];
    __shared__ double s_P[NC * NC];

    for (int i = threadIdx.x; i < D.m; i += NT) rowused[i] = 0;
    for (int j = threadIdx.x; j < D.n; j += NT) colused[j] = 0;
    __syncthreads();

    int k = 0, ipiv = D.first_row, conv = 0, misses = 0;
    bool converged = false;
    double normS2 = 0.0;
    while (k + 1 <= D.kmax) {
        // ---- residual of pivot row element ipiv ----
        for (int idx = threadIdx.x; idx < NC * k; idx += NT) {
            int a = idx / k, q = idx - a * k;
            s_piv[a * kAcaMaxRank + q] = U[(int64_t)q * m3 + NC * ipiv + a];
        }
        __syncthreads();
        double best = -1.0;
        int bestj = -1;
        {
            const ElemGeo& R = geo[D.t_begin + ipiv];
            double x[3] = {R.c[0], R.c[1], R.c[2]};
            double fr[9];
            for (int t = 0; t < 9; ++t) fr[t] = R.fr[t];
            for (int j = threadIdx.x; j < D.n; j += NT) {
                double full[9], blk[NC * NC];
                dd_block(x, fr, geo[D.s_begin + j], kG, kN, full);
#pragma unroll
                for (int a = 0; a < NC; ++a)
#pragma unroll
                    for (int b = 0; b < NC; ++b) blk[NC * a + b] = full[3 * (ca + a) + ca + b];
                for (int q = 0; q < k; ++q) {
                    const double* vq = V + (int64_t)q * n3 + NC * j;
#pragma unroll
                    for (int a = 0; a < NC; ++a) {
                        double ua = s_piv[a * kAcaMaxRank + q];
#pragma unroll
                        for (int b = 0; b < NC; ++b) blk[NC * a + b] -= ua * vq[b];
                    }
                }
                double fro = 0.0;
                for (int a = 0; a < NC; ++a)
                    for (int b = 0; b < NC; ++b) {
                        Rrow[a * n3 + NC * j + b] = blk[NC * a + b];
                        fro += blk[NC * a + b] * blk[NC * a + b];
                    }
                if (!colused[j] && (fro > best)) {
                    best = fro;
                    bestj = j;
                }
            }
        }
        block_argmax<NT>(best, bestj, s_red, s_ired);
        const int jpiv = bestj;
        bool zero_row = (jpiv < 0) || !(best > 0.0);
        int k0 = k;
        if (!zero_row) {
            // ---- residual of pivot column element jpiv ----
            for (int idx = threadIdx.x; idx < NC * k; idx += NT) {
                int b = idx / k, q = idx - b * k;
                s_piv[b * kAcaMaxRank + q] = V[(int64_t)q * n3 + NC * jpiv + b];
            }
            __syncthreads();
            const ElemGeo& S = geo[D.s_begin + jpiv];
            for (int i = threadIdx.x; i < D.m; i += NT) {
                const ElemGeo& R = geo[D.t_begin + i];
                double x[3] = {R.c[0], R.c[1], R.c[2]};
                double fr[9];
                for (int t = 0; t < 9; ++t) fr[t] = R.fr[t];
                double full[9], blk[NC * NC];
                dd_block(x, fr, S, kG, kN, full);
#pragma unroll
                for (int a = 0; a < NC; ++a)
#pragma unroll
                    for (int b = 0; b < NC; ++b) blk[NC * a + b] = full[3 * (ca + a) + ca + b];
                for (int q = 0; q < k; ++q) {
                    const double* uq = U + (int64_t)q * m3 + NC * i;
#pragma unroll
                    for (int a = 0; a < NC; ++a) {
                        double ua = uq[a];
#pragma unroll
                        for (int b = 0; b < NC; ++b) blk[NC * a + b] -= ua * s_piv[b * kAcaMaxRank + q];
                    }
                }
                for (int a = 0; a < NC; ++a)
                    for (int b = 0; b < NC; ++b) Rcol[(NC * (int64_t)i + a) * NC + b] = blk[NC * a + b];
            }
            if (threadIdx.x < NC * NC)
                s_P[threadIdx.x] = Rrow[(threadIdx.x / NC) * n3 + NC * jpiv + threadIdx.x % NC];
            __syncthreads();
            // ---- eliminate the pivot block with complete pivoting ----
            double P[NC * NC];
            for (int t = 0; t < NC * NC; ++t) P[t] = s_P[t];
            double pmax0 = 0.0;
            for (int t = 0; t < NC * NC; ++t) pmax0 = fmax(pmax0, fabs(P[t]));
            bool rdone[NC], cdone[NC];
            for (int t = 0; t < NC; ++t) rdone[t] = cdone[t] = false;
            for (int sub = 0; sub < NC && k < D.kmax; ++sub) {
                int r = -1, c = -1;
                double pm = -1.0;
                for (int a = 0; a < NC; ++a)
                    for (int b = 0; b < NC; ++b)
                        if (!rdone[a] && !cdone[b] && fabs(P[NC * a + b]) > pm) {
                            pm = fabs(P[NC * a + b]);
                            r = a;
                            c = b;
                        }
                if (r < 0 || !(pm > 1e-10 * pmax0)) break;
                const double inv = 1.0 / P[NC * r + c];
                double* Uk = U + (int64_t)k * m3;
                double* Vk = V + (int64_t)k * n3;
                for (int64_t x = threadIdx.x; x < m3; x += NT) Uk[x] = Rcol[x * NC + c];
                for (int64_t y = threadIdx.x; y < n3; y += NT) Vk[y] = Rrow[r * n3 + y] * inv;
                __syncthreads();
                double vj[NC], ui[NC];
                for (int t = 0; t < NC; ++t) {
                    vj[t] = Vk[NC * jpiv + t];
                    ui[t] = Uk[NC * ipiv + t];
                }
                for (int64_t x = threadIdx.x; x < m3; x += NT) {
                    double u = Uk[x];
                    for (int t = 0; t < NC; ++t) Rcol[x * NC + t] -= u * vj[t];
                }
                for (int64_t y = threadIdx.x; y < n3; y += NT) {
                    double v = Vk[y];
                    for (int t = 0; t < NC; ++t) Rrow[t * n3 + y] -= ui[t] * v;
                }
                for (int a = 0; a < NC; ++a)
                    for (int b = 0; b < NC; ++b) P[NC * a + b] -= ui[a] * vj[b];
                rdone[r] = true;
                cdone[c] = true;
                ++k;
                __syncthreads();
            }
        }
        if (threadIdx.x == 0) {
            rowused[ipiv] = 1;
            if (jpiv >= 0) colused[jpiv] = 1;
        }
        __syncthreads();
        if (k == k0) {
            // nothing gained from this row: try the next unused row in order
            if (++misses > 8) {
                converged = (k > 0 && conv >= 1) || k == 0;
                break;
            }
            double v = -1.0;
            int nxt = -1;
            for (int i = threadIdx.x; i < D.m; i += NT)
                if (!rowused[i] && nxt < 0) {
                    v = (double)(D.m - i);  // smallest unused index wins
                    nxt = i;
                }
            block_argmax<NT>(v, nxt, s_red, s_ired);
            if (nxt < 0) {
                converged = true;
                break;
            }
            ipiv = nxt;
            continue;
        }
        // ---- Frobenius norm of the approximation, updated incrementally ----
        double step2 = 0.0;
        for (int qn = k0; qn < k; ++qn) {
            block_dots<NT>(U, U + (int64_t)qn * m3, m3, qn + 1, s_uu[qn - k0], s_red);
            block_dots<NT>(V, V + (int64_t)qn * n3, n3, qn + 1, s_vv[qn - k0], s_red);
        }
        for (int qn = k0; qn < k; ++qn) {
            double cross = 0.0;
            for (int q = 0; q < qn; ++q) cross += s_uu[qn - k0][q] * s_vv[qn - k0][q];
            normS2 += 2.0 * cross + s_uu[qn - k0][qn] * s_vv[qn - k0][qn];
            for (int pn = k0; pn < k; ++pn) {
                // (U_p . U_q)(V_p . V_q) for p, q in this step
                int lo = pn < qn ? pn : qn, hi = pn < qn ? qn : pn;
                step2 += s_uu[hi - k0][lo] * s_vv[hi - k0][lo];
            }
        }
        __syncthreads();
        conv = (step2 <= tol * tol * normS2) ? conv + 1 : 0;
        if (conv >= 2) {
            converged = true;
            break;
        }
        // ---- next pivot row: largest new column block among unused rows ----
        double v = -1.0;
        int nxt = -1;
        for (int i = threadIdx.x; i < D.m; i += NT) {
            if (rowused[i]) continue;
            double s = 0.0;
            for (int q = k0; q < k; ++q)
                for (int a = 0; a < NC; ++a) {
                    double u = U[(int64_t)q * m3 + NC * i + a];
                    s += u * u;
                }
            if (s > v) {
                v = s;
                nxt = i;
            }
        }
        block_argmax<NT>(v, nxt, s_red, s_ired);
        if (nxt < 0) {
            converged = true;  // every row has been sampled: the block is reproduced
            break;
        }
        ipiv = nxt;
        misses = 0;
    }
    // a cross approximation of full rank interpolates every row: exact
    if (k >= NC * min(D.m, D.n)) converged = true;
    if (threadIdx.x == 0) {
        out_rank[blockIdx.x] = k;
        out_status[blockIdx.x] = converged ? 0 : 1;
    }
}

// ------------------------------------------------------------------
// recompression of ACA factors (one workgroup per factorisation)
// ------------------------------------------------------------------
// For U V^T of rank k (columns of U and V contiguous): with D = diag(|u_q|),
// U D^-1 has unit columns; its Gram matrix A = (U D^-1)^T (U D^-1) and
// G = (V D)^T (V D) give the singular values of U V^T without another pass
// over the long factors:
//   * A = R^T R (Cholesky): U D^-1 = Q R with Q orthonormal, and the core
//     R G R^T = W S^2 W^T (cyclic Jacobi): T_u = D^-1 R^-1 W, T_v = D R^T W;
//   * when a Cholesky pivot is not clearly positive (nearly dependent cross
//     columns), A = Z L Z^T (Jacobi) instead; directions with eigenvalues
//     below 1e-14 of the largest are dropped (U has no component there), and
//     the core L^1/2 Z^T G Z L^1/2 = W S^2 W^T gives
//     T_u = D^-1 Z L^-1/2 W, T_v = D Z L^1/2 W.
// The k' largest singular values are kept with discarded energy
// sum_{i >= k'} s_i^2 <= tol^2 sum_i s_i^2, and U' = U T_u, V' = V T_v are
// always written (also when k' = k): U' has orthonormal columns and V'
// carries the singular values, so rounding the factors to a short format
// perturbs the block by that format's relative precision times its norm,
// whatever cancellation the cross approximation's columns had.
// Work matrices (k x k each): ranks up to 64 keep all four in LDS; ranks up
// to 128 keep the Jacobi target in LDS and the rest in a global slot of the
// workgroup; higher ranks (up to the cross-approximation cap) keep all four
// in the slot and stage the Gram products through LDS.  Eigenvector
// matrices are stored transposed (one eigenvector per row), so a rotation
// updates two contiguous rows.
constexpr int kRcSmall = 64;
constexpr int kRcMid = 128;
constexpr int kRcThreads = 1024;  // one workgroup per factorisation (the LDS use allows one per CU)
constexpr int kRcStage = 6144;    // doubles of LDS staging for the all-global kernel

template <int KMAX>
struct RcShape {
    static constexpr int LD = KMAX + 1;
    static constexpr size_t kMat = (size_t)KMAX * LD;          // doubles per work matrix
    static constexpr int kInLds = KMAX <= kRcSmall ? 4 : (KMAX <= kRcMid ? 1 : 0);  // matrices in LDS
    static constexpr size_t kSlot = (size_t)(4 - kInLds) * kMat;                      // doubles per global slot
    static constexpr size_t kLds = (kInLds ? kInLds * kMat : (size_t)kRcStage) * sizeof(double);
};

struct RcDesc {
    int64_t u_off, v_off;  // factor columns: U + q * lu, V + q * lv
    int64_t lu, lv;
    int64_t t_off;         // workspace: T_u [k][k'] then T_v [k][k']
    int32_t k, pad;
};

// A (k x k, upper triangle of a symmetric matrix) -> its Cholesky factor R
// (upper).  Returns false when a pivot is not clearly positive.
template <int LD>
__device__ bool rc_cholesky(double* A, int k, int* s_flag)
{
    double dmax = 0.0;
    for (int j = 0; j < k; ++j) dmax = fmax(dmax, A[j * LD + j]);
    for (int j = 0; j < k; ++j) {
        if (threadIdx.x == 0) {
            const double d = A[j * LD + j];
            if (!(d > 1e-14 * dmax)) {
                *s_flag = 1;
            } else {
                A[j * LD + j] = sqrt(d);
            }
        }
        __syncthreads();
        if (*s_flag) return false;
        const double r = A[j * LD + j];
        for (int l = j + 1 + threadIdx.x; l < k; l += blockDim.x) A[j * LD + l] /= r;
        __syncthreads();
        const int nn = k - j - 1;
        for (int idx = threadIdx.x; idx < nn * nn; idx += blockDim.x) {
            const int i = j + 1 + idx / nn, l = j + 1 + idx % nn;
            if (l >= i) A[i * LD + l] -= A[j * LD + i] * A[j * LD + l];
        }
        __syncthreads();
    }
    return true;
}

// Gram matrix G[a][b] = sum_i X[a][i] X[b][i] (a <= b) of k columns of
// length L, staged through LDS in column chunks; the pairs are taken in
// passes of (threads x kPer); fixed summation order.
template <int LD>
__device__ void rc_gram(const double* __restrict__ X, int64_t L, int k, double* G, double* stage, int stage_cap)
{
    const int T = max(1, stage_cap / k);
    const int npair = k * (k + 1) / 2;
    constexpr int kPer = 4;
    for (int p0 = 0; p0 < npair; p0 += (int)blockDim.x * kPer) {
        double acc[kPer];
        int pa[kPer], pb[kPer];
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            acc[t] = 0.0;
            // pair index -> (a, b), a <= b, row-major over the upper triangle
            int a = 0, rem = p0 + threadIdx.x + (int)blockDim.x * t;
            if (rem >= npair) {
                pa[t] = -1;
                pb[t] = -1;
                continue;
            }
            while (rem >= k - a) {
                rem -= k - a;
                ++a;
            }
            pa[t] = a;
            pb[t] = a + rem;
        }
        for (int64_t i0 = 0; i0 < L; i0 += T) {
            const int nt = (int)min((int64_t)T, L - i0);
            for (int idx = threadIdx.x; idx < k * nt; idx += blockDim.x) {
                const int q = idx / nt, t = idx % nt;
                stage[q * T + t] = X[(int64_t)q * L + i0 + t];
            }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < kPer; ++t) {
                if (pa[t] < 0) continue;
                const double* xa = stage + pa[t] * T;
                const double* xb = stage + pb[t] * T;
                double sacc = acc[t];
                for (int tt = 0; tt < nt; ++tt) sacc += xa[tt] * xb[tt];
                acc[t] = sacc;
            }
            __syncthreads();
        }
#pragma unroll
        for (int t = 0; t < kPer; ++t)
            if (pa[t] >= 0) G[pa[t] * LD + pb[t]] = acc[t];
    }
    __syncthreads();
}

// Eigen-decomposition of the symmetric k x k matrix S (full storage) by
// parallel cyclic Jacobi; Wt (k x k) must hold the identity on entry and
// receives the eigenvectors as rows (Wt[e][i] = component i of eigenvector
// e); the eigenvalues are left on the diagonal of S.
template <int LD>
__device__ void rc_jacobi(double* S, double* Wt, int k, double* s_c, double* s_s, int* s_p, int* s_q, double* s_red)
{
    // round-robin pairing over kk = k rounded up to even (the pad index is inert)
    const int kk = k + (k & 1);
    double fro2 = 0.0;
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) fro2 += S[a * LD + b] * S[a * LD + b];
    for (int sweep = 0; sweep < 30; ++sweep) {
        for (int round = 0; round < kk - 1; ++round) {
            // position 0 fixed, the others rotate
            for (int pi = threadIdx.x; pi < kk / 2; pi += blockDim.x) {
                int p0 = pi == 0 ? 0 : 1 + (pi - 1 + round) % (kk - 1);
                int q0 = 1 + (kk - 2 - pi + round) % (kk - 1);
                int p = min(p0, q0), q = max(p0, q0);
                double c = 1.0, sn = 0.0;
                if (q < k) {
                    const double apq = S[p * LD + q];
                    if (apq != 0.0) {
                        const double th = (S[q * LD + q] - S[p * LD + p]) / (2.0 * apq);
                        const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        sn = t * c;
                    }
                }
                s_p[pi] = p;
                s_q[pi] = q;
                s_c[pi] = c;
                s_s[pi] = sn;
            }
            __syncthreads();
            // rows: S <- J^T S
            for (int idx = threadIdx.x; idx < (kk / 2) * k; idx += blockDim.x) {
                const int pi = idx / k, j = idx % k;
                const int p = s_p[pi], q = s_q[pi];
                if (q >= k) continue;
                const double c = s_c[pi], sn = s_s[pi];
                const double xp = S[p * LD + j], xq = S[q * LD + j];
                S[p * LD + j] = c * xp - sn * xq;
                S[q * LD + j] = sn * xp + c * xq;
            }
            __syncthreads();
            // columns: S <- S J; eigenvectors: rows p, q of Wt <- J^T (rows p, q)
            for (int idx = threadIdx.x; idx < (kk / 2) * k; idx += blockDim.x) {
                const int pi = idx / k, j = idx % k;
                const int p = s_p[pi], q = s_q[pi];
                if (q >= k) continue;
                const double c = s_c[pi], sn = s_s[pi];
                const double xp = S[j * LD + p], xq = S[j * LD + q];
                S[j * LD + p] = c * xp - sn * xq;
                S[j * LD + q] = sn * xp + c * xq;
                const double wp = Wt[p * LD + j], wq = Wt[q * LD + j];
                Wt[p * LD + j] = c * wp - sn * wq;
                Wt[q * LD + j] = sn * wp + c * wq;
            }
            __syncthreads();
        }
        // off-diagonal energy
        double off = 0.0;
        for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x)
            if (idx / k != idx % k) off += S[(idx / k) * LD + idx % k] * S[(idx / k) * LD + idx % k];
        for (int o = 32; o > 0; o >>= 1) off += __shfl_xor(off, o);
        if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = off;
        __syncthreads();
        off = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) off += s_red[w];
        __syncthreads();
        if (!(off > 1e-30 * fro2)) break;
    }
}

// Order of the diagonal of S (descending, ties by index): sel[r] is the
// index of the r-th largest.
template <int LD>
__device__ void rc_order(const double* S, int k, int* sel)
{
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        const double li = S[i * LD + i];
        int r = 0;
        for (int j = 0; j < k; ++j) {
            const double lj = S[j * LD + j];
            if (lj > li || (lj == li && j < i)) ++r;
        }
        sel[r] = i;
    }
    __syncthreads();
}

template <int KMAX>
__global__ __launch_bounds__(kRcThreads) void k_recompress(const RcDesc* __restrict__ descs, const double* __restrict__ fac,
                                                     double tol, double* __restrict__ tws, int* __restrict__ out_k,
                                                     double* __restrict__ out_energy, double* __restrict__ slots)
{
    typedef RcShape<KMAX> Sh;
    constexpr int LD = Sh::LD;
    extern __shared__ double lds[];
    double* slot = slots + (size_t)blockIdx.x * Sh::kSlot;
    // A: U^T U -> R (or Z^T G); B: V^T V -> scaled (G), or W' of the eigen
    // route; C: R G, then W^T (or Z^T); S: the scaled U Gram, then the core
    double *A, *B, *C, *S, *stage;
    int stage_cap;
    if (Sh::kInLds == 4) {
        A = lds;
        B = A + Sh::kMat;
        C = B + Sh::kMat;
        S = C + Sh::kMat;
        stage = C;
        stage_cap = (int)(2 * Sh::kMat);
    } else if (Sh::kInLds == 1) {
        S = lds;
        A = slot;
        B = A + Sh::kMat;
        C = B + Sh::kMat;
        stage = S;
        stage_cap = (int)Sh::kMat;
    } else {
        A = slot;
        B = A + Sh::kMat;
        C = B + Sh::kMat;
        S = C + Sh::kMat;
        stage = lds;
        stage_cap = kRcStage;
    }
    __shared__ int s_flag;
    __shared__ double s_c[KMAX / 2], s_s[KMAX / 2];
    __shared__ int s_p[KMAX / 2], s_q[KMAX / 2];
    __shared__ double s_red[kRcThreads / 64];
    __shared__ int s_sel[KMAX], s_sel2[KMAX];
    __shared__ int s_kp, s_r;
    __shared__ double s_d[KMAX], s_l[KMAX];
    const RcDesc D = descs[blockIdx.x];
    const int k = D.k;
    if (threadIdx.x == 0) s_flag = 0;
    __syncthreads();
    // ---- Gram matrices ----
    rc_gram<LD>(fac + D.u_off, D.lu, k, A, stage, stage_cap);
    rc_gram<LD>(fac + D.v_off, D.lv, k, B, stage, stage_cap);
    // ---- column scaling D: unit columns of U, the scale moved into V ----
    for (int a = threadIdx.x; a < k; a += blockDim.x) s_d[a] = sqrt(A[a * LD + a]);
    __syncthreads();
    for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) {
        const int a = idx / k, b = idx % k;
        if (b < a) continue;
        const double dd = s_d[a] * s_d[b];
        A[a * LD + b] = dd > 0.0 ? A[a * LD + b] / dd : 0.0;
        B[a * LD + b] *= dd;
        B[b * LD + a] = B[a * LD + b];   // G in full storage
        S[a * LD + b] = A[a * LD + b];   // full symmetric copy for the eigen route
        S[b * LD + a] = A[a * LD + b];
    }
    __syncthreads();
    const bool chol = rc_cholesky<LD>(A, k, &s_flag);
    int r = k;
    if (chol) {
        // ---- C = R G, then B = R^T (G is not needed again) and S = C R^T;
        // each thread walks a row of the broadcast operand and a column of
        // the other, so a wavefront reads contiguous rows ----
        for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) {
            const int a = idx / k, b = idx % k;
            double sum = 0.0;
            for (int c = a; c < k; ++c) sum += A[a * LD + c] * B[c * LD + b];
            C[a * LD + b] = sum;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) {
            const int c = idx / k, b = idx % k;
            B[c * LD + b] = c >= b ? A[b * LD + c] : 0.0;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) {
            const int a = idx / k, b = idx % k;
            double sum = 0.0;
            for (int c = b; c < k; ++c) sum += C[a * LD + c] * B[c * LD + b];
            S[a * LD + b] = sum;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) C[(idx / k) * LD + idx % k] = (idx / k == idx % k);
        __syncthreads();
        rc_jacobi<LD>(S, C, k, s_c, s_s, s_p, s_q, s_red);
        rc_order<LD>(S, k, s_sel2);
    } else {
        // ---- eigen route: S = Z L Z^T (Z into C) ----
        for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) C[(idx / k) * LD + idx % k] = (idx / k == idx % k);
        __syncthreads();
        rc_jacobi<LD>(S, C, k, s_c, s_s, s_p, s_q, s_red);
        rc_order<LD>(S, k, s_sel);
        if (threadIdx.x == 0) {
            const double lmax = S[s_sel[0] * LD + s_sel[0]];
            int rr = 0;
            while (rr < k && S[s_sel[rr] * LD + s_sel[rr]] > 1e-14 * lmax && lmax > 0.0) ++rr;
            s_r = rr;
        }
        __syncthreads();
        r = s_r;
        for (int a = threadIdx.x; a < r; a += blockDim.x) s_l[a] = S[s_sel[a] * LD + s_sel[a]];
        __syncthreads();
        // A = Z_r^T G (r x k), then S = L^1/2 (A Z_r) L^1/2 (r x r), B = I
        for (int idx = threadIdx.x; idx < r * k; idx += blockDim.x) {
            const int a = idx / k, j = idx % k;
            double sum = 0.0;
            for (int c = 0; c < k; ++c) sum += C[s_sel[a] * LD + c] * B[c * LD + j];
            A[a * LD + j] = sum;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < r * r; idx += blockDim.x) {
            const int a = idx / r, b = idx % r;
            double sum = 0.0;
            for (int j = 0; j < k; ++j) sum += A[a * LD + j] * C[s_sel[b] * LD + j];
            S[a * LD + b] = sqrt(s_l[a] * s_l[b]) * sum;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < r * r; idx += blockDim.x) B[(idx / r) * LD + idx % r] = (idx / r == idx % r);
        __syncthreads();
        if (r > 0) rc_jacobi<LD>(S, B, r, s_c, s_s, s_p, s_q, s_red);
        rc_order<LD>(S, r, s_sel2);
    }
    // ---- choose k' on the core's eigenvalues (the squared singular values) ----
    if (threadIdx.x == 0) {
        double total = 0.0;
        for (int q = 0; q < r; ++q) total += fmax(0.0, S[s_sel2[q] * LD + s_sel2[q]]);
        const double budget = tol * tol * total;
        double tail = 0.0;
        int kp = r;
        // drop from the smallest while the discarded energy stays within the budget
        for (int q = r - 1; q >= 1; --q) {
            const double lq = fmax(0.0, S[s_sel2[q] * LD + s_sel2[q]]);
            if (tail + lq > budget) break;
            tail += lq;
            kp = q;
        }
        if (r == 0) kp = -1;   // a numerically zero block stays as it is
        s_kp = kp;
        out_k[blockIdx.x] = kp;
        out_energy[blockIdx.x] = total;
    }
    __syncthreads();
    const int kp = s_kp;
    if (kp < 1) return;
    double* Tu = tws + D.t_off;
    double* Tv = Tu + (int64_t)k * kp;
    if (chol) {
        // ---- T_u = D^-1 R^-1 W_k' (back substitution per column), T_v = D R^T W_k' ----
        for (int col = threadIdx.x; col < kp; col += blockDim.x) {
            const int e = s_sel2[col];
            for (int i = k - 1; i >= 0; --i) {
                double sum = C[e * LD + i];
                for (int c = i + 1; c < k; ++c) sum -= A[i * LD + c] * Tu[(int64_t)c * kp + col];
                Tu[(int64_t)i * kp + col] = sum / A[i * LD + i];
            }
            for (int i = 0; i < k; ++i) Tu[(int64_t)i * kp + col] /= s_d[i];
        }
        for (int idx = threadIdx.x; idx < k * kp; idx += blockDim.x) {
            const int col = idx / k, q = idx % k;
            const int e = s_sel2[col];
            double sum = 0.0;
            for (int c = 0; c <= q; ++c) sum += A[c * LD + q] * C[e * LD + c];
            Tv[(int64_t)q * kp + col] = sum * s_d[q];
        }
    } else {
        // ---- T_u = D^-1 Z_r L^-1/2 W_k', T_v = D Z_r L^1/2 W_k' ----
        for (int idx = threadIdx.x; idx < k * kp; idx += blockDim.x) {
            const int i = idx / kp, col = idx % kp;
            const int e = s_sel2[col];
            double su = 0.0, sv = 0.0;
            for (int a = 0; a < r; ++a) {
                const double zw = C[s_sel[a] * LD + i] * B[e * LD + a];
                const double sl = sqrt(s_l[a]);
                su += zw / sl;
                sv += zw * sl;
            }
            Tu[(int64_t)i * kp + col] = s_d[i] > 0.0 ? su / s_d[i] : 0.0;
            Tv[(int64_t)i * kp + col] = sv * s_d[i];
        }
    }
}

// X'[q'][i] = sum_q X[q][i] T[q][q'] for the U and V factors of one block
struct RcApply {
    int64_t src_u, src_v, dst_u, dst_v, lu, lv, t_off;
    int32_t k, kp;
};

// One item: an entry i of a factor and a tile of up to kRcCols output
// columns, so each X[q][i] is read once per tile; fixed summation order.
constexpr int kRcCols = 16;

__global__ void k_rc_apply(const RcApply* __restrict__ d, const double* __restrict__ fac,
                           const double* __restrict__ tws, double* __restrict__ out)
{
    const RcApply D = d[blockIdx.y];
    const int ntile = (D.kp + kRcCols - 1) / kRcCols;
    const int64_t nu = D.lu * ntile, nv = D.lv * ntile;
    const double* Tu = tws + D.t_off;
    const double* Tv = Tu + (int64_t)D.k * D.kp;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < nu + nv;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const bool isu = idx < nu;
        const int64_t e = isu ? idx : idx - nu;
        const int64_t L = isu ? D.lu : D.lv;
        const int tile = (int)(e / L);
        const int64_t i = e - (int64_t)tile * L;
        const double* X = fac + (isu ? D.src_u : D.src_v);
        const double* T = (isu ? Tu : Tv) + tile * kRcCols;
        const int nc = min(kRcCols, D.kp - tile * kRcCols);
        double acc[kRcCols];
#pragma unroll
        for (int c = 0; c < kRcCols; ++c) acc[c] = 0.0;
        for (int q = 0; q < D.k; ++q) {
            const double x = X[(int64_t)q * L + i];
            const double* t = T + (int64_t)q * D.kp;
#pragma unroll
            for (int c = 0; c < kRcCols; ++c)
                if (c < nc) acc[c] += x * t[c];
        }
        double* o = out + (isu ? D.dst_u : D.dst_v) + (int64_t)tile * kRcCols * L + i;
#pragma unroll
        for (int c = 0; c < kRcCols; ++c)
            if (c < nc) o[(int64_t)c * L] = acc[c];
    }
}

// ------------------------------------------------------------------
// packing into the apply layout
// ------------------------------------------------------------------
// Panel row r reads source row (r / rper) * rstride + roff + r % rper (and
// likewise for columns): (1, 1, 0) takes every DOF, (2, 3, 0) the shear and
// (1, 3, 2) the normal components of element-major 3-component data.
struct Sel {
    int32_t per, stride, off;
};
constexpr Sel kSelAll{1, 1, 0}, kSelShear3{2, 3, 0}, kSelNormal3{1, 3, 2};

struct PackDesc {
    int64_t src_off;  // FP64 source
    int64_t dst_off;  // panel start
    int64_t ld;       // source leading dimension
    int32_t rows, cols;
    int32_t mode;     // 0: row-major src[row*ld + col]; 1: src[col*ld + row] (source indices)
    int32_t zero_self;  // dense diagonal block: zero entries whose source row and column are one element
    Sel rs, cs;
    int32_t prow0;    // first row inside the destination panel (stacked panels)
    int32_t prows;    // destination panel rows (0: rows)
};

template <class T>
__global__ void k_pack(const PackDesc* __restrict__ descs, const double* __restrict__ src, T* __restrict__ dst, int w)
{
    const PackDesc D = descs[blockIdx.y];
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)D.rows * D.cols) return;
    int row = (int)(e / D.cols), col = (int)(e - (int64_t)row * D.cols);
    const int64_t sr = (int64_t)(row / D.rs.per) * D.rs.stride + D.rs.off + row % D.rs.per;
    const int64_t sc = (int64_t)(col / D.cs.per) * D.cs.stride + D.cs.off + col % D.cs.per;
    double v = D.mode == 0 ? src[D.src_off + sr * D.ld + sc] : src[D.src_off + sc * D.ld + sr];
    if (D.zero_self && sr / 3 == sc / 3) v = 0.0;
    const int M = D.prows ? D.prows : D.rows;
    dst[D.dst_off + panel_offset(M, D.cols, w, D.prow0 + row, col)] = cvt<T>(v);
}

// FP64 self blocks of each element, written in original element order
__global__ void k_extract_self(const DenseDesc* __restrict__ descs, const int* __restrict__ diag_ids, int n_diag,
                               const double* __restrict__ dense, const int64_t* __restrict__ perm,
                               double* __restrict__ self)
{
    int b = blockIdx.y;
    if (b >= n_diag) return;
    const DenseDesc D = descs[diag_ids[b]];
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= D.m) return;
    int64_t ld = 3 * (int64_t)D.n;
    int64_t e = perm[D.t_begin + i];
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) self[e * 9 + 3 * a + c] = dense[D.out_off + (3 * (int64_t)i + a) * ld + 3 * i + c];
}

// Copy each block's ACA factors (rank k) from its workspace slot to the
// compact FP64 store: one launch per ACA batch instead of one copy per block.
struct CompactDesc {
    int64_t src, dst, len;  // doubles
};

__global__ void k_compact(const CompactDesc* __restrict__ d, const double* __restrict__ ws, double* __restrict__ out)
{
    const CompactDesc D = d[blockIdx.y];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D.len; i += (int64_t)gridDim.x * blockDim.x)
        out[D.dst + i] = ws[D.src + i];
}

// ------------------------------------------------------------------
// host side
// ------------------------------------------------------------------
static double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void ensure_mesh_geo(Mesh& mesh)
{
    int dev = 0;
    HM_CHECK_HIP(hipGetDevice(&dev));
    if (mesh.d_geo.get() && mesh.d_geo_device == dev) return;
    mesh.d_geo.alloc(mesh.geo.size() * sizeof(ElemGeo));
    HM_CHECK_HIP(hipMemcpy(mesh.d_geo.get(), mesh.geo.data(), mesh.geo.size() * sizeof(ElemGeo), hipMemcpyHostToDevice));
    mesh.d_geo_device = dev;
}

void moduli(double young, double nu, double& G, double& kG, double& kN)
{
    HM_REQUIRE(young > 0.0 && std::isfinite(young), HM_EINVAL, "Young's modulus must be positive");
    HM_REQUIRE(nu > -1.0 && nu < 0.5, HM_EINVAL, "Poisson ratio must lie in (-1, 1/2)");
    G = young / (2.0 * (1.0 + nu));
    kG = G / (4.0 * M_PI);
    kN = G / (4.0 * M_PI * (1.0 - nu));
}

void leaf_blocks_coef(const Op& op, double* out, hipStream_t s)
{
    double G, kG, kN;
    moduli(op.young, op.nu, G, kG, kN);
    const Plan& p = op.plan;
    std::vector<DenseDesc> dd(p.leaves.size());
    int64_t off = 0, max_pairs = 0;
    for (size_t lf = 0; lf < p.leaves.size(); ++lf) {
        const Cluster& c = p.nodes[p.leaves[lf]];
        dd[lf] = DenseDesc{c.begin, c.begin, off, (int32_t)c.size(), (int32_t)c.size()};
        off += 9 * c.size() * c.size();
        max_pairs = std::max<int64_t>(max_pairs, c.size() * c.size());
    }
    HM_REQUIRE(off == op.leaf_inv_elems, HM_EINTERNAL, "leaf block layout mismatch");
    DevBuf d_dd;
    upload(d_dd, dd, s);
    for (size_t b0 = 0; b0 < dd.size(); b0 += 65535) {
        unsigned nb = (unsigned)std::min<size_t>(65535, dd.size() - b0);
        hipLaunchKernelGGL(k_dense_coef, dim3((unsigned)((max_pairs + 255) / 256), nb), dim3(256), 0, s,
                           op.d_geo.as<ElemGeo>(), d_dd.as<DenseDesc>() + b0, kG, kN, out);
        HM_CHECK_HIP(hipGetLastError());
    }
    // d_dd is released on return: finish its readers first
    HM_CHECK_HIP(hipStreamSynchronize(s));
}

void kernel_block(Mesh& mesh, double young, double nu, int64_t nr, const int64_t* d_rows, int64_t nc,
                  const int64_t* d_cols, double* d_out, hipStream_t s)
{
    double G, kG, kN;
    moduli(young, nu, G, kG, kN);
    HM_REQUIRE(nr >= 0 && nc >= 0, HM_EINVAL, "negative sizes");
    if (nr == 0 || nc == 0) return;
    HM_REQUIRE(d_rows && d_cols && d_out, HM_EINVAL, "null pointer");
    ensure_mesh_geo(mesh);
    int64_t total = nr * nc;
    int64_t grid = (total + 255) / 256;
    HM_REQUIRE(grid < (int64_t)1 << 31, HM_EINVAL, "block too large");
    hipLaunchKernelGGL(k_kernel_block, dim3((unsigned)grid), dim3(256), 0, s, mesh.d_geo.as<ElemGeo>(), d_rows, d_cols,
                       nr, nc, kG, kN, d_out);
    HM_CHECK_HIP(hipGetLastError());
}

namespace {

struct PackJob {
    std::vector<PackDesc> descs;
    int64_t max_entries = 0;
    void add(const PackDesc& d)
    {
        descs.push_back(d);
        max_entries = std::max<int64_t>(max_entries, (int64_t)d.rows * d.cols);
    }
};

template <class T>
void run_pack(const PackJob& job, const double* src, void* dst, int w, hipStream_t s)
{
    if (job.descs.empty()) return;
    DevBuf d;
    upload(d, job.descs, s);
    const size_t chunk = 65535;
    for (size_t b0 = 0; b0 < job.descs.size(); b0 += chunk) {
        size_t nb = std::min(chunk, job.descs.size() - b0);
        dim3 grid((unsigned)((job.max_entries + 255) / 256), (unsigned)nb);
        hipLaunchKernelGGL(k_pack<T>, grid, dim3(256), 0, s, d.as<PackDesc>() + b0, src, static_cast<T*>(dst), w);
        HM_CHECK_HIP(hipGetLastError());
    }
    HM_CHECK_HIP(hipStreamSynchronize(s));
}

void pack_dispatch(int prec, const PackJob& job, const double* src, void* dst, hipStream_t s)
{
    int w = prec_w(prec);
    if (prec == HM_F64) run_pack<double>(job, src, dst, w, s);
    else if (prec == HM_F32) run_pack<float>(job, src, dst, w, s);
    else run_pack<uint16_t>(job, src, dst, w, s);
}

}  // namespace

// Pack one precision variant and build its task lists.
//
// Every stored piece maps one section (shear: 2 DOF per element, normal: 1)
// of a target leaf to one section of a source leaf or to a T chunk:
//   * dense leaf pair: SS, SN, NS, NN pieces; SS and NN only when the two
//     leaves are coplanar (the SN, NS couplings vanish);
//   * low-rank factorisation of comps = 3: U split into a shear and a normal
//     slice per target leaf, V^T into a shear and a normal sub-panel per
//     source leaf, one T chunk; comps = 2 / 1 (the shear / normal part of a
//     coplanar block): one slice and one sub-panel per leaf.
// Phase B has one task per (target leaf, section).
namespace {

enum Section { kShear = 0, kNormal = 1 };

int sec_rows(int64_t m, int sec) { return sec == kShear ? 2 * (int)m : (int)m; }
int64_t sec_off(int64_t m, int sec) { return sec == kShear ? 0 : chunk_n_off(m); }

}  // namespace

static void make_variant(Op& op, Variant& v, const std::vector<DenseDesc>& dd, const double* d_dense,
                         const double* d_fac, hipStream_t s)
{
    const Plan& p = op.plan;
    const int wn = prec_w(v.near_prec), wf = prec_w(v.far_prec);
    const int nleaf = (int)p.leaves.size();
    // phase-B items, by (target leaf, section)
    std::vector<std::vector<PanelRef>> itemsB(2 * (size_t)nleaf);
    // ---- dense pieces ----
    int64_t near_elems = 0;
    v.near_entries = 0;
    {
        PackJob job;
        for (size_t b = 0; b < dd.size(); ++b) {
            const Cluster& tc = p.nodes[p.dense[b].first];
            const Cluster& sc = p.nodes[p.dense[b].second];
            const bool diag = p.dense[b].first == p.dense[b].second;
            const bool cop = coplanar_pair(p, p.dense[b].first, p.dense[b].second);
            for (int ts = 0; ts < 2; ++ts)
                for (int ss = 0; ss < 2; ++ss) {
                    if (cop && ts != ss) continue;
                    const int rows = sec_rows(tc.size(), ts), cols = sec_rows(sc.size(), ss);
                    job.add(PackDesc{dd[b].out_off, near_elems, 3 * (int64_t)dd[b].n, rows, cols, 0,
                                     (diag && v.self_separate) ? 1 : 0, ts == kShear ? kSelShear3 : kSelNormal3,
                                     ss == kShear ? kSelShear3 : kSelNormal3});
                    itemsB[2 * (size_t)tc.leaf_id + ts].push_back(
                        PanelRef{near_elems, (op.leaf_xoff[sc.leaf_id] + sec_off(sc.size(), ss)) * kNrhs, rows, cols,
                                 0, 0});
                    near_elems += panel_elems(rows, cols, wn);
                    v.near_entries += (int64_t)rows * cols;
                }
        }
        v.near_a.alloc(std::max<int64_t>(1, near_elems) * prec_bytes(v.near_prec));
        HM_CHECK_HIP(hipMemsetAsync(v.near_a.get(), 0, v.near_a.bytes(), s));
        pack_dispatch(v.near_prec, job, d_dense, v.near_a.get(), s);
    }
    v.bytes_near = near_elems * prec_bytes(v.near_prec);
    // ---- T chunks ----
    v.t_off.assign(op.lr.size(), 0);
    int64_t tfrag = 0;
    for (size_t b = 0; b < op.lr.size(); ++b) {
        if (op.lr[b].rank == 0) continue;
        v.t_off[b] = tfrag;
        tfrag += round_up(op.lr[b].rank, kChunkAlign) * kNrhs;
    }
    // ---- low-rank pieces: U slices per target leaf, stacked V^T sub-panels per source leaf ----
    v.vgroups.clear();
    v.bytes_far_u = v.bytes_far_v = 0;
    int64_t far_elems = 0;
    PackJob job;
    // sections carried by a factorisation and how to read them from it
    auto sections = [](const LowRank& L) {
        std::vector<std::pair<int, Sel>> secs;
        if (L.comps == 3)
            secs = {{kShear, kSelShear3}, {kNormal, kSelNormal3}};
        else
            secs = {{L.comp0 == 2 ? kNormal : kShear, kSelAll}};
        return secs;
    };
    // stack key: source cluster and section set (0 both, 1 shear, 2 normal)
    std::map<std::pair<int, int>, int> group_of;
    for (size_t b = 0; b < op.lr.size(); ++b) {
        const LowRank& L = op.lr[b];
        const Cluster& t = p.nodes[L.t_node];
        const int k = L.rank;
        if (k == 0) continue;
        const int nc = L.comps;
        const auto secs = sections(L);
        for (int lf = t.first_leaf; lf < t.first_leaf + t.n_leaves; ++lf) {
            const Cluster& c = p.nodes[p.leaves[lf]];
            for (const auto& sec : secs) {
                const int rows = sec_rows(c.size(), sec.first);
                job.add(PackDesc{L.u_off + nc * (c.begin - t.begin), far_elems, nc * L.m, rows, k, 1, 0, sec.second,
                                 kSelAll});
                itemsB[2 * (size_t)lf + sec.first].push_back(PanelRef{far_elems, v.t_off[b], rows, k, 1, 0});
                far_elems += panel_elems(rows, k, wf);
                v.bytes_far_u += panel_elems(rows, k, wf) * prec_bytes(v.far_prec);
            }
        }
        const int kind = nc == 3 ? 0 : (L.comp0 == 2 ? 2 : 1);
        // join the open stack of (source cluster, sections) unless it would
        // pass the row cap, else open a new one
        auto it = group_of.emplace(std::make_pair(L.s_node, kind), (int)v.vgroups.size());
        if (it.second) {
            v.vgroups.emplace_back();
        } else if (v.stackRowsA >= 1 && v.vgroups[it.first->second].K + k > v.stackRowsA) {
            it.first->second = (int)v.vgroups.size();
            v.vgroups.emplace_back();
        }
        Variant::VGroup& G = v.vgroups[it.first->second];
        G.blocks.push_back((int)b);
        G.lo.push_back(G.K);
        G.K += k;
    }
    for (Variant::VGroup& G : v.vgroups) {
        const LowRank& L0 = op.lr[G.blocks[0]];
        const Cluster& sc = p.nodes[L0.s_node];
        const auto secs = sections(L0);
        for (int lf = sc.first_leaf; lf < sc.first_leaf + sc.n_leaves; ++lf) {
            const Cluster& c = p.nodes[p.leaves[lf]];
            for (const auto& sec : secs) {
                const int cols = sec_rows(c.size(), sec.first);
                for (size_t j = 0; j < G.blocks.size(); ++j) {
                    const LowRank& L = op.lr[G.blocks[j]];
                    job.add(PackDesc{L.v_off + L.comps * (c.begin - sc.begin), far_elems, L.comps * L.n, L.rank,
                                     cols, 0, 0, kSelAll, sec.second, G.lo[j], G.K});
                }
                G.items.push_back(
                    PanelRef{far_elems, (op.leaf_xoff[lf] + sec_off(c.size(), sec.first)) * kNrhs, G.K, cols, 1, 0});
                far_elems += panel_elems(G.K, cols, wf);
                v.bytes_far_v += panel_elems(G.K, cols, wf) * prec_bytes(v.far_prec);
            }
        }
    }
    v.far_a.alloc(std::max<int64_t>(1, far_elems) * prec_bytes(v.far_prec));
    HM_CHECK_HIP(hipMemsetAsync(v.far_a.get(), 0, v.far_a.bytes(), s));
    pack_dispatch(v.far_prec, job, d_fac, v.far_a.get(), s);
    v.bytes_far = far_elems * prec_bytes(v.far_prec);

    // ---- phase-B sections: one per (target leaf, section), cut into row windows ----
    std::vector<PanelRef>& ib = v.hItemsB;
    v.sectionsB.clear();
    ib.clear();
    for (int lf = 0; lf < nleaf; ++lf) {
        const Cluster& c = p.nodes[p.leaves[lf]];
        for (int sec = 0; sec < 2; ++sec) {
            const auto& its = itemsB[2 * (size_t)lf + sec];
            v.sectionsB.push_back(TaskB{op.leaf_xoff[lf] + sec_off(c.size(), sec), sec_rows(c.size(), sec),
                                        (int32_t)ib.size(), (int32_t)its.size(), 0, 0, 0});
            ib.insert(ib.end(), its.begin(), its.end());
        }
    }
    build_tasksB(v, v.windowB);
    v.tfrag_elems = tfrag;
    if (v.leavesPerTaskA > 0) {
        build_tasksA(op, v, v.leavesPerTaskA);
    } else {
        // auto: 16 sub-panels per task (fewer partial slots) when that still
        // leaves at least 8 tasks per resident phase-A wavefront, else 8
        // (shorter tasks balance the launch's tail)
        build_tasksA(op, v, 16);
        if ((int64_t)v.hTasksA.size() < 8 * (int64_t)phaseA_resident_waves(v.near_prec, v.far_prec))
            build_tasksA(op, v, 8);
    }
    // ---- workspaces: the build stream's own is made now ----
    v.xel = op.xtot * kNrhs;
    upload_tasks(v, s);
    (void)v.workspace(s);
    HM_CHECK_HIP(hipStreamSynchronize(s));
}

void build_tasksB(Variant& v, int window)
{
    HM_REQUIRE(window >= 1 && window <= kTileWindowB, HM_EINVAL, "phase-B window must be 1 to 8 row tiles");
    v.windowB = window;
    std::vector<TaskB>& tb = v.hTasksB;
    tb.clear();
    for (const TaskB& sec : v.sectionsB) {
        const int tiles = (sec.rows + 15) / 16;
        for (int r0 = 0; r0 < tiles; r0 += window) {
            TaskB t = sec;
            t.r0 = r0;
            t.nt = std::min(window, tiles - r0);
            tb.push_back(t);
        }
    }
    v.splitB = order_tasksB(tb, v.hItemsB, v.near_prec, v.far_prec, true);
    v.nTasksB = (int)tb.size();
}

// Phase-A tasks: one per row window of a stacked panel set and run of at
// most items_per_task of its sub-panels.  A set covered by one run writes the
// members' T chunks directly; the others go through partial slots (one per
// run, stacked rows) and the reduction.
void build_tasksA(const Op& op, Variant& v, int items_per_task)
{
    (void)op;
    HM_REQUIRE(items_per_task >= 1, HM_EINVAL, "sub-panels per phase-A task must be positive");
    v.leavesPerTaskA = items_per_task;
    std::vector<TaskA>& ta = v.hTasksA;
    std::vector<PanelRef>& ia = v.hItemsA;
    std::vector<MemberT>& mt = v.hMembersA;
    std::vector<ReduceDesc>& red = v.hReduce;
    ta.clear();
    ia.clear();
    mt.clear();
    red.clear();
    int64_t tpart = 0;
    for (const Variant::VGroup& G : v.vgroups) {
        const int64_t slot = round_up(G.K, 16) * kNrhs;
        HM_REQUIRE(slot < (int64_t)1 << 31, HM_EINTERNAL, "stacked panel too tall");
        const auto& vs = G.items;
        const bool direct = vs.size() <= (size_t)items_per_task;
        const int64_t slot0 = tpart;
        int n_slots = 0;
        for (size_t q0 = 0; q0 < vs.size(); q0 += items_per_task) {
            TaskA t{direct ? 0 : tpart, G.K, (int32_t)ia.size(), 0, direct ? 1 : 0, 0, 0, 0, 0};
            for (size_t q = q0; q < std::min(vs.size(), q0 + (size_t)items_per_task); ++q) {
                ia.push_back(vs[q]);
                t.n_items++;
            }
            // one task per row window; the windows share the items and the slot
            for (int r0 = 0; r0 < (G.K + 15) / 16; r0 += kTileWindow) {
                t.r0 = r0;
                if (direct) {
                    const int w_lo = 16 * r0, w_hi = 16 * (r0 + window_tiles(G.K, r0));
                    t.mem_begin = (int32_t)mt.size();
                    t.n_mem = 0;
                    for (size_t j = 0; j < G.blocks.size(); ++j) {
                        const int k = op.lr[G.blocks[j]].rank;
                        if (G.lo[j] < w_hi && G.lo[j] + k > w_lo) {
                            mt.push_back(MemberT{v.t_off[G.blocks[j]], G.lo[j], k});
                            t.n_mem++;
                        }
                    }
                }
                ta.push_back(t);
            }
            if (!direct) {
                tpart += slot;
                n_slots++;
            }
        }
        if (!direct)
            for (size_t j = 0; j < G.blocks.size(); ++j)
                red.push_back(ReduceDesc{slot0 + (int64_t)G.lo[j] * kNrhs, v.t_off[G.blocks[j]], n_slots,
                                         op.lr[G.blocks[j]].rank, 0, (int32_t)slot});
    }
    v.splitA = order_tasksA(ta, ia, true);
    v.nTasksA = (int)ta.size();
    v.nReduce = (int)red.size();
    v.tpart_elems = tpart;
}

// Cut tasks (in their current order) into 8 contiguous ranges of about
// equal cost; with longest_first, sort each range by cost, longest first
// (stable).  Measured: sorting shortens one operator's product (the long
// tasks start first, the tail is short), while a merged batch of many
// operators runs faster in its natural order (each operator's tasks
// together, in leaf or source order, so an XCD's L2 holds one operator's
// vectors at a time).
template <class T>
static XcdSplit xcd_balance(std::vector<T>& tasks, const std::vector<int64_t>& cost, bool longest_first)
{
    XcdSplit sp{};
    const size_t n = tasks.size();
    std::vector<int64_t> pre(n + 1, 0);
    for (size_t q = 0; q < n; ++q) pre[q + 1] = pre[q] + cost[q];
    sp.begin[0] = 0;
    size_t q = 0;
    for (int x = 1; x < 8; ++x) {
        const int64_t target = pre[n] * x / 8;
        while (q < n && pre[q + 1] <= target) ++q;
        sp.begin[x] = (int32_t)q;
    }
    sp.begin[8] = (int32_t)n;
    if (!longest_first) return sp;
    for (int x = 0; x < 8; ++x) {
        std::vector<std::pair<int64_t, T>> part;
        for (int32_t t = sp.begin[x]; t < sp.begin[x + 1]; ++t) part.push_back({cost[t], tasks[t]});
        std::stable_sort(part.begin(), part.end(),
                         [](const std::pair<int64_t, T>& a, const std::pair<int64_t, T>& b) { return a.first > b.first; });
        for (size_t i = 0; i < part.size(); ++i) tasks[sp.begin[x] + i] = part[i].second;
    }
    return sp;
}

// bytes a task streams: its panels' rows inside the window times their
// granules, plus one 1 KB in-vector k-step per unit
static int64_t task_bytes(const PanelRef* it, int n_items, int R, int r0, int wn, int wf)
{
    int64_t c = 0;
    for (int q = 0; q < n_items; ++q) {
        const PanelRef& P = it[q];
        const int w = P.far ? wf : wn;
        const int64_t gran = (P.cols + w - 1) / w;
        c += (int64_t)std::min(16 * R, P.rows - 16 * r0) * gran * 16 + (gran + 3) / 4 * 1024;
    }
    return c;
}

XcdSplit order_tasksA(std::vector<TaskA>& ta, const std::vector<PanelRef>& items, bool longest_first)
{
    for (const TaskA& t : ta) {
        const int R = window_tiles(t.rows, t.r0);
        HM_REQUIRE(R >= 1 && R <= kTileWindow, HM_EINTERNAL, "phase-A window out of range");
    }
    // by operator, then source chunk: one XCD's L2 holds only its share of X
    std::stable_sort(ta.begin(), ta.end(), [&](const TaskA& a, const TaskA& b) {
        return a.op != b.op ? a.op < b.op : items[a.item_begin].b_off < items[b.item_begin].b_off;
    });
    std::vector<int64_t> cost(ta.size());
    for (size_t q = 0; q < ta.size(); ++q) {
        const TaskA& t = ta[q];
        // every sub-panel is far; the element width only scales the cost
        cost[q] = task_bytes(items.data() + t.item_begin, t.n_items, window_tiles(t.rows, t.r0), t.r0, 4, 4);
    }
    return xcd_balance(ta, cost, longest_first);
}

XcdSplit order_tasksB(std::vector<TaskB>& tb, const std::vector<PanelRef>& items, int near_prec, int far_prec,
                      bool longest_first)
{
    for (const TaskB& t : tb)
        HM_REQUIRE(t.nt >= 1 && t.nt <= kTileWindowB && 16 * (t.r0 + t.nt) < t.rows + 16, HM_EINTERNAL,
                   "phase-B window out of range");
    const int wn = prec_w(near_prec), wf = prec_w(far_prec);
    std::vector<int64_t> cost(tb.size());
    for (size_t q = 0; q < tb.size(); ++q)
        cost[q] = task_bytes(items.data() + tb[q].item_begin, tb[q].n_items, tb[q].nt, tb[q].r0, wn, wf);
    return xcd_balance(tb, cost, longest_first);
}

// Upload the task lists; the workspaces are resized on their next use (the
// partial-slot section depends on the phase-A task list).
void upload_tasks(Variant& v, hipStream_t s)
{
    v.maxNtB = 1;
    for (const TaskB& t : v.hTasksB) v.maxNtB = std::max(v.maxNtB, t.nt);
    upload(v.tasksB, v.hTasksB, s);
    upload(v.itemsB, v.hItemsB, s);
    upload(v.tasksA, v.hTasksA, s);
    upload(v.itemsA, v.hItemsA, s);
    upload(v.membersA, v.hMembersA, s);
    upload(v.reduce, v.hReduce, s);
    HM_CHECK_HIP(hipStreamSynchronize(s));
    std::lock_guard<std::mutex> g(v.ws_mu);
    ++v.gen;
}

// Recompress every factorisation of rank >= 2 at relative Frobenius
// tolerance tol (one workgroup each, one kernel per rank class: up to 64,
// up to 128, above, the larger in batches); the factors of every
// block with a usable result are rewritten as U T_u, V T_v, the rest (a
// numerically zero block) copied unchanged.  Replaces d_fac.
static void recompress_factors(Op& op, DevBuf& d_fac, double tol, hipStream_t s)
{
    const size_t nb = op.lr.size();
    std::vector<int64_t> t_off(nb, -1);
    int64_t tws = 0;
    std::vector<int> small, mid, large;
    for (size_t b = 0; b < nb; ++b) {
        const int k = op.lr[b].rank;
        if (k < 2) continue;
        HM_REQUIRE(k <= kAcaMaxRank, HM_EINTERNAL, "rank above the cross-approximation cap");
        t_off[b] = tws;
        tws += 2 * (int64_t)k * k;
        (k <= kRcSmall ? small : (k <= kRcMid ? mid : large)).push_back((int)b);
    }
    DevBuf d_t(std::max<int64_t>(1, tws) * sizeof(double));
    std::vector<int> kp(nb, -1);
    auto run = [&](const std::vector<int>& ids, auto kernel, size_t lds, size_t slot_doubles, size_t per_launch) {
        if (ids.empty()) return;
        HM_CHECK_HIP(hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        DevBuf d_slots(std::max<size_t>(1, slot_doubles * std::min(per_launch, ids.size())) * sizeof(double));
        for (size_t c0 = 0; c0 < ids.size(); c0 += per_launch) {
            const size_t n = std::min(per_launch, ids.size() - c0);
            std::vector<RcDesc> rc;
            for (size_t q = c0; q < c0 + n; ++q) {
                const LowRank& L = op.lr[ids[q]];
                const int64_t lu = (int64_t)L.comps * L.m, lv = (int64_t)L.comps * L.n;
                rc.push_back(RcDesc{L.u_off, L.v_off, lu, lv, t_off[ids[q]], L.rank, 0});
            }
            DevBuf d_rc, d_k(n * sizeof(int)), d_e(n * sizeof(double));
            upload(d_rc, rc, s);
            hipLaunchKernelGGL(kernel, dim3((unsigned)n), dim3(kRcThreads), lds, s, d_rc.as<RcDesc>(), d_fac.as<double>(),
                               tol, d_t.as<double>(), d_k.as<int>(), d_e.as<double>(), d_slots.as<double>());
            HM_CHECK_HIP(hipGetLastError());
            std::vector<int> ks(n);
            HM_CHECK_HIP(hipMemcpyAsync(ks.data(), d_k.get(), n * sizeof(int), hipMemcpyDeviceToHost, s));
            HM_CHECK_HIP(hipStreamSynchronize(s));
            for (size_t q = 0; q < n; ++q) kp[ids[c0 + q]] = ks[q];
        }
    };
    run(small, k_recompress<kRcSmall>, RcShape<kRcSmall>::kLds, 0, 1 << 20);
    // global slots of the work matrices outside LDS, 1024 workgroups per launch
    run(mid, k_recompress<kRcMid>, RcShape<kRcMid>::kLds, RcShape<kRcMid>::kSlot, 1024);
    run(large, k_recompress<kAcaMaxRank>, RcShape<kAcaMaxRank>::kLds, RcShape<kAcaMaxRank>::kSlot, 512);
    // new ranks and compact store: recompressed blocks through k_rc_apply, the rest copied
    std::vector<int> newk(nb);
    for (size_t b = 0; b < nb; ++b) newk[b] = kp[b] >= 1 ? kp[b] : op.lr[b].rank;
    int64_t total = 0;
    std::vector<int64_t> nu(nb), nv(nb);
    for (size_t b = 0; b < nb; ++b) {
        const LowRank& L = op.lr[b];
        nu[b] = total;
        total += (int64_t)newk[b] * L.comps * L.m;
        nv[b] = total;
        total += (int64_t)newk[b] * L.comps * L.n;
    }
    DevBuf out(std::max<int64_t>(1, total) * sizeof(double));
    std::vector<RcApply> ap;
    std::vector<CompactDesc> cp;
    for (size_t b = 0; b < nb; ++b) {
        const LowRank& L = op.lr[b];
        if (L.rank == 0) continue;
        const int64_t lu = (int64_t)L.comps * L.m, lv = (int64_t)L.comps * L.n;
        if (kp[b] >= 1) {
            ap.push_back(RcApply{L.u_off, L.v_off, nu[b], nv[b], lu, lv, t_off[b], L.rank, kp[b]});
        } else {
            cp.push_back(CompactDesc{L.u_off, nu[b], (int64_t)L.rank * lu});
            cp.push_back(CompactDesc{L.v_off, nv[b], (int64_t)L.rank * lv});
        }
    }
    if (!ap.empty()) {
        DevBuf d_ap;
        upload(d_ap, ap, s);
        for (size_t c0 = 0; c0 < ap.size(); c0 += 65535) {
            const unsigned n = (unsigned)std::min<size_t>(65535, ap.size() - c0);
            hipLaunchKernelGGL(k_rc_apply, dim3(32, n), dim3(256), 0, s, d_ap.as<RcApply>() + c0, d_fac.as<double>(),
                               d_t.as<double>(), out.as<double>());
            HM_CHECK_HIP(hipGetLastError());
        }
    }
    if (!cp.empty()) {
        DevBuf d_cp;
        upload(d_cp, cp, s);
        for (size_t c0 = 0; c0 < cp.size(); c0 += 65535) {
            const unsigned n = (unsigned)std::min<size_t>(65535, cp.size() - c0);
            hipLaunchKernelGGL(k_compact, dim3(64, n), dim3(256), 0, s, d_cp.as<CompactDesc>() + c0,
                               d_fac.as<double>(), out.as<double>());
            HM_CHECK_HIP(hipGetLastError());
        }
    }
    HM_CHECK_HIP(hipStreamSynchronize(s));
    for (size_t b = 0; b < nb; ++b) {
        op.lr[b].rank = newk[b];
        op.lr[b].u_off = nu[b];
        op.lr[b].v_off = nv[b];
    }
    d_fac = std::move(out);
}

void build_operator(Op& op, const Mesh& mesh_in, const hm_build_opts& o, hipStream_t s)
{
    Mesh& mesh = const_cast<Mesh&>(mesh_in);
    double t_start = now_ms();
    double G, kG, kN;
    moduli(op.young, op.nu, G, kG, kN);
    op.G = G;
    HM_REQUIRE(o.aca_tol > 0.0 && o.aca_tol < 1.0, HM_EINVAL, "aca_tol must be in (0, 1)");
    HM_REQUIRE(o.max_rank >= 3 && o.max_rank <= kAcaMaxRank, HM_EINVAL, "max_rank must be in [3, 192]");
    HM_REQUIRE(o.stack_rows >= -1, HM_EINVAL, "stack_rows must be >= -1");
    HM_REQUIRE(o.phase_a_items >= 0 && o.phase_a_items <= 4096, HM_EINVAL, "phase_a_items must be in [0, 4096]");
    HM_REQUIRE(o.phase_b_window >= 0 && o.phase_b_window <= kTileWindowB, HM_EINVAL, "phase_b_window must be in [0, 8]");
    HM_REQUIRE(o.near_prec == HM_F64 || o.near_prec == HM_F32, HM_EUNSUPPORTED, "near_prec must be F64 or F32");
    HM_REQUIRE(o.far_prec == HM_F64 || o.far_prec == HM_F32 || o.far_prec == HM_BF16 || o.far_prec == HM_BF16_1,
               HM_EUNSUPPORTED, "far_prec must be F64, F32, BF16 or BF16_1");
    HM_REQUIRE(!(o.near_prec == HM_F64 && o.far_prec != HM_F64), HM_EUNSUPPORTED,
               "an FP64 near field requires an FP64 far field");
    HM_REQUIRE(!(o.near_prec == HM_F32 && o.far_prec == HM_F64), HM_EUNSUPPORTED,
               "an FP32 near field takes an FP32 or BF16 far field");
    HM_CHECK_HIP(hipGetDevice(&op.device));
    op.ne = mesh.ne;
    op.e_cent = mesh.cent;
    op.e_frame = mesh.frame;
    op.e_h.resize(mesh.ne);
    for (int64_t e = 0; e < mesh.ne; ++e) op.e_h[e] = std::sqrt(mesh.area[e]);
    op.plan = make_plan(mesh, o.leaf_size, o.eta);
    const Plan& p = op.plan;
    const int nleaf = (int)p.leaves.size();
    op.leaf_xoff.resize(nleaf);
    op.xtot = 0;
    for (int lf = 0; lf < nleaf; ++lf) {
        op.leaf_xoff[lf] = op.xtot;
        op.xtot += chunk_len(p.nodes[p.leaves[lf]].size());
    }
    // element tables
    std::vector<ElemGeo> geo(mesh.ne);
    for (int64_t q = 0; q < mesh.ne; ++q) geo[q] = mesh.geo[p.perm[q]];
    // cluster-order geometry and permutation stay with the operator (the leaf
    // preconditioner recomputes its diagonal blocks from them)
    DevBuf& d_geo = op.d_geo;
    DevBuf& d_perm = op.d_perm;
    upload(d_geo, geo, s);
    upload(d_perm, p.perm, s);
    {
        std::vector<LeafIo> io(nleaf);
        for (int lf = 0; lf < nleaf; ++lf) {
            const Cluster& c = p.nodes[p.leaves[lf]];
            HM_REQUIRE(chunk_len(c.size()) <= kLeafDofMax, HM_EINTERNAL, "leaf chunk larger than the gather tile");
            io[lf] = LeafIo{op.leaf_xoff[lf], c.begin, (int32_t)c.size(), 0};
        }
        upload(op.d_leaf_io, io, s);
    }
    // ---- low-rank blocks: ACA rounds; a block that does not converge within
    //      max_rank is replaced by its children (leaf pairs that fail become dense) ----
    double t0 = now_ms();
    Plan& pm = op.plan;
    std::vector<std::pair<int, int>> cand = pm.lowrank;
    pm.lowrank.clear();
    op.lr.clear();
    std::vector<DevBuf> batch_fac;
    int64_t fac_total = 0;
    std::vector<std::pair<int, int64_t>> fac_where;  // per op.lr entry: batch, offset
    int64_t rank_sum = 0;
    int rmin = 1 << 30, rmax = 0, rounds = 0;
    const int64_t budget = (int64_t)6 << 30;  // bytes of ACA workspace per batch
    // One ACA job per part of a candidate pair: the full 3-component block,
    // or its shear and normal parts when the two clusters are coplanar.
    struct Job {
        int cand;
        int nc, ca;
        AcaDesc d;
    };
    while (!cand.empty()) {
        HM_REQUIRE(++rounds <= 40, HM_EINTERNAL, "block splitting did not terminate");
        std::vector<std::vector<Job>> jobs(cand.size());
        std::vector<int64_t> need(cand.size(), 0);
        for (size_t b = 0; b < cand.size(); ++b) {
            const Cluster& t = pm.nodes[cand[b].first];
            const Cluster& sc = pm.nodes[cand[b].second];
            const int64_t m = t.size(), n = sc.size();
            // first pivot: element nearest to the target cluster's mean collocation point
            double cm[3] = {0, 0, 0};
            for (int64_t q = t.begin; q < t.end; ++q)
                for (int k = 0; k < 3; ++k) cm[k] += mesh.cent[3 * pm.perm[q] + k];
            for (int k = 0; k < 3; ++k) cm[k] /= (double)t.size();
            int first = 0;
            double bd = 1e300;
            for (int64_t q = t.begin; q < t.end; ++q) {
                double d2 = 0.0;
                for (int k = 0; k < 3; ++k) {
                    double dx = mesh.cent[3 * pm.perm[q] + k] - cm[k];
                    d2 += dx * dx;
                }
                if (d2 < bd) {
                    bd = d2;
                    first = (int)(q - t.begin);
                }
            }
            std::vector<std::pair<int, int>> parts;
            if (coplanar_pair(pm, cand[b].first, cand[b].second))
                parts = {{2, 0}, {1, 2}};
            else
                parts = {{3, 0}};
            for (const auto& pc : parts) {
                const int nc = pc.first;
                const int kmax = (int)std::min<int64_t>(o.max_rank, nc * std::min(m, n));
                AcaDesc d{t.begin, sc.begin, 0, 0, 0, 0, 0, (int32_t)m, (int32_t)n, first, kmax, pc.second, 0};
                jobs[b].push_back(Job{(int)b, nc, pc.second, d});
                need[b] += 8 * ((int64_t)kmax * nc * (m + n) + (int64_t)nc * nc * (m + n)) + m + n + 64;
            }
        }
        // large blocks first inside each batch for load balance; the parts of
        // one pair stay in one batch
        std::vector<int> order(cand.size());
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return jobs[a][0].d.m + jobs[a][0].d.n > jobs[b][0].d.m + jobs[b][0].d.n;
        });
        std::vector<std::vector<int>> batches;
        {
            int64_t used = 0;
            std::vector<int> cur;
            for (int b : order) {
                if (!cur.empty() && used + need[b] > budget) {
                    batches.push_back(cur);
                    cur.clear();
                    used = 0;
                }
                cur.push_back(b);
                used += need[b];
            }
            if (!cur.empty()) batches.push_back(cur);
        }
        std::vector<std::pair<int, int>> next;
        for (const auto& bl : batches) {
            // workspace offsets for every job of the batch
            int64_t off = 0, foff = 0;
            std::vector<Job*> all;
            for (int b : bl)
                for (Job& j : jobs[b]) {
                    AcaDesc& d = j.d;
                    d.u_off = off;
                    off += (int64_t)d.kmax * j.nc * d.m;
                    d.v_off = off;
                    off += (int64_t)d.kmax * j.nc * d.n;
                    d.rrow_off = off;
                    off += (int64_t)j.nc * j.nc * d.n;
                    d.rcol_off = off;
                    off += (int64_t)j.nc * j.nc * d.m;
                    d.flag_off = foff;
                    foff += d.m + d.n;
                    all.push_back(&j);
                }
            DevBuf ws(off * sizeof(double)), fl(std::max<int64_t>(1, foff));
            std::vector<int> rk(all.size()), st(all.size());
            // blocks with a side of kAcaBig elements or more run with the
            // larger workgroup on a second stream, beside the others
            hipStream_t s2 = nullptr;
            hipEvent_t e_in = nullptr, e_out = nullptr;
            HM_CHECK_HIP(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
            HM_CHECK_HIP(hipEventCreateWithFlags(&e_in, hipEventDisableTiming));
            HM_CHECK_HIP(hipEventCreateWithFlags(&e_out, hipEventDisableTiming));
            for (int nc = 3; nc >= 1; --nc) {
                std::vector<AcaDesc> descs[2];
                std::vector<int> idx[2];
                for (size_t q = 0; q < all.size(); ++q)
                    if (all[q]->nc == nc) {
                        const int big = std::max(all[q]->d.m, all[q]->d.n) >= kAcaBig ? 1 : 0;
                        descs[big].push_back(all[q]->d);
                        idx[big].push_back((int)q);
                    }
                DevBuf d_bd[2], d_rank[2], d_stat[2];
                for (int big = 0; big < 2; ++big) {
                    if (descs[big].empty()) continue;
                    d_rank[big].alloc(descs[big].size() * sizeof(int));
                    d_stat[big].alloc(descs[big].size() * sizeof(int));
                    upload(d_bd[big], descs[big], s);
                }
                HM_CHECK_HIP(hipEventRecord(e_in, s));
                HM_CHECK_HIP(hipStreamWaitEvent(s2, e_in, 0));
                for (int big = 0; big < 2; ++big) {
                    if (descs[big].empty()) continue;
                    const dim3 grid((unsigned)descs[big].size());
                    hipStream_t sl = big ? s2 : s;
                    const unsigned nt = big ? kAcaThreadsBig : kAcaThreads;
                    auto args = [&](auto kernel) {
                        hipLaunchKernelGGL(kernel, grid, dim3(nt), 0, sl, d_geo.as<ElemGeo>(), d_bd[big].as<AcaDesc>(),
                                           kG, kN, o.aca_tol, ws.as<double>(), fl.as<uint8_t>(),
                                           d_rank[big].as<int>(), d_stat[big].as<int>());
                    };
                    if (nc == 3)
                        big ? args(k_aca<3, kAcaThreadsBig>) : args(k_aca<3, kAcaThreads>);
                    else if (nc == 2)
                        big ? args(k_aca<2, kAcaThreadsBig>) : args(k_aca<2, kAcaThreads>);
                    else
                        big ? args(k_aca<1, kAcaThreadsBig>) : args(k_aca<1, kAcaThreads>);
                    HM_CHECK_HIP(hipGetLastError());
                }
                HM_CHECK_HIP(hipEventRecord(e_out, s2));
                HM_CHECK_HIP(hipStreamWaitEvent(s, e_out, 0));
                for (int big = 0; big < 2; ++big) {
                    if (descs[big].empty()) continue;
                    std::vector<int> r(descs[big].size()), t(descs[big].size());
                    HM_CHECK_HIP(hipMemcpyAsync(r.data(), d_rank[big].get(), r.size() * sizeof(int),
                                                hipMemcpyDeviceToHost, s));
                    HM_CHECK_HIP(hipMemcpyAsync(t.data(), d_stat[big].get(), t.size() * sizeof(int),
                                                hipMemcpyDeviceToHost, s));
                    HM_CHECK_HIP(hipStreamSynchronize(s));
                    for (size_t q = 0; q < idx[big].size(); ++q) {
                        rk[idx[big][q]] = r[q];
                        st[idx[big][q]] = t[q];
                    }
                }
            }
            HM_CHECK_HIP(hipStreamSynchronize(s2));
            HM_CHECK_HIP(hipEventDestroy(e_in));
            HM_CHECK_HIP(hipEventDestroy(e_out));
            HM_CHECK_HIP(hipStreamDestroy(s2));
            // a pair is kept when every part converged (compact copy of its
            // factors); otherwise it is split
            std::vector<int> jrank(all.size());
            std::vector<char> pair_ok(cand.size(), 1);
            for (size_t q = 0; q < all.size(); ++q) {
                jrank[q] = rk[q];
                if (st[q] != 0) pair_ok[all[q]->cand] = 0;
            }
            int64_t csz = 0;
            for (size_t q = 0; q < all.size(); ++q)
                if (pair_ok[all[q]->cand]) csz += (int64_t)jrank[q] * all[q]->nc * (all[q]->d.m + all[q]->d.n);
            batch_fac.emplace_back(std::max<int64_t>(1, csz) * sizeof(double));
            const int bi = (int)batch_fac.size() - 1;
            int64_t c = 0;
            std::vector<CompactDesc> cd;
            size_t q = 0;
            for (int b : bl) {
                const int t_node = cand[b].first, s_node = cand[b].second;
                if (!pair_ok[b]) {
                    q += jobs[b].size();
                    split_block(pm, t_node, s_node, next, pm.dense);
                    continue;
                }
                for (const Job& j : jobs[b]) {
                    LowRank L;
                    L.t_node = t_node;
                    L.s_node = s_node;
                    L.m = j.d.m;
                    L.n = j.d.n;
                    L.comps = j.nc;
                    L.comp0 = j.ca;
                    L.rank = jrank[q];
                    L.u_off = c;
                    if (L.rank) cd.push_back(CompactDesc{j.d.u_off, c, (int64_t)L.rank * j.nc * L.m});
                    c += (int64_t)L.rank * j.nc * L.m;
                    L.v_off = c;
                    if (L.rank) cd.push_back(CompactDesc{j.d.v_off, c, (int64_t)L.rank * j.nc * L.n});
                    c += (int64_t)L.rank * j.nc * L.n;
                    fac_where.push_back({bi, 0});
                    op.lr.push_back(L);
                    rank_sum += L.rank;
                    rmin = std::min(rmin, L.rank);
                    rmax = std::max(rmax, L.rank);
                    ++q;
                }
                pm.lowrank.push_back({t_node, s_node});
            }
            if (!cd.empty()) {
                DevBuf d_cd;
                upload(d_cd, cd, s);
                for (size_t c0 = 0; c0 < cd.size(); c0 += 65535) {
                    const unsigned nb = (unsigned)std::min<size_t>(65535, cd.size() - c0);
                    hipLaunchKernelGGL(k_compact, dim3(64, nb), dim3(256), 0, s, d_cd.as<CompactDesc>() + c0,
                                       ws.as<double>(), batch_fac.back().as<double>());
                    HM_CHECK_HIP(hipGetLastError());
                }
            }
            HM_CHECK_HIP(hipStreamSynchronize(s));
            fac_total += (int64_t)(batch_fac.back().bytes() / sizeof(double));
        }
        cand.swap(next);
    }
    // merge batch stores into one FP64 factor buffer (offsets rebased)
    DevBuf d_fac(std::max<int64_t>(1, fac_total) * sizeof(double));
    {
        int64_t base = 0;
        std::vector<int64_t> bbase(batch_fac.size());
        for (size_t bi = 0; bi < batch_fac.size(); ++bi) {
            bbase[bi] = base;
            int64_t n = batch_fac[bi].bytes() / sizeof(double);
            HM_CHECK_HIP(hipMemcpyAsync(d_fac.as<double>() + base, batch_fac[bi].get(), n * sizeof(double),
                                        hipMemcpyDeviceToDevice, s));
            base += n;
        }
        for (size_t b = 0; b < op.lr.size(); ++b) {
            op.lr[b].u_off += bbase[fac_where[b].first];
            op.lr[b].v_off += bbase[fac_where[b].first];
        }
        HM_CHECK_HIP(hipStreamSynchronize(s));
        batch_fac.clear();
    }
    // SVD truncation of the cross approximations at half the block tolerance
    // (the cross approximation itself stops near the other half)
    int64_t rank_sum_aca = rank_sum;
    double t_rc0 = now_ms();
    if (o.recompress) {
        recompress_factors(op, d_fac, 0.5 * o.aca_tol, s);
        rank_sum = 0;
        rmin = 1 << 30;
        rmax = 0;
        for (const LowRank& L : op.lr) {
            rank_sum += L.rank;
            rmin = std::min(rmin, L.rank);
            rmax = std::max(rmax, L.rank);
        }
    }
    double t_rc1 = now_ms();
    sort_blocks(pm);  // dense list may have grown; keep it in target order
    double t1 = now_ms();
    // ---- dense leaves: FP64 coefficients ----
    std::vector<DenseDesc> dd(p.dense.size());
    int64_t dense_total = 0, max_pairs = 0;
    std::vector<int> diag_ids;
    for (size_t b = 0; b < p.dense.size(); ++b) {
        const Cluster& t = p.nodes[p.dense[b].first];
        const Cluster& sc = p.nodes[p.dense[b].second];
        dd[b] = DenseDesc{t.begin, sc.begin, dense_total, (int32_t)t.size(), (int32_t)sc.size()};
        dense_total += 9 * t.size() * sc.size();
        max_pairs = std::max<int64_t>(max_pairs, t.size() * sc.size());
        if (p.dense[b].first == p.dense[b].second) diag_ids.push_back((int)b);
    }
    DevBuf d_dense(std::max<int64_t>(1, dense_total) * sizeof(double));
    DevBuf d_dd;
    upload(d_dd, dd, s);
    for (size_t b0 = 0; b0 < dd.size(); b0 += 65535) {
        unsigned nb = (unsigned)std::min<size_t>(65535, dd.size() - b0);
        hipLaunchKernelGGL(k_dense_coef, dim3((unsigned)((max_pairs + 255) / 256), nb), dim3(256), 0, s,
                           d_geo.as<ElemGeo>(), d_dd.as<DenseDesc>() + b0, kG, kN, d_dense.as<double>());
        HM_CHECK_HIP(hipGetLastError());
    }
    op.d_self.alloc(9 * mesh.ne * sizeof(double));
    HM_CHECK_HIP(hipMemsetAsync(op.d_self.get(), 0, op.d_self.bytes(), s));
    if (!diag_ids.empty()) {
        DevBuf d_diag;
        upload(d_diag, diag_ids, s);
        for (size_t b0 = 0; b0 < diag_ids.size(); b0 += 65535) {
            unsigned nb = (unsigned)std::min<size_t>(65535, diag_ids.size() - b0);
            hipLaunchKernelGGL(k_extract_self, dim3((unsigned)((p.leaf_size + 255) / 256), nb), dim3(256), 0, s,
                               d_dd.as<DenseDesc>(), d_diag.as<int>() + b0, (int)nb, d_dense.as<double>(),
                               d_perm.as<int64_t>(), op.d_self.as<double>());
            HM_CHECK_HIP(hipGetLastError());
        }
        HM_CHECK_HIP(hipStreamSynchronize(s));
    }
    HM_CHECK_HIP(hipStreamSynchronize(s));
    double t2 = now_ms();

    // ---- leaf descriptors of the leaf block-Jacobi preconditioner ----
    {
        std::vector<LeafPc> lp(nleaf);
        int64_t off = 0;
        for (int lf = 0; lf < nleaf; ++lf) {
            const Cluster& c = p.nodes[p.leaves[lf]];
            HM_REQUIRE(3 * c.size() <= kLeafDofMax, HM_EINTERNAL, "leaf larger than the preconditioner supports");
            lp[lf] = LeafPc{off, c.begin, (int32_t)c.size(), 0};
            off += 9 * c.size() * c.size();
        }
        upload(op.d_leaf_desc, lp, s);
        op.leaf_inv_elems = off;
        op.d_leaf_inv.release();
        op.leaf_pc_current = false;
    }

    // ---- pack variants ----
    op.main.near_prec = o.near_prec;
    op.main.far_prec = o.far_prec;
    op.main.self_separate = o.near_prec != HM_F64;
    // 0: 128 rows for single-BF16 in-vectors (fewer, taller stacks measured
    // faster there), 64 otherwise; -1: no cap
    op.main.stackRowsA = o.stack_rows ? o.stack_rows : (o.far_prec == HM_BF16_1 ? 128 : 64);
    op.main.leavesPerTaskA = o.phase_a_items;
    // 0: 8-tile windows, so each in-vector k-step feeds up to 8 panel tiles
    // (equal or faster than 4 tiles in every form)
    op.main.windowB = o.phase_b_window ? o.phase_b_window : kTileWindowB;
    make_variant(op, op.main, dd, d_dense.as<double>(), d_fac.as<double>(), s);
    if (o.keep_f64_reference && o.near_prec != HM_F64) {
        op.ref.reset(new Variant());
        op.ref->near_prec = HM_F64;
        op.ref->far_prec = HM_F64;
        op.ref->self_separate = false;
        op.ref->stackRowsA = o.stack_rows ? o.stack_rows : 64;
        op.ref->leavesPerTaskA = o.phase_a_items;
        op.ref->windowB = o.phase_b_window ? o.phase_b_window : kTileWindowB;
        make_variant(op, *op.ref, dd, d_dense.as<double>(), d_fac.as<double>(), s);
    }
    double t3 = now_ms();
    // ---- statistics ----
    hm_op_stats& st = op.stats;
    std::memset(&st, 0, sizeof(st));
    st.n_elements = mesh.ne;
    st.n_dof = 3 * mesh.ne;
    st.n_leaves = nleaf;
    st.n_dense_blocks = (int64_t)p.dense.size();
    st.n_lowrank_blocks = (int64_t)p.lowrank.size();
    st.dense_entries = dense_total;
    int64_t lre = 0, lre_u = 0;
    for (const LowRank& L : op.lr) {
        lre += (int64_t)L.rank * L.comps * (L.m + L.n);
        lre_u += (int64_t)L.rank * L.comps * L.m;
    }
    st.lowrank_entries = lre;
    st.lowrank_entries_u = lre_u;
    st.dense_entries_stored = op.main.near_entries;
    st.self_f64_entries = op.main.self_separate ? 9 * mesh.ne : 0;
    st.bytes_near = op.main.bytes_near;
    st.bytes_far = op.main.bytes_far;
    st.bytes_self = st.self_f64_entries * 8;
    st.bytes_reference = op.ref ? op.ref->bytes_near + op.ref->bytes_far : 0;
    st.min_rank = op.lr.empty() ? 0 : rmin;
    st.max_rank = op.lr.empty() ? 0 : rmax;
    st.mean_rank = op.lr.empty() ? 0.0 : (double)rank_sum / (double)op.lr.size();
    st.near_prec = o.near_prec;
    st.far_prec = o.far_prec;
    st.coef_ms = t2 - t1;
    st.aca_ms = t_rc0 - t0;
    st.pack_ms = t3 - t2;
    st.build_ms = t3 - t_start;
    int64_t maxleaf = 0;
    {
        std::vector<int64_t> per(nleaf, 0);
        for (size_t b = 0; b < p.dense.size(); ++b)
            per[p.nodes[p.dense[b].first].leaf_id] +=
                (coplanar_pair(p, p.dense[b].first, p.dense[b].second) ? 5 : 9) * (int64_t)dd[b].m * dd[b].n *
                prec_bytes(o.near_prec);
        for (int64_t x : per) maxleaf = std::max(maxleaf, x);
    }
    st.max_dense_bytes_per_leaf = maxleaf;
    st.bytes_far_u = op.main.bytes_far_u;
    st.bytes_far_v = op.main.bytes_far_v;
    st.rank_sum = rank_sum;
    st.rank_sum_aca = rank_sum_aca;
    st.recompress_ms = t_rc1 - t_rc0;
}

}  // namespace hm
