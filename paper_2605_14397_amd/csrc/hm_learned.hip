// Learned correction of the block preconditioner of the tangent system
// A11 = E - eta/dt - C^ep (paper Sec. 3.1.1; the inner A11 solves of
// Sec. 3.3.1 are preconditioned by a cheap approximation of A11, point
// Jacobi in the paper).
//
// The preconditioner stays a fixed linear map of the residual r:
//     (M^-1 r)_e = B_e r_e + sum_{f in N(e)} W_ef r_f,
// with B_e the 3x3 block-Jacobi inverse (E_ee - D_e)^-1, N(e) the K
// elements nearest to e (e itself first; exact search over the cluster
// tree, ties by element id) and W_ef = (h_e / E') net(phi_ef), where net is
// a small MLP (32 -> H -> H -> 9, ReLU) of dimensionless pair features
// phi_ef and h_e = sqrt(area_e).  W_ef = 0 when e or f is inactive, so
// inactive rows keep z_e = r_e.  Training minimises
//     L = (1/ns) sum_s ||M^-1 b_s - x_s||^2 / ||x_s||^2
// over pairs A11 x_s = b_s of the method's tangent systems, with Adam.
// The network runs in FP32 (weights, activations); residuals, the loss and
// the weight-gradient sums are FP64 and reduced in a fixed order, so a
// training run is deterministic.
//
// Parameter layout (FP32, one array): W1 [32][H], b1 [H], W2 [H][H],
// b2 [H], W3 [H][9], b3 [9]; layer output o = b[o] + sum_k in[k] W[k][o];
// network output o = 3a + b is entry (a, b) of the 3x3 block.
//
// Features (per pair, FP32; entries 20..31 are zero):
//   0-2  position of f's centroid relative to e's, in e's frame, / h_e
//   3    distance / h_e
//   4-6  n_e.n_f, s1_e.s1_f, s2_e.s2_f
//   7-9  diagonal of D_e * h_e / E'
//   10-12 diagonal of D_f * h_f / E'
//   13   D_e(s1, n) * h_e / E'     14  D_f(s1, n) * h_f / E'
//   15   D_e(n, s1) * h_e / E'     16  h_f / h_e
//   17   1 if f = e
//   18-19 mean of D_nn h / E' and of (D_s1s1 + D_s2s2) h / (2 E') over the
//        active elements of e's cluster-tree leaf (the element's patch)
// with E' = E / (1 - nu^2).
#include <algorithm>
#include <cmath>
#include <queue>

#include "hm_op.hpp"

namespace hm {

constexpr int kF = 32;   // padded feature count
constexpr int kOut = 9;  // one 3x3 block per pair

struct NetDims {
    int H;
    int64_t oW1, ob1, oW2, ob2, oW3, ob3, total;
    explicit NetDims(int h) : H(h)
    {
        oW1 = 0;
        ob1 = oW1 + (int64_t)kF * H;
        oW2 = ob1 + H;
        ob2 = oW2 + (int64_t)H * H;
        oW3 = ob2 + H;
        ob3 = oW3 + (int64_t)H * kOut;
        total = ob3 + kOut;
    }
};

namespace {

unsigned g1(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

// ------------------------------------------------------------------
// features
// ------------------------------------------------------------------
__global__ void k_features(int64_t P, const int32_t* __restrict__ pe, const int32_t* __restrict__ pf,
                           const double* __restrict__ cent, const double* __restrict__ frame,
                           const double* __restrict__ hh, const double* __restrict__ D,
                           const uint8_t* __restrict__ mask, const double* __restrict__ patch, double inv_ep,
                           float* __restrict__ feat, double* __restrict__ scale)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int64_t e = pe[p], f = pf[p];
    const double* Fe = frame + 9 * e;
    const double* Ff = frame + 9 * f;
    const double d[3] = {cent[3 * f] - cent[3 * e], cent[3 * f + 1] - cent[3 * e + 1],
                         cent[3 * f + 2] - cent[3 * e + 2]};
    const double he = hh[e], hf = hh[f];
    float o[kF];
#pragma unroll
    for (int k = 0; k < kF; ++k) o[k] = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) o[a] = (float)(dot3(Fe + 3 * a, d) / he);
    o[3] = (float)(sqrt(dot3(d, d)) / he);
    o[4] = (float)dot3(Fe + 6, Ff + 6);
    o[5] = (float)dot3(Fe, Ff);
    o[6] = (float)dot3(Fe + 3, Ff + 3);
    if (D) {
        const double se = he * inv_ep, sf = hf * inv_ep;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            o[7 + a] = (float)(D[9 * e + 4 * a] * se);
            o[10 + a] = (float)(D[9 * f + 4 * a] * sf);
        }
        o[13] = (float)(D[9 * e + 2] * se);
        o[14] = (float)(D[9 * f + 2] * sf);
        o[15] = (float)(D[9 * e + 6] * se);
    }
    o[16] = (float)(hf / he);
    o[17] = e == f ? 1.f : 0.f;
    o[18] = (float)patch[2 * e];
    o[19] = (float)patch[2 * e + 1];
    float4* out = reinterpret_cast<float4*>(feat + p * kF);
#pragma unroll
    for (int k = 0; k < kF / 4; ++k) out[k] = make_float4(o[4 * k], o[4 * k + 1], o[4 * k + 2], o[4 * k + 3]);
    const bool act = !mask || (mask[e] && mask[f]);
    scale[p] = act ? he * inv_ep : 0.0;
}

// ------------------------------------------------------------------
// dense layers over pairs, one pair per thread, weights in LDS
// out[p][o] = act(b[o] + sum_k in[p][k] W[k][o])
// ------------------------------------------------------------------
template <int KIN, int KOUT, bool RELU>
__global__ __launch_bounds__(256) void k_layer_fwd(int64_t P, const float* __restrict__ in,
                                                   const float* __restrict__ W, const float* __restrict__ b,
                                                   float* __restrict__ out)
{
    __shared__ float sW[KIN * KOUT + KOUT];
    for (int i = threadIdx.x; i < KIN * KOUT; i += blockDim.x) sW[i] = W[i];
    for (int i = threadIdx.x; i < KOUT; i += blockDim.x) sW[KIN * KOUT + i] = b[i];
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float x[KIN];
    const float4* src = reinterpret_cast<const float4*>(in + p * KIN);
#pragma unroll
    for (int k = 0; k < KIN / 4; ++k) {
        const float4 v = src[k];
        x[4 * k] = v.x;
        x[4 * k + 1] = v.y;
        x[4 * k + 2] = v.z;
        x[4 * k + 3] = v.w;
    }
#pragma unroll 4
    for (int o = 0; o < KOUT; ++o) {
        float s = sW[KIN * KOUT + o];
#pragma unroll
        for (int k = 0; k < KIN; ++k) s = fmaf(x[k], sW[k * KOUT + o], s);
        out[p * KOUT + o] = (RELU && s < 0.f) ? 0.f : s;
    }
}

// dIn[p][k] = (sum_o dOut[p][o] W[k][o]) * [act[p][k] > 0]
template <int KIN, int KOUT>
__global__ __launch_bounds__(256) void k_layer_bwd(int64_t P, const float* __restrict__ dOut,
                                                   const float* __restrict__ W, const float* __restrict__ act,
                                                   float* __restrict__ dIn)
{
    __shared__ float sW[KIN * KOUT];
    for (int i = threadIdx.x; i < KIN * KOUT; i += blockDim.x) sW[i] = W[i];
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float g[KOUT];
#pragma unroll
    for (int o = 0; o < KOUT; ++o) g[o] = dOut[p * KOUT + o];
#pragma unroll 4
    for (int k = 0; k < KIN; ++k) {
        float s = 0.f;
#pragma unroll
        for (int o = 0; o < KOUT; ++o) s = fmaf(g[o], sW[k * KOUT + o], s);
        dIn[p * KIN + k] = act[p * KIN + k] > 0.f ? s : 0.f;
    }
}

// Weight gradient of one layer, gW[k][o] = sum_p in[p][k] dOut[p][o] and
// gb[o] = sum_p dOut[p][o]: a contraction over the P pairs on MFMA
// (16x16x4 FP32, the pair index as the reduction dimension).  Each
// workgroup reduces a chunk of kWgChunk pairs, staging 64-pair slices of
// both operands through LDS, and writes FP32 partial sums; the partials are
// then summed in FP64 in a fixed order (deterministic).
typedef float wf4 __attribute__((ext_vector_type(4)));
constexpr int kWgChunk = 4096;
constexpr int kWgStage = 64;

template <int KIN, int KOUT>
__global__ __launch_bounds__(256) void k_wgrad_mfma(int64_t P, const float* __restrict__ in,
                                                    const float* __restrict__ dOut, float* __restrict__ partial)
{
    constexpr int KOP = (KOUT + 15) / 16 * 16;  // output columns padded to tiles
    constexpr int RT = KIN / 16, CT = KOP / 16, NT = RT * CT;
    constexpr int TPW = (NT + 3) / 4;           // tiles per wave
    __shared__ float sIn[kWgStage][KIN + 1];
    __shared__ float sD[kWgStage][KOP + 1];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t p0 = (int64_t)blockIdx.x * kWgChunk;
    const int64_t p1 = min(P, p0 + kWgChunk);
    wf4 acc[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc[t] = wf4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;  // bias gradient: thread o < KOUT sums column o
    for (int64_t q0 = p0; q0 < p1; q0 += kWgStage) {
        for (int idx = threadIdx.x; idx < kWgStage * KIN; idx += 256) {
            const int r = idx / KIN, c = idx - r * KIN;
            sIn[r][c] = q0 + r < p1 ? in[(q0 + r) * KIN + c] : 0.f;
        }
        for (int idx = threadIdx.x; idx < kWgStage * KOP; idx += 256) {
            const int r = idx / KOP, c = idx - r * KOP;
            sD[r][c] = (q0 + r < p1 && c < KOUT) ? dOut[(q0 + r) * KOUT + c] : 0.f;
        }
        __syncthreads();
        if (threadIdx.x < KOUT)
            for (int r = 0; r < kWgStage; ++r) bsum += sD[r][threadIdx.x];
#pragma unroll
        for (int ks = 0; ks < kWgStage / 4; ++ks) {
            const int kr = 4 * ks + (lane >> 4);
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const int tile = wave + 4 * t;
                if (tile < NT) {
                    const int rt = tile / CT, ct = tile - rt * CT;
                    const float a = sIn[kr][16 * rt + (lane & 15)];
                    const float b = sD[kr][16 * ct + (lane & 15)];
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    // partial[wg][k][o] (k < KIN, o < KOUT), then partial[wg][KIN][o] = bias
    float* out = partial + (int64_t)blockIdx.x * (KIN + 1) * KOUT;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int tile = wave + 4 * t;
        if (tile < NT) {
            const int rt = tile / CT, ct = tile - rt * CT;
            const int o = 16 * ct + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int k = 16 * rt + 4 * (lane >> 4) + v;
                if (o < KOUT) out[k * KOUT + o] = acc[t][v];
            }
        }
    }
    if (threadIdx.x < KOUT) out[KIN * KOUT + threadIdx.x] = bsum;
}

__global__ void k_wgrad_final(int nwg, int n, const float* __restrict__ partial, float* __restrict__ gW,
                              float* __restrict__ gb, int Kin, int Kout)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    double s = 0.0;
    for (int w = 0; w < nwg; ++w) s += (double)partial[(int64_t)w * n + idx];
    const int k = idx / Kout, o = idx - k * Kout;
    if (k < Kin)
        gW[k * Kout + o] = (float)s;
    else
        gb[o] = (float)s;
}

// W_p = scale_p * out_p (FP32 blocks)
__global__ void k_out_to_blocks(int64_t P, const float* __restrict__ out, const double* __restrict__ scale,
                                float* __restrict__ Wb)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const double sc = scale[p];
#pragma unroll
    for (int k = 0; k < kOut; ++k) Wb[p * kOut + k] = (float)(sc * (double)out[p * kOut + k]);
}

// z_e = (M_base r)_e + sum_{pairs p of e} W_p r_{f(p)}  [- x_e], every
// column, with (M_base r)_e = B_e r_e (Binv given) or read from base
// (precomputed leaf block-Jacobi product; base may be z itself: each
// thread reads its element's base rows before writing them).  One element
// per thread; each W block is read once for all columns.
__global__ __launch_bounds__(256) void k_apply_learned(int64_t ne, int nrhs, const double* __restrict__ r,
                                                       int64_t ldr, double* z, int64_t ldz,
                                                       const double* __restrict__ Binv, const double* base,
                                                       int64_t ldbase, const int64_t* __restrict__ off,
                                                       const int32_t* __restrict__ pf,
                                                       const float* __restrict__ Wb, const double* __restrict__ X,
                                                       int64_t ldx)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    double y[kNrhs][3];
    if (Binv) {
        double Bk[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) Bk[k] = Binv[9 * e + k];
#pragma unroll
        for (int c = 0; c < kNrhs; ++c) {
            if (c < nrhs) {
                const double* rc = r + c * ldr + 3 * e;
                const double r0 = rc[0], r1 = rc[1], r2 = rc[2];
#pragma unroll
                for (int a = 0; a < 3; ++a) y[c][a] = Bk[3 * a] * r0 + Bk[3 * a + 1] * r1 + Bk[3 * a + 2] * r2;
            }
        }
    } else {
#pragma unroll
        for (int c = 0; c < kNrhs; ++c)
            if (c < nrhs)
#pragma unroll
                for (int a = 0; a < 3; ++a) y[c][a] = base[c * ldbase + 3 * e + a];
    }
    const int64_t p1 = off[e + 1];
    for (int64_t p = off[e]; p < p1; ++p) {
        float w[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) w[k] = Wb[p * kOut + k];
        const int64_t f = pf[p];
#pragma unroll
        for (int c = 0; c < kNrhs; ++c) {
            if (c < nrhs) {
                const double* rf = r + c * ldr + 3 * f;
                const double r0 = rf[0], r1 = rf[1], r2 = rf[2];
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    y[c][a] += (double)w[3 * a] * r0 + (double)w[3 * a + 1] * r1 + (double)w[3 * a + 2] * r2;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < kNrhs; ++c) {
        if (c < nrhs) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
                z[c * ldz + 3 * e + a] = y[c][a] - (X ? X[c * ldx + 3 * e + a] : 0.0);
        }
    }
}

// dL/dout_p = scale_p * sum_s w_s rho_{s,e} (outer) b_{s,f}
__global__ void k_pair_grad(int64_t P, const int32_t* __restrict__ pe, const int32_t* __restrict__ pf,
                            const double* __restrict__ scale, int ns, const double* __restrict__ rho, int64_t ldr,
                            const double* __restrict__ Bs, int64_t ldb, const double* __restrict__ wsamp,
                            float* __restrict__ dOut)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int64_t e = pe[p], f = pf[p];
    double g[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = 0; s < ns; ++s) {
        const double* re = rho + s * ldr + 3 * e;
        const double* bf = Bs + s * ldb + 3 * f;
        const double ws = wsamp[s];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double ra = ws * re[a];
#pragma unroll
            for (int b = 0; b < 3; ++b) g[3 * a + b] += ra * bf[b];
        }
    }
    const double sc = scale[p];
#pragma unroll
    for (int k = 0; k < 9; ++k) dOut[p * kOut + k] = (float)(sc * g[k]);
}

// per-column sum of squares, partial sums in fixed order
constexpr int kSumsqBlocks = 256;
__global__ __launch_bounds__(256) void k_sumsq_partial(int64_t n, const double* __restrict__ v, int64_t ld,
                                                       double* __restrict__ partial)
{
    const int c = blockIdx.y;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s += v[c * ld + i] * v[c * ld + i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[(int64_t)c * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_adam(int64_t n, float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// splitmix64 (seeded initialisation of the network)
uint64_t splitmix(uint64_t& s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ------------------------------------------------------------------
// exact K-nearest search over the cluster tree (host)
// ------------------------------------------------------------------
struct Knn {
    const Plan& p;
    const double* cent;
    int K;
    // max-heap on (d2, id): the worst kept candidate on top
    std::priority_queue<std::pair<double, int64_t>> heap;

    static double box_d2(const Cluster& c, const double* q)
    {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double g = std::fmax(0.0, std::fmax(c.bmin[k] - q[k], q[k] - c.bmax[k]));
            s += g * g;
        }
        return s;
    }
    void offer(double d2, int64_t id)
    {
        if ((int)heap.size() < K) {
            heap.push({d2, id});
        } else if (std::make_pair(d2, id) < heap.top()) {
            heap.pop();
            heap.push({d2, id});
        }
    }
    // cluster boxes bound the element vertices, hence the centroids: a
    // cluster farther than the current K-th candidate cannot contribute
    void visit(int node, const double* q)
    {
        const Cluster& c = p.nodes[node];
        if ((int)heap.size() == K && box_d2(c, q) > heap.top().first) return;
        if (c.is_leaf()) {
            for (int64_t i = c.begin; i < c.end; ++i) {
                const int64_t f = p.perm[i];
                double d2 = 0.0;
                for (int k = 0; k < 3; ++k) {
                    const double dx = cent[3 * f + k] - q[k];
                    d2 += dx * dx;
                }
                offer(d2, f);
            }
            return;
        }
        const int a = c.child[0], b = c.child[1];
        if (box_d2(p.nodes[a], q) <= box_d2(p.nodes[b], q)) {
            visit(a, q);
            visit(b, q);
        } else {
            visit(b, q);
            visit(a, q);
        }
    }
};

}  // namespace

// ------------------------------------------------------------------
// host side
// ------------------------------------------------------------------
Learned::Learned(int hidden, int neighbors, uint64_t seed) : H(hidden), K(neighbors)
{
    HM_REQUIRE(hidden == 16 || hidden == 32 || hidden == 64, HM_EINVAL, "hidden width must be 16, 32 or 64");
    HM_REQUIRE(neighbors >= 1 && neighbors <= 64, HM_EINVAL, "neighbours must be in [1, 64]");
    NetDims d(H);
    n = d.total;
    std::vector<float> h(n, 0.f);
    uint64_t st = seed;
    auto uni = [&]() { return (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0); };
    auto fill = [&](int64_t o, int fin, int fout, double gain) {
        const double a = gain * std::sqrt(6.0 / (fin + fout));
        for (int64_t i = 0; i < (int64_t)fin * fout; ++i) h[o + i] = (float)((2.0 * uni() - 1.0) * a);
    };
    fill(d.oW1, kF, H, 1.0);
    fill(d.oW2, H, H, 1.0);
    fill(d.oW3, H, kOut, 0.01);  // the correction starts near zero: M^-1 starts at block-Jacobi
    params.alloc(n * sizeof(float));
    m.alloc(n * sizeof(float));
    v.alloc(n * sizeof(float));
    grad.alloc(n * sizeof(float));
    HM_CHECK_HIP(hipMemcpy(params.get(), h.data(), n * sizeof(float), hipMemcpyHostToDevice));
    reset_moments();
}

void Learned::reset_moments()
{
    HM_CHECK_HIP(hipMemset(m.get(), 0, n * sizeof(float)));
    HM_CHECK_HIP(hipMemset(v.get(), 0, n * sizeof(float)));
    HM_CHECK_HIP(hipMemset(grad.get(), 0, n * sizeof(float)));
    step = 0;
}

namespace {

template <int H>
void forward_h(const Learned& L, int64_t P, const float* feat, float* a1, float* a2, float* out, hipStream_t s)
{
    NetDims d(H);
    const float* th = L.params.as<float>();
    hipLaunchKernelGGL((k_layer_fwd<kF, H, true>), dim3(g1(P)), dim3(256), 0, s, P, feat, th + d.oW1, th + d.ob1,
                       a1);
    hipLaunchKernelGGL((k_layer_fwd<H, H, true>), dim3(g1(P)), dim3(256), 0, s, P, a1, th + d.oW2, th + d.ob2, a2);
    hipLaunchKernelGGL((k_layer_fwd<H, kOut, false>), dim3(g1(P)), dim3(256), 0, s, P, a2, th + d.oW3, th + d.ob3,
                       out);
    HM_CHECK_HIP(hipGetLastError());
}

void forward(const Learned& L, int64_t P, const float* feat, float* a1, float* a2, float* out, hipStream_t s)
{
    switch (L.H) {
    case 16: forward_h<16>(L, P, feat, a1, a2, out, s); break;
    case 32: forward_h<32>(L, P, feat, a1, a2, out, s); break;
    default: forward_h<64>(L, P, feat, a1, a2, out, s); break;
    }
}

int wgrad_groups(int64_t P) { return (int)std::max<int64_t>(1, (P + kWgChunk - 1) / kWgChunk); }

// doubles of workspace the (FP32) partial sums of a width-H network need
size_t wgrad_partial_size(int64_t P, int H)
{
    const int per = std::max({(kF + 1) * H, (H + 1) * H, (H + 1) * kOut});
    return ((size_t)wgrad_groups(P) * per + 1) / 2;
}

template <int KIN, int KOUT>
void weight_grad(int64_t P, const float* in, const float* dOut, float* gW, float* gb, double* part, size_t part_cap,
                 hipStream_t s)
{
    const int nwg = wgrad_groups(P);
    const int n = (KIN + 1) * KOUT;
    HM_REQUIRE(((size_t)nwg * n + 1) / 2 <= part_cap, HM_EINTERNAL, "weight-gradient workspace too small");
    float* pf = reinterpret_cast<float*>(part);
    hipLaunchKernelGGL((k_wgrad_mfma<KIN, KOUT>), dim3(nwg), dim3(256), 0, s, P, in, dOut, pf);
    hipLaunchKernelGGL(k_wgrad_final, dim3(g1(n)), dim3(256), 0, s, nwg, n, pf, gW, gb, KIN, KOUT);
    HM_CHECK_HIP(hipGetLastError());
}

template <int H>
void backward_h(Learned& L, int64_t P, const float* feat, const float* a1, const float* a2, const float* dO,
                float* d2, float* d1, double* part, size_t cap, hipStream_t s)
{
    NetDims d(H);
    const float* th = L.params.as<float>();
    float* gr = L.grad.as<float>();
    weight_grad<H, kOut>(P, a2, dO, gr + d.oW3, gr + d.ob3, part, cap, s);
    hipLaunchKernelGGL((k_layer_bwd<H, kOut>), dim3(g1(P)), dim3(256), 0, s, P, dO, th + d.oW3, a2, d2);
    weight_grad<H, H>(P, a1, d2, gr + d.oW2, gr + d.ob2, part, cap, s);
    hipLaunchKernelGGL((k_layer_bwd<H, H>), dim3(g1(P)), dim3(256), 0, s, P, d2, th + d.oW2, a1, d1);
    weight_grad<kF, H>(P, feat, d1, gr + d.oW1, gr + d.ob1, part, cap, s);
    HM_CHECK_HIP(hipGetLastError());
}

void backward(Learned& L, int64_t P, const float* feat, const float* a1, const float* a2, const float* dO, float* d2,
              float* d1, double* part, size_t cap, hipStream_t s)
{
    switch (L.H) {
    case 16: backward_h<16>(L, P, feat, a1, a2, dO, d2, d1, part, cap, s); break;
    case 32: backward_h<32>(L, P, feat, a1, a2, dO, d2, d1, part, cap, s); break;
    default: backward_h<64>(L, P, feat, a1, a2, dO, d2, d1, part, cap, s); break;
    }
}

// column sums of squares of v [ncol][ld] (first n entries), fixed order
std::vector<double> sumsq(int ncol, int64_t n, const double* v, int64_t ld, double* part, size_t cap, hipStream_t s)
{
    HM_REQUIRE((size_t)ncol * kSumsqBlocks <= cap, HM_EINTERNAL, "reduction workspace too small");
    hipLaunchKernelGGL(k_sumsq_partial, dim3(kSumsqBlocks, ncol), dim3(256), 0, s, n, v, ld, part);
    HM_CHECK_HIP(hipGetLastError());
    std::vector<double> hp((size_t)ncol * kSumsqBlocks);
    HM_CHECK_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HM_CHECK_HIP(hipStreamSynchronize(s));
    std::vector<double> out(ncol, 0.0);
    for (int c = 0; c < ncol; ++c)
        for (int k = 0; k < kSumsqBlocks; ++k) out[c] += hp[(size_t)c * kSumsqBlocks + k];
    return out;
}

}  // namespace

void learned_prepare(Op& op, int K, hipStream_t s)
{
    HM_REQUIRE(K >= 1 && K <= 64, HM_EINVAL, "neighbours must be in [1, 64]");
    const Plan& p = op.plan;
    const int64_t ne = op.ne;
    LearnedPairs& lp = op.lp;
    if (lp.K != K) {
        std::vector<int32_t> pe, pf;
        std::vector<int64_t> off(ne + 1, 0);
        pe.reserve((size_t)ne * K);
        pf.reserve((size_t)ne * K);
        Knn knn{p, op.e_cent.data(), (int)std::min<int64_t>(K, ne), {}};
        std::vector<std::pair<double, int64_t>> got;
        for (int64_t e = 0; e < ne; ++e) {
            knn.visit(0, &op.e_cent[3 * e]);
            got.clear();
            while (!knn.heap.empty()) {
                got.push_back(knn.heap.top());
                knn.heap.pop();
            }
            std::sort(got.begin(), got.end());
            for (auto& g : got) {
                pe.push_back((int32_t)e);
                pf.push_back((int32_t)g.second);
            }
            off[e + 1] = (int64_t)pe.size();
        }
        lp.P = (int64_t)pe.size();
        upload(lp.pe, pe, s);
        upload(lp.pf, pf, s);
        upload(lp.off, off, s);
        lp.feat.alloc(lp.P * kF * sizeof(float));
        lp.scale.alloc(lp.P * sizeof(double));
        lp.W.alloc(lp.P * kOut * sizeof(float));
        lp.K = K;
        lp.features_current = false;
        lp.attached = false;
    }
    if (lp.features_current) return;
    const double Ep = op.young / (1.0 - op.nu * op.nu);
    std::vector<double> Dh, patch(2 * ne, 0.0);
    std::vector<uint8_t> mh;
    if (op.has_D) {
        Dh.resize(9 * ne);
        HM_CHECK_HIP(hipMemcpyAsync(Dh.data(), op.d_D.get(), 9 * ne * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    if (op.has_mask) {
        mh.resize(ne);
        HM_CHECK_HIP(hipMemcpyAsync(mh.data(), op.d_mask.get(), ne, hipMemcpyDeviceToHost, s));
    }
    HM_CHECK_HIP(hipStreamSynchronize(s));
    if (op.has_D) {
        for (int leaf : p.leaves) {
            const Cluster& c = p.nodes[leaf];
            double sn = 0.0, ss = 0.0;
            int64_t na = 0;
            for (int64_t q = c.begin; q < c.end; ++q) {
                const int64_t e = p.perm[q];
                if (op.has_mask && !mh[e]) continue;
                const double sc = op.e_h[e] / Ep;
                sn += Dh[9 * e + 8] * sc;
                ss += 0.5 * (Dh[9 * e] + Dh[9 * e + 4]) * sc;
                ++na;
            }
            if (na == 0) continue;
            for (int64_t q = c.begin; q < c.end; ++q) {
                patch[2 * p.perm[q]] = sn / (double)na;
                patch[2 * p.perm[q] + 1] = ss / (double)na;
            }
        }
    }
    DevBuf dcent, dframe, dh, dpatch;
    upload(dcent, op.e_cent, s);
    upload(dframe, op.e_frame, s);
    upload(dh, op.e_h, s);
    upload(dpatch, patch, s);
    if (lp.P > 0)
        hipLaunchKernelGGL(k_features, dim3(g1(lp.P)), dim3(256), 0, s, lp.P, lp.pe.as<int32_t>(),
                           lp.pf.as<int32_t>(), dcent.as<double>(), dframe.as<double>(), dh.as<double>(),
                           op.has_D ? op.d_D.as<double>() : nullptr, op.has_mask ? op.d_mask.as<uint8_t>() : nullptr,
                           dpatch.as<double>(), 1.0 / Ep, lp.feat.as<float>(), lp.scale.as<double>());
    HM_CHECK_HIP(hipGetLastError());
    HM_CHECK_HIP(hipStreamSynchronize(s));
    lp.features_current = true;
}

double learned_loss_grad(Learned& L, Op& op, int ns, const double* B, int64_t ldb, const double* X, int64_t ldx,
                         hipStream_t s)
{
    HM_REQUIRE(ns >= 1 && ns <= kNrhs, HM_EINVAL, "samples per gradient must be in [1, 16]");
    HM_REQUIRE(B && X, HM_EINVAL, "null sample pointer");
    HM_REQUIRE(ldb >= 3 * op.ne && ldx >= 3 * op.ne, HM_EINVAL, "leading dimension below 3N");
    learned_prepare(op, L.K, s);
    const LearnedPairs& lp = op.lp;
    const int64_t P = lp.P, nd = 3 * op.ne;
    const int H = L.H;
    // workspace: a1, a2, d2, d1 [P][H], out, dO, Wb [P][9] (float);
    // rho [ns][nd], reduction partials (every layer's weight gradient and
    // the column sums), sample weights (double)
    const size_t nfl = (size_t)P * (4 * H + 3 * kOut);
    const size_t npart = std::max<size_t>(wgrad_partial_size(P, H), (size_t)kNrhs * kSumsqBlocks);
    const bool leaf = L.base == HM_PC_LEAF;
    const size_t ndb = (size_t)(leaf ? 2 : 1) * ns * nd + npart + kNrhs;
    const size_t need = nfl * sizeof(float) + 256 + ndb * sizeof(double);
    if (L.ws.bytes() < need) L.ws.alloc(need);
    float* a1 = L.ws.as<float>();
    float* a2 = a1 + (size_t)P * H;
    float* d2 = a2 + (size_t)P * H;
    float* d1 = d2 + (size_t)P * H;
    float* out = d1 + (size_t)P * H;
    float* dO = out + (size_t)P * kOut;
    float* Wb = dO + (size_t)P * kOut;
    double* rho = reinterpret_cast<double*>(round_up((int64_t)(uintptr_t)(Wb + (size_t)P * kOut), (int64_t)256));
    double* part = rho + (size_t)ns * nd;
    double* wdev = part + npart;
    double* zb = leaf ? wdev + kNrhs : nullptr;  // leaf block-Jacobi times the samples

    forward(L, P, lp.feat.as<float>(), a1, a2, out, s);
    hipLaunchKernelGGL(k_out_to_blocks, dim3(g1(P)), dim3(256), 0, s, P, out, lp.scale.as<double>(), Wb);
    if (leaf) {
        leaf_pc_prepare(op, s);
        leaf_pc_apply(op, ns, B, ldb, zb, nd, s);
    }
    hipLaunchKernelGGL(k_apply_learned, dim3(g1(op.ne)), dim3(256), 0, s, op.ne, ns, B, ldb, rho, nd,
                       leaf ? nullptr : op.d_pc_block.as<double>(), zb, nd, lp.off.as<int64_t>(),
                       lp.pf.as<int32_t>(), Wb, X, ldx);
    HM_CHECK_HIP(hipGetLastError());
    const std::vector<double> xn = sumsq(ns, nd, X, ldx, part, npart, s);
    const std::vector<double> rn = sumsq(ns, nd, rho, nd, part, npart, s);
    double loss = 0.0;
    std::vector<double> w(ns);
    for (int c = 0; c < ns; ++c) {
        HM_REQUIRE(xn[c] > 0.0, HM_EINVAL, "a training solution is zero");
        loss += rn[c] / (ns * xn[c]);
        w[c] = 2.0 / (ns * xn[c]);
    }
    HM_CHECK_HIP(hipMemcpyAsync(wdev, w.data(), ns * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_pair_grad, dim3(g1(P)), dim3(256), 0, s, P, lp.pe.as<int32_t>(), lp.pf.as<int32_t>(),
                       lp.scale.as<double>(), ns, rho, nd, B, ldb, wdev, dO);
    backward(L, P, lp.feat.as<float>(), a1, a2, dO, d2, d1, part, npart, s);
    HM_CHECK_HIP(hipStreamSynchronize(s));
    return loss;
}

void learned_train(Learned& L, Op& op, int n, const double* B, int64_t ldb, const double* X, int64_t ldx, int steps,
                   int batch, double lr, double* hist, hipStream_t s)
{
    HM_REQUIRE(n >= 1 && steps >= 1, HM_EINVAL, "sample and step counts must be positive");
    HM_REQUIRE(batch >= 1 && batch <= kNrhs, HM_EINVAL, "batch must be in [1, 16]");
    HM_REQUIRE(lr > 0.0 && std::isfinite(lr), HM_EINVAL, "learning rate must be positive");
    HM_REQUIRE(B && X, HM_EINVAL, "null sample pointer");
    HM_REQUIRE(ldb >= 3 * op.ne && ldx >= 3 * op.ne, HM_EINVAL, "leading dimension below 3N");
    const int64_t nd = 3 * op.ne;
    batch = std::min(batch, n);
    DevBuf bb((size_t)batch * nd * sizeof(double)), xb((size_t)batch * nd * sizeof(double));
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int it = 0; it < steps; ++it) {
        // mini-batch: the next `batch` samples, cyclically
        for (int c = 0; c < batch; ++c) {
            const int64_t col = ((int64_t)it * batch + c) % n;
            HM_CHECK_HIP(hipMemcpyAsync(bb.as<double>() + (size_t)c * nd, B + (size_t)col * ldb, nd * sizeof(double),
                                        hipMemcpyDeviceToDevice, s));
            HM_CHECK_HIP(hipMemcpyAsync(xb.as<double>() + (size_t)c * nd, X + (size_t)col * ldx, nd * sizeof(double),
                                        hipMemcpyDeviceToDevice, s));
        }
        const double loss = learned_loss_grad(L, op, batch, bb.as<double>(), nd, xb.as<double>(), nd, s);
        if (hist) hist[it] = loss;
        L.step++;
        const float c1 = 1.f - std::pow(b1, (float)L.step), c2 = 1.f - std::pow(b2, (float)L.step);
        hipLaunchKernelGGL(k_adam, dim3(g1(L.n)), dim3(256), 0, s, L.n, L.params.as<float>(), L.grad.as<float>(),
                           L.m.as<float>(), L.v.as<float>(), (float)lr, b1, b2, eps, c1, c2);
        HM_CHECK_HIP(hipGetLastError());
    }
    HM_CHECK_HIP(hipStreamSynchronize(s));
    op.lp.attached = false;  // the parameters moved on: predict again before use
}

void learned_attach(Op& op, const Learned& L, hipStream_t s)
{
    learned_prepare(op, L.K, s);
    if (L.base == HM_PC_LEAF) leaf_pc_prepare(op, s);
    LearnedPairs& lp = op.lp;
    lp.base = L.base;
    const int64_t P = lp.P;
    if (P > 0) {
        DevBuf act((size_t)P * (2 * L.H + kOut) * sizeof(float));
        float* a1 = act.as<float>();
        float* a2 = a1 + (size_t)P * L.H;
        float* out = a2 + (size_t)P * L.H;
        forward(L, P, lp.feat.as<float>(), a1, a2, out, s);
        hipLaunchKernelGGL(k_out_to_blocks, dim3(g1(P)), dim3(256), 0, s, P, out, lp.scale.as<double>(),
                           lp.W.as<float>());
        HM_CHECK_HIP(hipGetLastError());
        HM_CHECK_HIP(hipStreamSynchronize(s));
    }
    lp.attached = true;
}

void learned_apply(const Op& op, int nrhs, const double* r, int64_t ldr, double* z, int64_t ldz, hipStream_t s)
{
    const LearnedPairs& lp = op.lp;
    const bool leaf = lp.base == HM_PC_LEAF;
    if (leaf) leaf_pc_apply(op, nrhs, r, ldr, z, ldz, s);  // z = leaf block-Jacobi r, then the correction
    hipLaunchKernelGGL(k_apply_learned, dim3(g1(op.ne)), dim3(256), 0, s, op.ne, nrhs, r, ldr, z, ldz,
                       leaf ? nullptr : op.d_pc_block.as<double>(), leaf ? z : nullptr, ldz, lp.off.as<int64_t>(),
                       lp.pf.as<int32_t>(), lp.W.as<float>(), nullptr, (int64_t)0);
    HM_CHECK_HIP(hipGetLastError());
}

}  // namespace hm
