// Internal structures of the hmdd library (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hmdd.h"
#include "hm_coef.hpp"

namespace hm {

// ------------------------------------------------------------------
// errors
// ------------------------------------------------------------------
struct Error : std::runtime_error {
    hm_status code;
    Error(hm_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define HM_CHECK_HIP(expr)                                                                             \
    do {                                                                                               \
        hipError_t _e = (expr);                                                                        \
        if (_e != hipSuccess)                                                                          \
            throw ::hm::Error(_e == hipErrorOutOfMemory ? HM_ENOMEM : HM_EDEVICE,                       \
                              std::string(#expr) + ": " + hipGetErrorString(_e));                      \
    } while (0)

#define HM_REQUIRE(cond, code, msg)                                                                    \
    do {                                                                                               \
        if (!(cond)) throw ::hm::Error(code, msg);                                                     \
    } while (0)

// ------------------------------------------------------------------
// device memory owned by a handle
// ------------------------------------------------------------------
class DevBuf {
  public:
    DevBuf() = default;
    explicit DevBuf(size_t bytes) { alloc(bytes); }
    ~DevBuf() { release(); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p_(o.p_), n_(o.n_) { o.p_ = nullptr; o.n_ = 0; }
    DevBuf& operator=(DevBuf&& o) noexcept
    {
        if (this != &o) {
            release();
            p_ = o.p_;
            n_ = o.n_;
            o.p_ = nullptr;
            o.n_ = 0;
        }
        return *this;
    }
    void alloc(size_t bytes)
    {
        release();
        if (bytes == 0) return;
        HM_CHECK_HIP(hipMalloc(&p_, bytes));
        n_ = bytes;
    }
    void release()
    {
        if (p_) (void)hipFree(p_);
        p_ = nullptr;
        n_ = 0;
    }
    template <class T>
    T* as() const { return static_cast<T*>(p_); }
    void* get() const { return p_; }
    size_t bytes() const { return n_; }

  private:
    void* p_ = nullptr;
    size_t n_ = 0;
};

template <class T>
inline void upload(DevBuf& b, const std::vector<T>& v, hipStream_t s)
{
    b.alloc(v.size() * sizeof(T));
    if (!v.empty()) HM_CHECK_HIP(hipMemcpyAsync(b.get(), v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// ------------------------------------------------------------------
// mesh (host)
// ------------------------------------------------------------------
struct Mesh {
    int nvpe = 0;
    int64_t ne = 0, nv = 0;
    std::vector<double> xyz;
    std::vector<int64_t> conn;
    std::vector<double> cent, frame, area;   // per element: [3], [9], [1]
    std::vector<ElemGeo> geo;                // per element, original order
    DevBuf d_geo;                            // uploaded on first device use
    int d_geo_device = -1;
};

void mesh_validate_and_frame(Mesh& m);

// ------------------------------------------------------------------
// cluster tree and block tree (host)
// ------------------------------------------------------------------
struct Cluster {
    int64_t begin = 0, end = 0;   // positions in cluster order
    double bmin[3], bmax[3];      // bounding box of element vertices
    int child[2] = {-1, -1};
    int level = 0;
    int leaf_id = -1;             // index among leaves (leaves only)
    int first_leaf = 0, n_leaves = 0;  // leaves under this node (contiguous)
    // all elements lie in one plane n . x = d (within the plan's tolerance)
    bool planar = false;
    double pn[3] = {0, 0, 0}, pd = 0.0;
    bool is_leaf() const { return child[0] < 0; }
    int64_t size() const { return end - begin; }
};

struct Plan {
    int leaf_size = 64;
    double eta = 2.0;
    std::vector<int64_t> perm;        // cluster position -> element id
    std::vector<int64_t> iperm;       // element id -> cluster position
    std::vector<Cluster> nodes;       // nodes[0] = root
    std::vector<int> leaves;          // node id of each leaf, in position order
    std::vector<std::pair<int, int>> dense;    // (target leaf node, source leaf node)
    std::vector<std::pair<int, int>> lowrank;  // (target node, source node)
    int depth = 0;
    double plane_tol = 0.0;           // distance below which points count as in a plane
};

Plan make_plan(const Mesh& m, int leaf_size, double eta);
// blocks replacing an admissible pair whose compression failed (children, same rules)
void split_block(Plan& p, int t, int s, std::vector<std::pair<int, int>>& lowrank,
                 std::vector<std::pair<int, int>>& dense);
void sort_blocks(Plan& p);
// Both clusters lie in one common plane.  Between elements of one plane
// the normal DD component and the two shear components do not interact
// (the planar-crack operator decouples opening from slip), so such a block
// is stored as a shear part and a normal part.
bool coplanar_pair(const Plan& p, int t, int s);

// ------------------------------------------------------------------
// panel layout shared by pack and apply kernels
// ------------------------------------------------------------------
// A panel is a row-major M x K matrix stored in "MFMA fragment" order so
// that one wavefront streams it with 16-byte per-lane loads.  A granule is
// 16 bytes (w = 2 doubles, 4 floats or 8 bf16); a k-step covers 4 granules
// (Kstep = 4 w columns).  Storage is k-step major: k-step ks holds all M
// rows, as row tiles of 16 (rr = min(16, M - 16 rt) rows) times gg =
// min(4, Gr - 4 ks) granules (Gr = ceil(K / w)) in [g][i] order, so lane
// (g, i) of a wavefront owns granule g of row i and one k-step of all row
// tiles is contiguous.  Padding is only to the granule: the panel occupies
// M * Gr granules.
__host__ __device__ inline int64_t panel_granules(int K, int w) { return (K + w - 1) / w; }
__host__ __device__ inline int64_t panel_elems(int M, int K, int w) { return (int64_t)M * panel_granules(K, w) * w; }

__host__ __device__ inline int64_t panel_offset(int M, int K, int w, int row, int col)
{
    int64_t Gr = panel_granules(K, w);
    int kstep = 4 * w;
    int ks = col / kstep;
    int g = (col % kstep) / w;
    int t = col % w;
    int gg = (int)(Gr - 4 * ks < 4 ? Gr - 4 * ks : 4);
    int rt = row >> 4, i = row & 15;
    int rr = M - 16 * rt < 16 ? M - 16 * rt : 16;
    int64_t gran = (int64_t)ks * M * 4 + (int64_t)rt * 16 * gg + (int64_t)g * rr + i;
    return gran * w + t;
}

// In-vector chunk ("B fragment") for 16 right-hand sides: dof q, rhs c.
// Lane l = g*16 + c of k-step ks reads 16 bytes at element (ks*64 + l) * w.
__host__ __device__ inline int64_t bfrag_offset(int w, int q, int c)
{
    int kstep = 4 * w;
    int ks = q / kstep;
    int g = (q % kstep) / w;
    int t = q % w;
    return ((int64_t)(ks * 4 + g) * 16 + c) * w + t;
}

constexpr int kChunkAlign = 32;   // dofs; multiple of every k-step

__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// In-vector chunk of a leaf of m elements: a shear section (s1, s2 of each
// element, element-major) then a normal section (n of each element), each
// starting on a k-step boundary.
__host__ __device__ inline int64_t chunk_n_off(int64_t m) { return round_up(2 * m, kChunkAlign); }
__host__ __device__ inline int64_t chunk_len(int64_t m) { return chunk_n_off(m) + round_up(m, kChunkAlign); }
constexpr int kNrhs = 16;         // right-hand sides per fragment

inline int prec_w(int prec) { return prec == HM_F64 ? 2 : (prec == HM_F32 ? 4 : 8); }
inline int prec_bytes(int prec) { return prec == HM_F64 ? 8 : (prec == HM_F32 ? 4 : 2); }

// descriptors consumed by the apply kernels
struct PanelRef {
    int64_t a_off;    // panel start (elements of its precision)
    int64_t b_off;    // in-vector chunk start (elements of the in-vector buffer)
    int32_t rows, cols;
    int32_t far;      // 0: near-field buffer / X, 1: far-field buffer / T
    int32_t pad;
};

// Tasks cover a window of row tiles of their panels (tiles r0 .. r0 + R - 1),
// so every launch runs a small accumulator set; the windows of one panel set
// re-read its in-vector chunks.  Phase-A windows hold at most kTileWindow
// tiles (a stack of up to 64 rows in one window).
constexpr int kTileWindow = 4;
// phase-B windows may be taller (whole 128-row shear sections): each unit's
// in-vector load then feeds up to eight row tiles; lists whose windows stay
// within kTileWindow tiles run a build with fewer registers
constexpr int kTileWindowB = 8;
__host__ __device__ inline int window_tiles(int rows, int r0)
{
    const int t = (rows + 15) / 16 - r0;
    return t < kTileWindow ? t : kTileWindow;
}

// Contiguous task ranges of the 8 XCDs (workgroups are dealt to the XCDs
// round-robin): XCD x runs tasks begin[x] .. begin[x + 1] - 1, cut so that
// the ranges carry about equal loads, longest task first inside a range.
struct XcdSplit {
    int32_t begin[9];
};

// Claim counters of the phase kernels' work queues: one per XCD range and
// phase (8 for phase A, then 8 for phase B), each on its own 256-byte line.
// The gather kernel that opens every product sets them to zero.
constexpr int kQueueStride = 64;                 // ints between counters
constexpr int kQueueInts = 16 * kQueueStride;

struct TaskB {        // one row window of one section of a target leaf
    int64_t y_off;    // output rows start in Y (section start)
    int32_t rows;     // rows of the section (= rows of each of its panels)
    int32_t item_begin, n_items;
    int32_t op;       // operator index into the base-pointer table
    int32_t r0;       // first row tile of the window
    int32_t nt;       // row tiles of the window (1 .. kTileWindowB)
};

// Phase A works on stacked V^T panels: the factorisations that share a
// source cluster (and carry the same sections) have their V^T sub-panels of
// each source leaf stored as one panel of sum-of-ranks rows, so one load of
// an in-vector k-step feeds every row tile of the window.
struct TaskA {        // one row window of a stacked panel set: T partial = sum V^T X
    int64_t out_off;  // partial slot start (elements, [rows_pad][16]) when not direct
    int32_t rows;     // stacked rows (sum of the members' ranks)
    int32_t item_begin, n_items;
    int32_t direct;   // 1: the task covers every source leaf and writes the members' T chunks
    int32_t op;
    int32_t r0;       // first row tile of the window
    int32_t mem_begin, n_mem;  // members meeting the window (direct tasks)
};

struct MemberT {      // one factorisation inside a stacked panel
    int64_t t_off;    // its T fragment chunk (elements)
    int32_t lo;       // its first stacked row
    int32_t rows;     // its rank
};

struct ReduceDesc {   // T_b = sum of partial slots
    int64_t slot_begin;   // member's first row in the first partial slot (elements)
    int64_t t_off;        // T fragment chunk start (elements)
    int32_t n_slots, rank;
    int32_t op;
    int32_t slot_stride;  // elements between consecutive slots of the stack
};

// Device buffers of one operator (one precision variant), looked up by the
// op index of a task so that several operators can share one launch.
struct Bases {
    const void* nearA;   // dense-leaf panels
    const void* farA;    // U slices and V^T sub-panels
    void* xnear;         // X chunks, near precision
    void* xfhi;          // X chunks read by phase A (far precision, or xnear)
    void* xflo;          // BF16 lo part or null
    void* thi;           // T chunks
    void* tlo;
    void* tpart;         // phase-A partial slots (accumulation precision)
    void* y;             // phase-B output rows (accumulation precision)
};

// One diagonal leaf block of the leaf block-Jacobi preconditioner.
struct LeafPc {
    int64_t off;      // block start in the block store (doubles; 9 m^2 per leaf)
    int64_t begin;    // first cluster position of the leaf
    int32_t m, pad;   // elements
};
constexpr int kLeafDofMax = 192;  // 3 x the largest leaf (64 elements)

// One leaf's in-vector chunk: where it starts and which elements it holds.
struct LeafIo {
    int64_t xoff;     // chunk start (padded dofs)
    int64_t begin;    // first cluster position of the leaf
    int32_t m, pad;   // elements
};

// One operator's share of the gather and scatter of a product (one
// workgroup per leaf: global leaf index leaf0 + l).
struct Segment {
    int64_t ne, ldx, ldy;
    const double* X;
    double* Y;
    const int64_t* perm;    // cluster position -> element
    const LeafIo* leaves;   // [nleaf]
    int32_t nleaf, leaf0;
    const double* self;     // FP64 self blocks or null
    const double* D;        // tangent blocks or null
    const uint8_t* mask;    // active mask or null
    int32_t op;
    int32_t tangent;
    int32_t accumulate;     // 1: Y += result
    int32_t pad;
};

}  // namespace hm
