// Product entry point that allocates nothing: the workspace of the product
// lives in a fixed device array of the library instead of a per-stream block
// allocated on first use.  For callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops).
//
// Every call on one device uses the same array, which keeps what the last
// call left: the product zeroes the sections that must start at zero before
// it runs, and calls that overlap on one device (other streams, other
// threads) race on the array.
#include <mutex>

#include "hm_handles.hpp"

// each device holds its own copy of this array (allocated when the code
// object is loaded on it, kept until the process ends)
static __device__ __align__(256) unsigned char scratch[HM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of the current device's array, looked up once per device
// with that device current (the array's name is only a host stand-in)
void* scratch_address()
{
    int dev = 0;
    HM_CHECK_HIP(hipGetDevice(&dev));
    HM_REQUIRE(dev >= 0 && dev < kMaxDevices, HM_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HM_CHECK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        HM_REQUIRE(ptr != nullptr, HM_EDEVICE, "no device address for the scratch array");
        HM_REQUIRE(((uintptr_t)ptr & 255) == 0, HM_EINTERNAL, "scratch array not 256-byte aligned");
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" hm_status hm_operator_apply_noalloc(const hm_op* op, int nrhs, const double* d_X, int64_t ldx,
                                               double* d_Y, int64_t ldy, unsigned flags, void* hip_stream)
{
    return guarded([&] {
        HM_REQUIRE(op, HM_EINVAL, "op is null");
        HM_REQUIRE((flags & ~(HM_APPLY_REFERENCE | HM_APPLY_TANGENT | HM_APPLY_ACCUMULATE)) == 0, HM_EINVAL,
                   "unknown flag");
        const hm::Op& o = op->op;
        HM_REQUIRE(!(flags & HM_APPLY_REFERENCE) || o.ref || o.main.near_prec == HM_F64, HM_EINVAL,
                   "no FP64 reference copy (build with keep_f64_reference)");
        const hm::Variant& v = (flags & HM_APPLY_REFERENCE) ? o.ref_variant() : o.main;
        const size_t need = v.ws_layout().total;
        HM_REQUIRE(need <= (size_t)HM_NOALLOC_SCRATCH_BYTES, HM_EINVAL,
                   "operator needs " + std::to_string(need) + " bytes of product workspace; the no-allocation "
                   "scratch holds " + std::to_string((size_t)HM_NOALLOC_SCRATCH_BYTES) +
                   " (use hm_operator_apply)");
        hm::apply_in(o, v, scratch_address(), nrhs, d_X, ldx, d_Y, ldy, (flags & HM_APPLY_TANGENT) != 0,
                     (hipStream_t)hip_stream, (flags & HM_APPLY_ACCUMULATE) != 0);
    });
}
