// The opaque handles of the C ABI and the exception guard every extern "C"
// entry point runs its body in.
#pragma once

#include <new>
#include <string>

#include "hm_op.hpp"

struct hm_mesh {
    hm::Mesh m;
};
struct hm_op {
    hm::Op op;
};
struct hm_batch {
    hm::Batch* b = nullptr;
    ~hm_batch() { hm::batch_destroy(b); }
};
struct hm_flow {
    hm::Flow* f = nullptr;
    ~hm_flow() { hm::flow_destroy(f); }
};
struct hm_learned {
    hm::Learned net;
    hm_learned(int h, int k, uint64_t seed) : net(h, k, seed) {}
};

// Run f, turning every exception into a status code and the calling
// thread's last-error message.
template <class F>
static hm_status guarded(F&& f)
{
    try {
        hm::set_last_error("");
        f();
        return HM_OK;
    } catch (const hm::Error& e) {
        hm::set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        hm::set_last_error("host allocation failed");
        return HM_ENOMEM;
    } catch (const std::exception& e) {
        hm::set_last_error(e.what());
        return HM_EINTERNAL;
    } catch (...) {
        hm::set_last_error("unknown internal error");
        return HM_EINTERNAL;
    }
}
