// Device workspace blocks and the process-wide default allocator.
#include "devmem.h"

#include <cstdint>
#include <mutex>

namespace tph {

namespace {
std::mutex g_alloc_mu;
Allocator g_default;
}  // namespace

Allocator default_allocator() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_default;
}

void set_default_allocator(const Allocator& a) {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_default = a;
}

hipError_t DeviceArena::alloc(void** p, size_t bytes, std::string* what) {
    *p = nullptr;
    if (bytes == 0) bytes = 1;
    if (a.alloc) {
        void* q = a.alloc(bytes, a.ctx);
        if (!q) {
            if (what) *what = "the caller's allocator returned NULL for " + std::to_string(bytes) + " bytes";
            return hipErrorOutOfMemory;
        }
        if (reinterpret_cast<uintptr_t>(q) % 256 != 0) {
            a.free(q, a.ctx);
            if (what) *what = "the caller's allocator returned a block that is not 256-byte aligned";
            return hipErrorInvalidValue;
        }
        blocks_.push_back(Block{q, a});
        *p = q;
        return hipSuccess;
    }
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();   // a failed allocation must not surface at a later launch check
        if (what) *what = "device allocation of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e);
        return e;
    }
    blocks_.push_back(Block{q, Allocator{}});
    *p = q;
    return hipSuccess;
}

void DeviceArena::release_all() {
    for (auto it = blocks_.rbegin(); it != blocks_.rend(); ++it) {
        if (it->a.free) it->a.free(it->p, it->a.ctx);
        else (void)hipFree(it->p);
    }
    blocks_.clear();
}

}  // namespace tph
