// Device workspace of one library handle (solver, batch, marker set).
//
// Every block is obtained from an allocator: the caller's (tph_set_allocator)
// or hipMalloc / hipFree.  Each block remembers the allocator that made it,
// so a handle whose allocator changes later still frees every block with the
// function that allocated it.  The process-wide default allocator is read
// when a handle is created.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>
#include <vector>

namespace tph {

struct Allocator {
    void* (*alloc)(size_t bytes, void* ctx) = nullptr;   // null: hipMalloc / hipFree
    void (*free)(void* ptr, void* ctx) = nullptr;
    void* ctx = nullptr;
};

// the process-wide default (thread-safe copy)
Allocator default_allocator();
void set_default_allocator(const Allocator& a);

class DeviceArena {
public:
    Allocator a;                      // used for blocks allocated from now on

    // *p = a block of `bytes` (> 0) device bytes, 256-byte aligned.  Returns
    // hipSuccess, hipErrorOutOfMemory (the allocator returned NULL, or
    // hipMalloc ran out of memory; *p = nullptr) or another HIP error;
    // `what` receives a message on failure.
    hipError_t alloc(void** p, size_t bytes, std::string* what);
    // free every block (the caller has synchronised the streams that use them)
    void release_all();
    bool empty() const { return blocks_.empty(); }
    size_t blocks() const { return blocks_.size(); }
    ~DeviceArena() { release_all(); }

private:
    struct Block {
        void* p;
        Allocator a;
    };
    std::vector<Block> blocks_;
};

}  // namespace tph
