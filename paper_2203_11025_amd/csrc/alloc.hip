// Device-memory allocation of the library's own workspaces, through a
// caller-registered allocator (helm_set_allocator) or hipMalloc / hipFree.
//
// Every workspace of a handle, an FGMRES solve, a network or the training
// triple generator comes from dev_malloc and goes back through dev_free.  A
// registered allocator receives the size at release as well, kept here per
// pointer.  Before any release through a registered allocator the device is
// synchronised: the library's kernels may still be reading the block on
// internal streams, and a caching allocator would hand it out again at once
// (hipFree itself waits for the device).
#include <mutex>
#include <unordered_map>

#include "helm_internal.h"

namespace helm {

namespace {

struct Registry {
    std::mutex mu;
    helm_alloc_fn alloc = nullptr;
    helm_free_fn release = nullptr;
    void *ctx = nullptr;
    // pointer -> its size and the release function (and context) of the
    // allocator it came from (null: hipMalloc), so a block goes back where it
    // came from even after the registration changes
    struct Block {
        size_t bytes;
        helm_free_fn release;
        void *ctx;
    };
    std::unordered_map<void *, Block> live;
};

Registry &reg()
{
    static Registry r;
    return r;
}

}  // namespace

hipError_t dev_malloc(void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 1;
    Registry &r = reg();
    helm_alloc_fn fn;
    helm_free_fn rel;
    void *ctx;
    {
        std::lock_guard<std::mutex> lk(r.mu);
        fn = r.alloc;
        rel = r.release;
        ctx = r.ctx;
    }
    void *q = nullptr;
    if (fn) {
        q = fn(bytes, ctx);
        if (!q) return hipErrorOutOfMemory;
    } else {
        hipError_t e = hipMalloc(&q, bytes);
        if (e != hipSuccess) return e;
    }
    std::lock_guard<std::mutex> lk(r.mu);
    r.live[q] = Registry::Block{bytes, fn ? rel : nullptr, ctx};
    *p = q;
    return hipSuccess;
}

hipError_t dev_free(void *p)
{
    if (!p) return hipSuccess;
    Registry &r = reg();
    Registry::Block blk{0, nullptr, nullptr};
    {
        std::lock_guard<std::mutex> lk(r.mu);
        auto it = r.live.find(p);
        if (it != r.live.end()) {
            blk = it->second;
            r.live.erase(it);
        }
    }
    if (!blk.release) return hipFree(p);
    hipError_t e = hipDeviceSynchronize();
    blk.release(p, blk.bytes, blk.ctx);
    return e;
}

size_t dev_live_bytes()
{
    Registry &r = reg();
    std::lock_guard<std::mutex> lk(r.mu);
    size_t s = 0;
    for (auto &kv : r.live) s += kv.second.bytes;
    return s;
}

}  // namespace helm

using namespace helm;

extern "C" int helm_set_allocator(helm_alloc_fn alloc, helm_free_fn release, void *ctx)
{
    if ((alloc == nullptr) != (release == nullptr)) {
        set_error("helm_set_allocator: give both functions, or neither to restore hipMalloc / hipFree");
        return HELM_E_INVALID;
    }
    Registry &r = reg();
    std::lock_guard<std::mutex> lk(r.mu);
    r.alloc = alloc;
    r.release = release;
    r.ctx = ctx;
    return HELM_OK;
}

extern "C" size_t helm_allocated_bytes(void) { return dev_live_bytes(); }
