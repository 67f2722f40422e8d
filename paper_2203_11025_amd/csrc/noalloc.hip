// helm_sl_vcycle_noalloc: the SL V-cycle (Algorithm 1) on a workspace that
// lives in a fixed device array of this library, for callers that cannot
// allocate device memory (code under graph capture, tight serving loops).
//
// The restricted right-hand sides, the level corrections and the partial
// sums of the coarsest-level GEMM are carved from `scratch`, a file-scope
// device array of VC_SCRATCH_BYTES.  Each device holds its own copy of the
// array; its device address is looked up once per device with
// hipGetSymbolAddress, with that device current, the first time the entry
// point runs on it, and only that address is ever handed to kernels.
// Calls on one device share the array: calls that overlap in time on one
// device (different streams or threads) race.  No part of the workspace
// needs clearing: every kernel of the cycle writes what it later reads.
#include <mutex>

#include "handle.h"

namespace helm {

namespace {

constexpr size_t VC_SCRATCH_BYTES = 64ull << 20;  // 64 MiB per device
constexpr size_t VC_SCRATCH_ELEMS = VC_SCRATCH_BYTES / sizeof(float2);

__device__ __align__(256) float2 scratch[VC_SCRATCH_ELEMS];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
float2 *g_ptr[MAX_DEVICES] = {};

// device address of this device's copy of `scratch` (looked up once per device)
int scratch_ptr(float2 **out)
{
    int dev = 0;
    HELM_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) {
        set_error("helm_sl_vcycle_noalloc: device index out of range");
        return HELM_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("helm_sl_vcycle_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
            return HELM_E_HIP;
        }
        g_ptr[dev] = (float2 *)p;
    }
    *out = g_ptr[dev];
    return HELM_OK;
}

}  // namespace

}  // namespace helm

using namespace helm;

extern "C" size_t helm_sl_vcycle_noalloc_max_bytes(void) { return VC_SCRATCH_BYTES; }

extern "C" size_t helm_sl_vcycle_noalloc_bytes(const helm_handle *h, int nrhs)
{
    if (!h || nrhs <= 0) return 0;
    return vcycle_ws_elems(h, nrhs) * sizeof(float2);
}

extern "C" int helm_sl_vcycle_noalloc(helm_handle *h, const float *f, float *v, int nrhs, void *stream)
{
    if (!h || nrhs < 0 || (nrhs > 0 && (!f || !v))) {
        set_error("helm_sl_vcycle_noalloc: invalid argument");
        return HELM_E_INVALID;
    }
    if (nrhs == 0) return HELM_OK;
    const size_t need = vcycle_ws_elems(h, nrhs);
    if (need > VC_SCRATCH_ELEMS) {
        set_error("helm_sl_vcycle_noalloc: workspace of " + std::to_string(need * sizeof(float2)) +
                  " bytes exceeds the fixed " + std::to_string(VC_SCRATCH_BYTES) +
                  " bytes; use fewer right-hand sides per call or helm_sl_vcycle");
        return HELM_E_INVALID;
    }
    float2 *base = nullptr;
    int rc = scratch_ptr(&base);
    if (rc) return rc;
    VcycleWs ws;
    vcycle_carve(h, nrhs, base, ws);
    const size_t N = (size_t)h->n * h->n;
    prof_suspend(true);  // the timing hook creates events; not here
    vcycle_with(h, ws, (const float2 *)f, N, (float2 *)v, N, nrhs, nullptr, (hipStream_t)stream);
    prof_suspend(false);
    HELM_HIP_CHECK(hipGetLastError());
    return HELM_OK;
}
