// Allocation-free padded strip solve, for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
// strip solver's workspace lives in a file-scope device array of fixed size instead of a
// buffer of the handle; the strip factors themselves were allocated by helm_factor.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <string>

#include "helm_internal.hpp"

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;   // 64 MiB per device, held until exit

// In host code `scratch` is a host-side stand-in, never a device address: it is passed to
// no kernel and no copy.  Its address on a device comes from hipGetSymbolAddress, taken once
// per device with that device current, and kept in g_scratch_ptr.
__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int SCRATCH_MAX_DEV = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEV] = {};

hipError_t scratch_on(int dev, void** out) {
    *out = nullptr;
    if (dev < 0 || dev >= SCRATCH_MAX_DEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// the workspace keeps the previous call's contents: the used part is cleared by a kernel
// (not a memset node, so the call may be captured into a graph)
__global__ void k_zero_words(uint4* p, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace

extern "C" helm_status helm_strip_solve_noalloc(helm_t H, int strip, int nrhs, const void* r, void* x) {
    if (!H) return HELM_EINVAL;
    if (!helm::handle_factored(H))
        return helm::handle_fail(H, HELM_ESTATE, "helm_strip_solve_noalloc before helm_factor");
    if (strip < 0 || strip >= helm::handle_strips(H) || nrhs < 1 || !r || !x)
        return helm::handle_fail(H, HELM_EINVAL, "helm_strip_solve_noalloc: bad arguments");
    const size_t need = helm::strip_workspace_bytes(H, nrhs);
    if (need > SCRATCH_BYTES)
        return helm::handle_fail(H, HELM_EINVAL,
                                 "helm_strip_solve_noalloc: " + std::to_string(nrhs) + " right-hand sides need " +
                                     std::to_string(need) + " bytes of workspace, the static workspace holds " +
                                     std::to_string(SCRATCH_BYTES) + " (solve fewer right-hand sides per call)");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return helm::handle_fail(H, HELM_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (cur != helm::handle_device(H))
        return helm::handle_fail(H, HELM_EINVAL, "helm_strip_solve_noalloc: the handle's device must be current");
    void* ws = nullptr;
    e = scratch_on(cur, &ws);
    if (e != hipSuccess)
        return helm::handle_fail(H, HELM_EHIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    const size_t words = (need + sizeof(uint4) - 1) / sizeof(uint4);
    const unsigned blocks = (unsigned)std::min<size_t>((words + 255) / 256, 2048);
    hipLaunchKernelGGL(k_zero_words, dim3(blocks), dim3(256), 0, helm::handle_stream(H), static_cast<uint4*>(ws),
                       words);
    e = hipGetLastError();
    if (e != hipSuccess) return helm::handle_fail(H, HELM_EHIP, std::string("workspace clear: ") + hipGetErrorString(e));
    return helm::strip_solve_into(H, strip, nrhs, r, x, ws);
}
