// skfab_solve_noalloc: skfab_solve for callers that cannot allocate device memory.
//
// The workspace of the solve (basis, SELL copy of A, sketches, small-problem
// buffers) lives in `scratch`, a file-scope device array of SKFAB_NOALLOC_WS_BYTES
// bytes.  The code object holds one copy per device it is loaded on, for the life
// of the process.  In host code the name `scratch` is only a stand-in, not a device
// address: skfab_create (with its device current) looks up the device address once
// per device with hipGetSymbolAddress and keeps it in `g_scratch`; the entry point
// hands that address to the ordinary solve as its workspace.  The solve clears what
// it needs (control block, Hessenberg matrix, partial sums) itself, so the array's
// contents left by an earlier call do not matter; two calls that overlap on one
// device share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/skfab.h"

static __device__ __align__(256) unsigned char scratch[SKFAB_NOALLOC_WS_BYTES];

namespace skfab {

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch[NOALLOC_MAX_DEVICES] = {};  // device address of `scratch`, per device
}  // namespace

// Called by skfab_create with `device` current.
skfab_status noalloc_init_device(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return SKFAB_ERR_ARG;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch[device]) return SKFAB_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SKFAB_ERR_HIP;
    g_scratch[device] = ptr;
    return SKFAB_OK;
}

int ctx_device(const skfab_ctx* ctx);

}  // namespace skfab

extern "C" skfab_status skfab_solve_noalloc(skfab_ctx* ctx, const skfab_csr* A, const double* b, double* x,
                                            const skfab_params* p, skfab_info* info) {
    if (!ctx || !A || !p || !b || !x) return SKFAB_ERR_ARG;
    size_t need = 0;
    const skfab_status v = skfab_workspace_bytes(A, p, 1, &need);
    if (v != SKFAB_OK) return v;
    if (need > (size_t)SKFAB_NOALLOC_WS_BYTES) return SKFAB_ERR_TOO_LARGE;
    const int dev = skfab::ctx_device(ctx);
    void* ws = nullptr;
    {
        std::lock_guard<std::mutex> lock(skfab::g_mu);
        if (dev >= 0 && dev < skfab::NOALLOC_MAX_DEVICES) ws = skfab::g_scratch[dev];
    }
    if (!ws) return SKFAB_ERR_HIP;  // skfab_create could not resolve the array on this device
    return skfab_solve(ctx, A, b, A->n, 1, x, A->n, p, ws, (size_t)SKFAB_NOALLOC_WS_BYTES, info);
}
