// dmk_noalloc.hip -- dmk_residual_eval for callers that cannot allocate
// device memory (code under graph capture, tight serving loops, harnesses
// that forbid allocation).
//
// dmk_residual_eval needs a workspace for the strengths in the sorted order.
// This variant takes it from `scratch`, a file-scope device array of
// DMK_NOALLOC_WS_BYTES that every GPU the library runs on holds until the
// process ends.  The array's device address on the current device is looked
// up once per device (hipGetSymbolAddress, under a lock) on the first call on
// that device and kept; host code passes that address to the kernels, never
// the array's name.  Every call on one GPU shares that GPU's array: calls
// that overlap on one GPU (different streams, or host threads) race.  The
// workspace is fully written by the strength gather before the pair kernel
// reads it, so nothing in it has to start at zero.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dmk_internal.h"

static __device__ __align__(256) unsigned char scratch[DMK_NOALLOC_WS_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_lock;
void *g_scratch[MAX_DEVICES];  // device address of `scratch` per device, once looked up

// address of `scratch` on the current device
int scratch_on_current_device(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return DMK_EHIP;
    if (dev < 0 || dev >= MAX_DEVICES) return DMK_EUNSUPPORTED;
    std::lock_guard<std::mutex> hold(g_lock);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return DMK_EHIP;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return DMK_OK;
}

}  // namespace

extern "C" int dmk_residual_eval_noalloc(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec,
                                         double sigma, double rc, const double *rho, double *u, hipStream_t stream)
{
    if (!grid || !bins) return DMK_EINVAL;
    if (kernel < 0 || kernel > 3) return DMK_EUNSUPPORTED;
    const size_t need = dmk_residual_ws_bytes(grid, bins, kernel, prec, 0);
    if (need == 0) return DMK_EINVAL;
    if (need > (size_t)DMK_NOALLOC_WS_BYTES) return DMK_ESIZE;
    void *ws = nullptr;
    const int st = scratch_on_current_device(&ws);
    if (st != DMK_OK) return st;
    return dmk_residual_eval(grid, bins, kernel, prec, sigma, rc, rho, u, ws, (size_t)DMK_NOALLOC_WS_BYTES, stream);
}
