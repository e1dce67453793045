// bs_residual_noalloc: the residual and its per-patch norms with the per-tile
// partial sums in a file-scope device array instead of the patch set's
// allocation, for callers that cannot allocate device memory.
#include <mutex>

#include "patchset.h"
#include "relax.h"

namespace bs {

namespace {

constexpr int kStaticTiles = 1 << 16;   // 512 KiB of partial sums per device
constexpr int kMaxDevices = 64;

// Device address of `scratch` per device, found once per device with that
// device current (each device holds its own copy of the array).
static __device__ __align__(256) double scratch[kStaticTiles];

std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};

bs_status scratch_ptr(int dev, double **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(BS_ERR_UNSUPPORTED, "bs_residual_noalloc: device %d", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_ptr[dev];
    return BS_OK;
}

}  // namespace

}  // namespace bs

using namespace bs;

extern "C" {

bs_status bs_residual_noalloc(const bs_patchset *ps, const double *u, const double *f, double *r, double *rnorm2,
                              hipStream_t stream)
{
    if (!r && !rnorm2) return fail(BS_ERR_INVALID, "bs_residual_noalloc: r and rnorm2 are both null");
    if (!ps || !u || !f) return fail(BS_ERR_INVALID, "bs_residual_noalloc: null patch set, u or f");
    if (ps->nrtiles > kStaticTiles)
        return fail(BS_ERR_UNSUPPORTED, "bs_residual_noalloc: the patch set has %d residual tiles, the static scratch "
                                        "holds %d", ps->nrtiles, kStaticTiles);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != ps->device)
        return fail(BS_ERR_INVALID, "bs_residual_noalloc: device %d is current, the patch set is on %d", dev,
                    ps->device);
    double *partial = nullptr;
    bs_status st = scratch_ptr(dev, &partial);
    if (st != BS_OK) return st;
    ResidArgs a{};
    a.u = u;
    a.f = f;
    a.r = r;
    a.partial = rnorm2 ? partial : nullptr;   // every tile writes its own partial: nothing to clear
    a.pd = static_cast<const PatchDesc *>(ps->desc_d.p);
    a.tiles = static_cast<const ResidTile *>(ps->rtile_d.p);
    if ((e = launch_residual(a, ps->nrtiles, stream)) != hipSuccess) return hip_fail(e, "residual kernel");
    if (rnorm2) {
        e = launch_residual_final(partial, static_cast<const int32_t *>(ps->rtile_first_d.p), ps->npatch, rnorm2,
                                  stream);
        if (e != hipSuccess) return hip_fail(e, "residual reduction kernel");
    }
    return BS_OK;
}

}  // extern "C"
