// Streaming ceiling of the device for the sweeps' access volume: c = a + b
// over n doubles (two reads and one write per element, the 24 bytes per cell
// that a line sweep must move).  It bounds what any sweep kernel can reach on
// the same buffers, so the bench reports the sweeps against it beside the
// published HBM peak.  mode 1 reads b with nontemporal loads (the Jacobi
// sweeps read f that way on data beyond the Infinity Cache).
#include "bs_internal.h"

namespace bs {

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeVec = 4;   // double2 loads per operand per thread

template <int MODE>
__global__ void __launch_bounds__(kProbeThreads) k_triad(const double2 *__restrict__ a, const double2 *__restrict__ b,
                                                         double2 *__restrict__ c, int64_t n2)
{
    const int64_t base = static_cast<int64_t>(xcd_block(blockIdx.x, gridDim.x)) * (kProbeThreads * kProbeVec) +
                         threadIdx.x;
    double2 x[kProbeVec], y[kProbeVec];
#pragma unroll
    for (int v = 0; v < kProbeVec; ++v) {
        const int64_t i = base + v * kProbeThreads;
        const int64_t ic = i < n2 ? i : n2 - 1;
        x[v] = a[ic];
        if constexpr (MODE == 1) {
            y[v].x = __builtin_nontemporal_load(&b[ic].x);
            y[v].y = __builtin_nontemporal_load(&b[ic].y);
        } else {
            y[v] = b[ic];
        }
    }
#pragma unroll
    for (int v = 0; v < kProbeVec; ++v) {
        const int64_t i = base + v * kProbeThreads;
        if (i < n2) c[i] = make_double2(x[v].x + y[v].x, x[v].y + y[v].y);
    }
}

}  // namespace

}  // namespace bs

// Host-side hook (not part of the public header): c[0..n) = a + b, n even,
// 16-byte aligned buffers; mode 0 plain loads, 1 nontemporal loads of b.
extern "C" int bsi_stream_triad(const double *a, const double *b, double *c, int64_t n, int mode, hipStream_t s)
{
    using namespace bs;
    if (!a || !b || !c || n < 2 || (n & 1) || mode < 0 || mode > 1) return 1;
    if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(c)) & 15)
        return 1;
    const int64_t n2 = n / 2;
    const int64_t per = static_cast<int64_t>(kProbeThreads) * kProbeVec;
    const int64_t grid = (n2 + per - 1) / per;
    if (grid > INT32_MAX) return 1;
    const double2 *a2 = reinterpret_cast<const double2 *>(a), *b2 = reinterpret_cast<const double2 *>(b);
    double2 *c2 = reinterpret_cast<double2 *>(c);
    if (mode == 1)
        hipLaunchKernelGGL(k_triad<1>, dim3(static_cast<unsigned>(grid)), dim3(kProbeThreads), 0, s, a2, b2, c2, n2);
    else
        hipLaunchKernelGGL(k_triad<0>, dim3(static_cast<unsigned>(grid)), dim3(kProbeThreads), 0, s, a2, b2, c2, n2);
    return hipGetLastError() == hipSuccess ? 0 : 4;
}
