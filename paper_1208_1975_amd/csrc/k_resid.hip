// Residual r = h^2 f - A u (eq. stencil3d7 with axis weights) and its
// per-patch 2-norm^2, reduced in a fixed order (bit-reproducible); plus the
// copies the Jacobi second vector needs.
#include "bs_internal.h"

namespace bs {

constexpr int kResidThreads = 256;
constexpr int kResidPerThread = kResidCellsPerBlock / kResidThreads;

// Block b covers cells [first, first + 2048) of patch block_patch[b] in f order.
__global__ void __launch_bounds__(kResidThreads) k_residual(ResidArgs a)
{
    __shared__ double red[kResidThreads];
    const int b = blockIdx.x;
    const PatchDesc *pd = a.pd + a.block_patch[b];
    const int nx = pd->n[0], ny = pd->n[1], nz = pd->n[2];
    const int64_t ncell = (int64_t)nx * ny * nz;
    const int64_t sx = nx + 2, sy = sx * (int64_t)(ny + 2);
    const double ex = pd->eps[0], ey = pd->eps[1], ez = pd->eps[2];
    const double d = 2.0 * (ex + ey + ez);
    const int first = a.block_first[b];
    const int ncell32 = (int)ncell;
    const double *u = a.u;
    double acc = 0.0;
    double rv[kResidPerThread];
    int cfv[kResidPerThread];
#pragma unroll
    for (int m = 0; m < kResidPerThread; ++m) {
        const int cf0 = first + m * kResidThreads + (int)threadIdx.x;
        const int cf = cf0 < ncell32 ? cf0 : ncell32 - 1;      // clamped: loads need no branch
        const int i = cf % nx;
        const int jk = cf / nx;
        const int j = jk % ny, k = jk / ny;
        const int64_t c = pd->uoff + (int64_t)(k + 1) * sy + (int64_t)(j + 1) * sx + (i + 1);
        const double nb = ex * (u[c - 1] + u[c + 1]) + ey * (u[c - sx] + u[c + sx]) + ez * (u[c - sy] + u[c + sy]);
        const double r = fma(-d, u[c], fma(pd->h2, a.f[pd->foff + cf], nb));
        rv[m] = r;
        cfv[m] = cf0 < ncell32 ? cf : -1;
        acc = cf0 < ncell32 ? fma(r, r, acc) : acc;
    }
    if (a.r) {
#pragma unroll
        for (int m = 0; m < kResidPerThread; ++m)
            if (cfv[m] >= 0) a.r[pd->foff + cfv[m]] = rv[m];
    }
    // low-precision copies for the mixed plane solves (rounded from FP64)
    if (a.e32) {
#pragma unroll
        for (int m = 0; m < kResidPerThread; ++m)
            if (cfv[m] >= 0) a.e32[pd->foff + cfv[m]] = (float)rv[m];
    }
    if (a.e16) {
#pragma unroll
        for (int m = 0; m < kResidPerThread; ++m)
            if (cfv[m] >= 0)
                a.e16[pd->foff + cfv[m]] = __builtin_bit_cast(unsigned short, static_cast<__bf16>(rv[m]));
    }
    if (!a.partial) return;
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kResidThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.partial[b] = red[0];
}

// One workgroup per patch: fixed-order sum of the patch's block partials.
__global__ void __launch_bounds__(256) k_residual_final(const double *partial, const int32_t *first_block,
                                                        double *out)
{
    __shared__ double red[256];
    const int p = blockIdx.x;
    const int b0 = first_block[p], b1 = first_block[p + 1];
    double acc = 0.0;
    for (int b = b0 + (int)threadIdx.x; b < b1; b += 256) acc += partial[b];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[p] = red[0];
}

// Face ghosts of every patch: src -> dst.  blockIdx.y = patch.
__global__ void __launch_bounds__(256) k_ghost_copy(const double *src, double *dst, const PatchDesc *pds)
{
    const PatchDesc *pd = pds + blockIdx.y;
    const int nx = pd->n[0], ny = pd->n[1], nz = pd->n[2];
    const int64_t sx = nx + 2, sy = sx * (int64_t)(ny + 2);
    const int64_t fz = (int64_t)(ny + 2) * (nx + 2);     // one z face (whole padded plane)
    const int64_t fy = (int64_t)nz * (nx + 2);           // one y face (interior k)
    const int64_t fx = (int64_t)nz * ny;                 // one x face (interior j, k)
    const int64_t total = 2 * fz + 2 * fy + 2 * fx;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        int64_t c;
        if (g < 2 * fz) {
            const int64_t side = g / fz, e = g % fz;
            c = (side ? (int64_t)(nz + 1) * sy : 0) + e;
        } else if (g < 2 * fz + 2 * fy) {
            const int64_t h = g - 2 * fz, side = h / fy, e = h % fy;
            const int64_t k = e / (nx + 2), i = e % (nx + 2);
            c = (k + 1) * sy + (side ? (int64_t)(ny + 1) * sx : 0) + i;
        } else {
            const int64_t h = g - 2 * fz - 2 * fy, side = h / fx, e = h % fx;
            const int64_t k = e / ny, j = e % ny;
            c = (k + 1) * sy + (j + 1) * sx + (side ? nx + 1 : 0);
        }
        dst[pd->uoff + c] = src[pd->uoff + c];
    }
}

// Interior cells of every patch: src -> dst.  blockIdx.y = patch.
__global__ void __launch_bounds__(256) k_interior_copy(const double *src, double *dst, const PatchDesc *pds)
{
    const PatchDesc *pd = pds + blockIdx.y;
    const int nx = pd->n[0], ny = pd->n[1], nz = pd->n[2];
    const int64_t sx = nx + 2, sy = sx * (int64_t)(ny + 2);
    const int64_t rows = (int64_t)ny * nz;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const int64_t j = row % ny, k = row / ny;
        const int64_t base = pd->uoff + (k + 1) * sy + (j + 1) * sx + 1;
        for (int i = threadIdx.x; i < nx; i += blockDim.x) dst[base + i] = src[base + i];
    }
}

hipError_t launch_residual(const ResidArgs &a, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_residual, dim3(nblocks), dim3(kResidThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_residual_final(const double *partial, const int32_t *patch_first_block, int npatch,
                                 double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_residual_final, dim3(npatch), dim3(256), 0, s, partial, patch_first_block, out);
    return hipGetLastError();
}

hipError_t launch_ghost_copy(const double *src, double *dst, const PatchDesc *pd, int npatch, hipStream_t s)
{
    hipLaunchKernelGGL(k_ghost_copy, dim3(64, npatch), dim3(256), 0, s, src, dst, pd);
    return hipGetLastError();
}

hipError_t launch_interior_copy(const double *src, double *dst, const PatchDesc *pd, int npatch, hipStream_t s)
{
    hipLaunchKernelGGL(k_interior_copy, dim3(1024, npatch), dim3(256), 0, s, src, dst, pd);
    return hipGetLastError();
}

}  // namespace bs
