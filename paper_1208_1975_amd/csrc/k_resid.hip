// Residual r = h^2 f - A u (eq. stencil3d7 with axis weights; on an
// extrapolated face the ghost is the negated adjacent cell) and its
// per-patch 2-norm^2, reduced in a fixed order (bit-reproducible); plus the
// copies the Jacobi second vector needs.
#include "bs_internal.h"

namespace bs {

constexpr int kResidThreads = 256;

// Value of lane l-1 (DIR < 0) or l+1 (DIR > 0) of the wavefront (DPP wave shift).
template <int DIR>
__device__ __forceinline__ double wave_nb(double v)
{
    constexpr int ctrl = DIR < 0 ? 0x138 : 0x130;   // wave_shr:1 / wave_shl:1
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), ctrl, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), ctrl, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// One tile: a workgroup of tx x ty columns (tx lanes along x, tx the power of
// two in [1, 64] nearest above nx, ty = 256 / tx) marched along z.  The z
// neighbours stay in registers (each u plane is read once per tile, plus one
// halo plane on each side), the x neighbours come from the adjacent lanes
// (DPP), except at a row's ends, which load theirs, and every load of the
// next plane (centre u two planes ahead, f, the y-neighbour rows, the row-end
// x values) is issued one step ahead.  The tile's sum of r^2 is accumulated
// per thread in increasing z and reduced in a fixed tree: the norm is
// bit-reproducible.
__global__ void __launch_bounds__(kResidThreads) k_residual(ResidArgs a)
{
    __shared__ double red[kResidThreads];
    const int b = xcd_block(blockIdx.x, gridDim.x);   // tiles in patch, z, y, x order: an XCD gets a contiguous run
    const ResidTile t = a.tiles[b];
    const PatchDesc *pd = a.pd + t.patch;
    const int nx = pd->n[0], ny = pd->n[1], nz = pd->n[2];
    const int64_t sx = nx + 2, sy = sx * (int64_t)(ny + 2), pf = (int64_t)nx * ny;
    const double ex = pd->eps[0], ey = pd->eps[1], ez = pd->eps[2];
    const double d = 2.0 * (ex + ey + ez), h2 = pd->h2;
    int tx = 64;
    while (tx > 1 && (tx >> 1) >= nx) tx >>= 1;
    const int li = (int)(threadIdx.x & (tx - 1));
    const int i = t.x0 + li;
    const int j = t.y0 + (int)(threadIdx.x / tx);
    const bool valid = i < nx && j < ny;
    const int ic = i < nx ? i : nx - 1, jc = j < ny ? j : ny - 1;   // in-patch addresses for every lane
    const bool need_l = li == 0, need_r = li == tx - 1 || i >= nx - 1;
    const int64_t xo = need_l ? -1 : 1;                            // the row-end lane's own neighbour
    const int bc = pd->bc;
    const bool xlo = (bc & 1) && i == 0, xhi = (bc & 2) && i == nx - 1;
    const bool ylo = (bc & 4) && j == 0, yhi = (bc & 8) && j == ny - 1;
    const bool zlo = (bc & 16) != 0, zhi = (bc & 32) != 0;
    const int k0 = t.z0, k1 = t.z1;
    const double *u = a.u + pd->uoff + (int64_t)(jc + 1) * sx + (ic + 1);   // column (i, j), plane index k + 1
    const int64_t fo = pd->foff + (int64_t)jc * nx + ic;                     // f / r column, plane index k
    double uzm = u[(int64_t)k0 * sy];
    double uc = u[(int64_t)(k0 + 1) * sy];
    double uzp = u[(int64_t)(k0 + 2) * sy];
    const double *u1 = u + (int64_t)(k0 + 1) * sy;
    double fv = a.f[fo + (int64_t)k0 * pf];
    double ym = u1[-sx], yp = u1[sx], xa = u1[xo], xb = tx == 1 ? u1[1] : 0.0;
    double acc = 0.0;
    for (int k = k0; k < k1; ++k) {
        // the next step's loads (clamped inside the patch on the last step)
        const int kn = k + 1 < nz ? k + 1 : nz - 1;
        const double *un = u + (int64_t)(kn + 1) * sy;
        const double uzp_n = un[sy];
        const double f_n = a.f[fo + (int64_t)kn * pf];
        const double ym_n = un[-sx], yp_n = un[sx], xa_n = un[xo];
        const double xb_n = tx == 1 ? un[1] : 0.0;
        // the moves run under full EXEC: the empty asm pins their results
        // before the selects, which the compiler may turn into branches
        double dl = wave_nb<-1>(uc), dr = wave_nb<+1>(uc);
        asm volatile("" : "+v"(dl), "+v"(dr));
        double left = need_l ? xa : dl;
        double right = need_r ? (need_l ? xb : xa) : dr;
        // extrapolated faces: the ghost is the negated cell itself
        left = xlo ? -uc : left;
        right = xhi ? -uc : right;
        const double yl = ylo ? -uc : ym, yh = yhi ? -uc : yp;
        const double zl = (zlo && k == 0) ? -uc : uzm, zh = (zhi && k == nz - 1) ? -uc : uzp;
        const double nb = fma(ex, left + right, fma(ey, yl + yh, ez * (zl + zh)));
        const double r = fma(-d, uc, fma(h2, fv, nb));
        if (valid) {
            const int64_t c = fo + (int64_t)k * pf;
            if (a.r) a.r[c] = r;
            if (a.e32) a.e32[c] = (float)r;
            if (a.r32) a.r32[c] = (float)r;
            if (a.e16) a.e16[c] = __builtin_bit_cast(unsigned short, static_cast<__bf16>(r));
            acc = fma(r, r, acc);
        }
        uzm = uc;
        uc = uzp;
        uzp = uzp_n;
        fv = f_n;
        ym = ym_n;
        yp = yp_n;
        xa = xa_n;
        xb = xb_n;
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

// One workgroup per patch: fixed-order sum of the patch's tile (or block) partials.
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

hipError_t launch_residual(const ResidArgs &a, int ntiles, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_residual, dim3(ntiles), dim3(kResidThreads), 0, s, a);
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
