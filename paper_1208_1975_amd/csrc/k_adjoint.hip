// Adjoint of damped Jacobi line sweeps.  With interior unknowns x, fixed
// ghosts g, x^{k+1} = x^k + omega M^{-1} r(x^k), r = h^2 F + B g - A_int x,
// and symmetric M and A, one reverse step for dL/dx^{k+1} = gbar is
//   lambda    = M^{-1} gbar                    (line solve, done by k_line)
//   dL/dF    += omega h^2 lambda
//   dL/dg    += omega B^T lambda               (face ghosts: eps_a lambda of the adjacent cell)
//   dL/deps_a += -omega <lambda, D_a U^k + (dM/deps_a) w^k>,  w^k = M^{-1} r(x^k)
//   gbar      <- gbar - omega A_int lambda
// with D_a U = 2U - U_{-a} - U_{+a} (ghosts included) and, for lines along
// axis a, dM/deps_a = tridiag(-1, 2, -1) on each line and dM/deps_b = 2 I.
#include <algorithm>

#include "bs_internal.h"

namespace bs {

struct AdjArgs {
    const double *lam;    // u layout, zero ghosts
    const double *U;      // U^k, u layout with the real ghosts
    const double *w;      // w^k, u layout, zero ghosts
    double *gbar;         // u layout: interior = gbar (updated), face ghosts accumulate dL/dg
    double *gf;           // f layout, accumulates dL/dF (may be null)
    double *acc;          // [nblocks][3] per-block accumulators of <lambda, ...>
    const PatchDesc *pd;
    const int32_t *block_patch;
    const int32_t *block_first;
    int axis;
    double omega;
};

constexpr int kAdjThreads = 256;
constexpr int kAdjPerThread = kBlockCells / kAdjThreads;

__global__ void __launch_bounds__(256) k_fill(double *x, int64_t n, double v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

// gbar = grad_uK on interior cells, 0 on ghost cells (blockIdx.y = patch).
__global__ void __launch_bounds__(256) k_adj_init(const double *gK, double *gbar, const PatchDesc *pds)
{
    const PatchDesc *pd = pds + blockIdx.y;
    const int nx = pd->n[0], ny = pd->n[1], nz = pd->n[2];
    const int64_t sx = nx + 2, sy = sx * (int64_t)(ny + 2);
    const int64_t total = sy * (nz + 2);
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < total; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = c % sx, j = (c / sx) % (ny + 2), k = c / sy;
        const bool interior = i >= 1 && i <= nx && j >= 1 && j <= ny && k >= 1 && k <= nz;
        gbar[pd->uoff + c] = interior ? gK[pd->uoff + c] : 0.0;
    }
}

__global__ void __launch_bounds__(kAdjThreads) k_adj_step(AdjArgs a)
{
    __shared__ double red[3][kAdjThreads];
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const PatchDesc *pd = a.pd + a.block_patch[b];
    const int nx = pd->n[0], ny = pd->n[1], nz = pd->n[2];
    const int ncell = nx * ny * nz;
    const int64_t sx = nx + 2, sy = sx * (int64_t)(ny + 2);
    const double e[3] = {pd->eps[0], pd->eps[1], pd->eps[2]};
    const int64_t st[3] = {1, sx, sy};
    const int first = a.block_first[b];
    const double om = a.omega;
    const double rnx = 1.0 / nx, rny = 1.0 / ny;
    double part[3] = {0.0, 0.0, 0.0};
    for (int m = 0; m < kAdjPerThread; ++m) {
        const int cf = first + m * kAdjThreads + (int)threadIdx.x;
        if (cf >= ncell) break;
        const int jk = div_rd(cf, nx, rnx), i = cf - jk * nx, k = div_rd(jk, ny, rny), j = jk - k * ny;
        const int64_t c = pd->uoff + (int64_t)(k + 1) * sy + (int64_t)(j + 1) * sx + (i + 1);
        const double l = a.lam[c];
        double al = 0.0;
        double contrib[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int64_t s = st[d];
            al = fma(e[d], 2.0 * l - a.lam[c - s] - a.lam[c + s], al);
            const double du = 2.0 * a.U[c] - a.U[c - s] - a.U[c + s];
            const double mw = d == a.axis ? 2.0 * a.w[c] - a.w[c - s] - a.w[c + s] : 2.0 * a.w[c];
            contrib[d] = l * (du + mw);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) part[d] += contrib[d];
        a.gbar[c] = fma(-om, al, a.gbar[c]);
        if (a.gf) a.gf[pd->foff + cf] = fma(om * pd->h2, l, a.gf[pd->foff + cf]);
        // face ghosts: each is next to exactly one interior cell, so no two
        // threads touch the same entry
        const int idx[3] = {i, j, k};
        const int nn[3] = {nx, ny, nz};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (idx[d] == 0) a.gbar[c - st[d]] = fma(om * e[d], l, a.gbar[c - st[d]]);
            if (idx[d] == nn[d] - 1) a.gbar[c + st[d]] = fma(om * e[d], l, a.gbar[c + st[d]]);
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) red[d][threadIdx.x] = part[d];
    __syncthreads();
    for (int s = kAdjThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int d = 0; d < 3; ++d) red[d][threadIdx.x] += red[d][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 3) a.acc[3 * (int64_t)b + threadIdx.x] += red[threadIdx.x][0];
}

// grad_eps[3p + d] = -omega * (fixed-order sum of the patch's block accumulators)
__global__ void __launch_bounds__(256) k_eps_final(const double *acc, const int32_t *first_block, double omega,
                                                   double *out)
{
    __shared__ double red[3][256];
    const int p = blockIdx.x;
    const int b0 = first_block[p], b1 = first_block[p + 1];
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = b0 + (int)threadIdx.x; b < b1; b += 256)
#pragma unroll
        for (int d = 0; d < 3; ++d) s[d] += acc[3 * (int64_t)b + d];
#pragma unroll
    for (int d = 0; d < 3; ++d) red[d][threadIdx.x] = s[d];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int d = 0; d < 3; ++d) red[d][threadIdx.x] += red[d][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[3 * p + threadIdx.x] = -omega * red[threadIdx.x][0];
}

hipError_t launch_fill(double *x, int64_t n, double v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, x, n, v);
    return hipGetLastError();
}

hipError_t launch_adj_init(const double *gK, double *gbar, const PatchDesc *pd, int npatch, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_init, dim3(256, npatch), dim3(256), 0, s, gK, gbar, pd);
    return hipGetLastError();
}

hipError_t launch_adj_step(const double *lam, const double *U, const double *w, double *gbar, double *gf,
                           double *acc, const PatchDesc *pd, const int32_t *block_patch,
                           const int32_t *block_first, int nblocks, int axis, double omega, hipStream_t s)
{
    AdjArgs a{lam, U, w, gbar, gf, acc, pd, block_patch, block_first, axis, omega};
    hipLaunchKernelGGL(k_adj_step, dim3(nblocks), dim3(kAdjThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_eps_final(const double *acc, const int32_t *first_block, int npatch, double omega, double *out,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_eps_final, dim3(npatch), dim3(256), 0, s, acc, first_block, omega, out);
    return hipGetLastError();
}

}  // namespace bs
