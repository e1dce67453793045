// Adjoint of damped Jacobi line or plane sweeps, and of each half-step of
// two-colour GS (the projection P onto one colour's blocks commutes with M;
// lambda = M^{-1} P gbar, w = P M^{-1} r).  With interior unknowns x, fixed
// ghosts g, x^{k+1} = x^k + omega M^{-1} r(x^k), r = h^2 F + B g - A_int x,
// and symmetric M and A, one reverse step for dL/dx^{k+1} = gbar is
//   lambda    = M^{-1} gbar                    (line solve, done by k_line)
//   dL/dF    += omega h^2 lambda
//   dL/dg    += omega B^T lambda               (face ghosts: eps_a lambda of the adjacent cell)
//   dL/deps_a += -omega <lambda, D_a U^k + (dM/deps_a) w^k>,  w^k = M^{-1} r(x^k)
//   gbar      <- gbar - omega A_int lambda
// with D_a U = 2U - U_{-a} - U_{+a} (ghosts included) and dM/deps_b =
// tridiag(-1, 2, -1) inside each block along an axis b the blocks span, 2 I
// along the others.
#include <algorithm>

#include "bs_internal.h"
#include "line_dev.h"

namespace bs {

struct AdjArgs {
    const double *lam;    // u layout, zero ghosts
    const double *U;      // U^k, u layout with the real ghosts
    const double *w;      // w^k, u layout, zero ghosts
    double *gbar;         // u layout: interior = gbar (updated), face ghosts accumulate dL/dg
    double *gf;           // f layout, accumulates dL/dF (may be null)
    double *acc;          // [ntiles][3] per-tile accumulators of <lambda, ...>
    const PatchDesc *pd;
    const ResidTile *tiles;
    int spans;            // bit b: the blocks span axis b
    double omega;
};

constexpr int kAdjThreads = 256;

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

// Interior of a u-layout field into f layout (blockIdx.y = patch).
__global__ void __launch_bounds__(256) k_u_to_f(const double *src, double *dst, const PatchDesc *pds)
{
    const PatchDesc *pd = pds + blockIdx.y;
    const int nx = pd->n[0], ny = pd->n[1], nz = pd->n[2];
    const int64_t sx = nx + 2, sy = sx * (int64_t)(ny + 2);
    const int64_t total = (int64_t)nx * ny * nz;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < total; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = c % nx, j = (c / nx) % ny, k = c / ((int64_t)nx * ny);
        dst[pd->foff + c] = src[pd->uoff + (k + 1) * sy + (j + 1) * sx + (i + 1)];
    }
}

// One tile of the residual's tiling (tx x ty columns marched along z): the
// z-neighbours of lambda, U and w stay in registers and the next plane's
// values are fetched a step ahead; the x-neighbours come from the adjacent
// lanes (DPP) except at a row's ends, which load theirs; w's neighbours are
// read only along the axes the blocks span (SP, the spans mask).  Each
// column's partial sums run in increasing z and the tile's sums reduce in a
// fixed tree, so the epsilon gradient is bit-reproducible.
template <int SP>
__global__ void __launch_bounds__(kAdjThreads) k_adj_step(AdjArgs a)
{
    __shared__ double red[3][kAdjThreads];
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const ResidTile t = a.tiles[b];
    const PatchDesc *pd = a.pd + t.patch;
    const int nx = pd->n[0], ny = pd->n[1], nz = pd->n[2];
    const int64_t sx = nx + 2, sy = sx * (int64_t)(ny + 2), pf = (int64_t)nx * ny;
    const double e0 = pd->eps[0], e1 = pd->eps[1], e2 = pd->eps[2];
    const double om = a.omega, omh2 = a.omega * pd->h2;
    int tx = 64;
    while (tx > 1 && (tx >> 1) >= nx) tx >>= 1;
    const int li = (int)(threadIdx.x & (tx - 1));
    const int i = t.x0 + li;
    const int j = t.y0 + (int)(threadIdx.x / tx);
    const bool valid = i < nx && j < ny;
    const int ic = i < nx ? i : nx - 1, jc = j < ny ? j : ny - 1;   // in-patch addresses for every lane
    // row ends take their x-neighbours from memory (both sides when tx = 1)
    const bool need_l = li == 0, need_r = li == tx - 1 || i >= nx - 1;
    const int64_t xo = need_l ? -1 : 1;
    const bool two = tx == 1;
    const int k0 = t.z0, k1 = t.z1;
    const int64_t col = pd->uoff + (int64_t)(jc + 1) * sx + (ic + 1);   // column (i, j); plane index k + 1
    const int64_t fo = pd->foff + (int64_t)jc * nx + ic;
    const double *Lc = a.lam + col, *Uc = a.U + col, *Wc = a.w + col;
    double lm = Lc[(int64_t)k0 * sy], lc = Lc[(int64_t)(k0 + 1) * sy], lp = Lc[(int64_t)(k0 + 2) * sy];
    double um = Uc[(int64_t)k0 * sy], uc = Uc[(int64_t)(k0 + 1) * sy], up = Uc[(int64_t)(k0 + 2) * sy];
    double wm = Wc[(int64_t)k0 * sy], wc = Wc[(int64_t)(k0 + 1) * sy], wp = Wc[(int64_t)(k0 + 2) * sy];
    double p0 = 0.0, p1 = 0.0, p2 = 0.0;
    for (int k = k0; k < k1; ++k) {
        const int64_t c = (int64_t)(k + 1) * sy;
        // the next step's plane (clamped inside the patch on the last step)
        const int64_t cn = (int64_t)((k + 1 < nz ? k + 1 : nz - 1) + 2) * sy;
        const double lp_n = Lc[cn], up_n = Uc[cn], wp_n = Wc[cn];
        const double lym = Lc[c - sx], lyp = Lc[c + sx], uym = Uc[c - sx], uyp = Uc[c + sx];
        const double lxa = Lc[c + xo], uxa = Uc[c + xo];
        const double lxb = two ? Lc[c + 1] : 0.0, uxb = two ? Uc[c + 1] : 0.0;
        // w's neighbours along x and y (z from registers); w is zero outside
        // the blocks' cells, so a block's edge sees zero beyond it
        double wym = 0.0, wyp = 0.0, wxa = 0.0, wxb = 0.0;
        if constexpr ((SP & 2) != 0) {
            wym = Wc[c - sx];
            wyp = Wc[c + sx];
        }
        if constexpr ((SP & 1) != 0) {
            wxa = Wc[c + xo];
            wxb = two ? Wc[c + 1] : 0.0;
        }
        const double g0 = a.gbar[col + c];
        const double gf0 = a.gf ? a.gf[fo + (int64_t)k * pf] : 0.0;
        // the moves run under full EXEC: the empty asm pins their results
        // before the selects
        double ldl = lane_shift<-1>(lc), ldr = lane_shift<+1>(lc);
        double udl = lane_shift<-1>(uc), udr = lane_shift<+1>(uc);
        asm volatile("" : "+v"(ldl), "+v"(ldr), "+v"(udl), "+v"(udr));
        const double lxm = need_l ? lxa : ldl, lxp = need_r ? (need_l ? lxb : lxa) : ldr;
        const double uxm = need_l ? uxa : udl, uxp = need_r ? (need_l ? uxb : uxa) : udr;
        double al = fma(e0, 2.0 * lc - lxm - lxp, 0.0);
        al = fma(e1, 2.0 * lc - lym - lyp, al);
        al = fma(e2, 2.0 * lc - lm - lp, al);
        const double w2 = 2.0 * wc;
        double mw0 = w2;
        if constexpr ((SP & 1) != 0) {
            double wdl = lane_shift<-1>(wc), wdr = lane_shift<+1>(wc);
            asm volatile("" : "+v"(wdl), "+v"(wdr));
            const double wxm = need_l ? wxa : wdl, wxp = need_r ? (need_l ? wxb : wxa) : wdr;
            mw0 = w2 - wxm - wxp;
        }
        const double mw1 = (SP & 2) ? w2 - wym - wyp : w2;
        const double mw2 = (SP & 4) ? w2 - wm - wp : w2;
        if (valid) {
            p0 += lc * ((2.0 * uc - uxm - uxp) + mw0);
            p1 += lc * ((2.0 * uc - uym - uyp) + mw1);
            p2 += lc * ((2.0 * uc - um - up) + mw2);
            double *gb = a.gbar + col + c;
            gb[0] = fma(-om, al, g0);
            if (a.gf) a.gf[fo + (int64_t)k * pf] = fma(omh2, lc, gf0);
            // face ghosts: each is next to exactly one interior cell, so no two
            // threads touch the same entry
            if (i == 0) gb[-1] = fma(om * e0, lc, gb[-1]);
            if (i == nx - 1) gb[1] = fma(om * e0, lc, gb[1]);
            if (j == 0) gb[-sx] = fma(om * e1, lc, gb[-sx]);
            if (j == ny - 1) gb[sx] = fma(om * e1, lc, gb[sx]);
            if (k == 0) gb[-sy] = fma(om * e2, lc, gb[-sy]);
            if (k == nz - 1) gb[sy] = fma(om * e2, lc, gb[sy]);
        }
        lm = lc; lc = lp; lp = lp_n;
        um = uc; uc = up; up = up_n;
        wm = wc; wc = wp; wp = wp_n;
    }
    red[0][threadIdx.x] = p0;
    red[1][threadIdx.x] = p1;
    red[2][threadIdx.x] = p2;
    __syncthreads();
    for (int s = kAdjThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int d = 0; d < 3; ++d) red[d][threadIdx.x] += red[d][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 3) a.acc[3 * (int64_t)b + threadIdx.x] += red[threadIdx.x][0];
}

// grad_eps[3p + d] = -omega * (fixed-order sum of the patch's tile accumulators)
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

hipError_t launch_u_to_f(const double *src, double *dst, const PatchDesc *pd, int npatch, hipStream_t s)
{
    hipLaunchKernelGGL(k_u_to_f, dim3(256, npatch), dim3(256), 0, s, src, dst, pd);
    return hipGetLastError();
}

hipError_t launch_adj_init(const double *gK, double *gbar, const PatchDesc *pd, int npatch, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_init, dim3(256, npatch), dim3(256), 0, s, gK, gbar, pd);
    return hipGetLastError();
}

hipError_t launch_adj_step(const double *lam, const double *U, const double *w, double *gbar, double *gf,
                           double *acc, const PatchDesc *pd, const ResidTile *tiles, int ntiles, int spans,
                           double omega, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    AdjArgs a{lam, U, w, gbar, gf, acc, pd, tiles, spans, omega};
    const dim3 g(ntiles), t(kAdjThreads);
    switch (spans) {
    case 1: hipLaunchKernelGGL(k_adj_step<1>, g, t, 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_adj_step<2>, g, t, 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_adj_step<3>, g, t, 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_adj_step<4>, g, t, 0, s, a); break;
    case 5: hipLaunchKernelGGL(k_adj_step<5>, g, t, 0, s, a); break;
    case 6: hipLaunchKernelGGL(k_adj_step<6>, g, t, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_eps_final(const double *acc, const int32_t *first_block, int npatch, double omega, double *out,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_eps_final, dim3(npatch), dim3(256), 0, s, acc, first_block, omega, out);
    return hipGetLastError();
}

}  // namespace bs
