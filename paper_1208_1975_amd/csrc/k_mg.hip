// Grid transfers of the geometric multigrid cycle that uses the block
// smoothers (section 1: line and plane smoothers as components of robust
// geometric multigrid; section 5: multilevel use).  Cell-centred grids: coarse
// cell (I,J,K) covers fine cells (2I+a, 2J+b, 2K+c), a, b, c in {0, 1}.
#include <algorithm>

#include "bs_internal.h"

namespace bs {

// f_c = (mean of the eight fine values of d) / h^2 with the fine h of the
// patch (blockIdx.y): the defect of A u = h^2 f restricted to the right-hand
// side of the coarse equation A e = (2h)^2 f_c.
__global__ void __launch_bounds__(256) k_restrict(const double *d, double *fc, const PatchDesc *pf,
                                                  const PatchDesc *pc)
{
    const PatchDesc *F = pf + blockIdx.y, *C = pc + blockIdx.y;
    const double scale = 1.0 / F->h2;
    const int nx = F->n[0], ny = F->n[1];
    const int mx = C->n[0], my = C->n[1], mz = C->n[2];
    const int64_t total = (int64_t)mx * my * mz;
    const double *df = d + F->foff;
    const int64_t px = nx, py = (int64_t)nx * ny;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < total; c += (int64_t)gridDim.x * blockDim.x) {
        const int I = (int)(c % mx);
        const int64_t r = c / mx;
        const int J = (int)(r % my), K = (int)(r / my);
        const int64_t b = 2 * (int64_t)K * py + 2 * (int64_t)J * px + 2 * I;
        const double s = ((df[b] + df[b + 1]) + (df[b + px] + df[b + px + 1])) +
                         ((df[b + py] + df[b + py + 1]) + (df[b + py + px] + df[b + py + px + 1]));
        fc[C->foff + c] = scale * (s * 0.125);
    }
}

// Coarse value at (t0, t1, t2), each index at most one cell outside the patch:
// read as stored (ghosts), except beyond an extrapolated face, where it is the
// negated value of the cell reflected back inside (once per such axis).
__device__ __forceinline__ double coarse_val(const double *uc, const int n[3], int64_t sx, int64_t sy, int bc,
                                             int t0, int t1, int t2)
{
    double sg = 1.0;
    int t[3] = {t0, t1, t2};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (t[a] < 0 && ((bc >> (2 * a)) & 1)) {
            t[a] = 0;
            sg = -sg;
        }
        if (t[a] >= n[a] && ((bc >> (2 * a + 1)) & 1)) {
            t[a] = n[a] - 1;
            sg = -sg;
        }
    }
    return sg * uc[(int64_t)(t[2] + 1) * sy + (int64_t)(t[1] + 1) * sx + (t[0] + 1)];
}

// u_f += trilinear interpolation of the coarse u_c: along each axis a fine
// cell takes 3/4 of its parent and 1/4 of the parent's neighbour on its side.
__global__ void __launch_bounds__(256) k_prolong_add(const double *uc, double *uf, const PatchDesc *pf,
                                                     const PatchDesc *pc, int bc)
{
    const PatchDesc *F = pf + blockIdx.y, *C = pc + blockIdx.y;
    const int nx = F->n[0], ny = F->n[1], nz = F->n[2];
    const int n[3] = {C->n[0], C->n[1], C->n[2]};
    const int64_t fsx = nx + 2, fsy = fsx * (ny + 2);
    const int64_t csx = n[0] + 2, csy = csx * (n[1] + 2);
    const double *u = uc + C->uoff;
    const int64_t total = (int64_t)nx * ny * nz;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < total; c += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(c % nx);
        const int64_t r = c / nx;
        const int j = (int)(r % ny), k = (int)(r / ny);
        const int I = i >> 1, J = j >> 1, K = k >> 1;
        const int di = (i & 1) ? 1 : -1, dj = (j & 1) ? 1 : -1, dk = (k & 1) ? 1 : -1;
        double v = 0.0;
#pragma unroll
        for (int cc = 0; cc < 2; ++cc)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const double w = (a ? 0.25 : 0.75) * (b ? 0.25 : 0.75) * (cc ? 0.25 : 0.75);
                    v = fma(w, coarse_val(u, n, csx, csy, bc, I + a * di, J + b * dj, K + cc * dk), v);
                }
        uf[F->uoff + (int64_t)(k + 1) * fsy + (int64_t)(j + 1) * fsx + (i + 1)] += v;
    }
}

hipError_t launch_restrict(const double *d, double *fc, const PatchDesc *pf, const PatchDesc *pc, int npatch,
                           int64_t max_cells, hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>((max_cells + 255) / 256, 4096);
    hipLaunchKernelGGL(k_restrict, dim3((unsigned)std::max<int64_t>(blocks, 1), npatch), dim3(256), 0, s, d, fc, pf,
                       pc);
    return hipGetLastError();
}

hipError_t launch_prolong_add(const double *uc, double *uf, const PatchDesc *pf, const PatchDesc *pc, int npatch,
                              int64_t max_cells, int bc, hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>((max_cells + 255) / 256, 4096);
    hipLaunchKernelGGL(k_prolong_add, dim3((unsigned)std::max<int64_t>(blocks, 1), npatch), dim3(256), 0, s, uc, uf,
                       pf, pc, bc);
    return hipGetLastError();
}

}  // namespace bs
