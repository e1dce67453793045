// Geometric cube blocks (section 2; the block Jacobi algorithm on GPUs, step
// 1): the residual of every cell of a run of equally shaped blocks, gathered
// into a block-major matrix R[block][cell] (cells of a block numbered x
// fastest).  Step 2, the product with the precomputed block inverse, is the
// FP64 matrix-core product R Ainv^T, whose epilogue applies step 3 (the
// update) through the same offset tables.
#include <cstdint>

#include "bs_internal.h"

namespace bs {

// A workgroup owns `per` consecutive blocks (256 / nb of them for blocks of
// up to 256 cells, else one); its threads walk the per * nb cells with the
// cell index fastest, so the x-runs of a block are read with consecutive
// lanes and R is written contiguously.
__global__ void __launch_bounds__(256) k_cube_resid(CubeResidArgs a)
{
    const int b0 = blockIdx.x * a.per;
    const int tot = a.per * a.nb;
    for (int e = threadIdx.x; e < tot; e += 256) {
        const int lb = e / a.nb;
        const int c = e - lb * a.nb;
        const int b = b0 + lb;
        if (b >= a.nblk) break;
        const int64_t iu = a.ubase[b] + a.uoff[c];
        const double uc = a.u[iu];
        const double ax = a.ex * (2.0 * uc - a.u[iu - 1] - a.u[iu + 1]);
        const double ay = a.ey * (2.0 * uc - a.u[iu - a.sy] - a.u[iu + a.sy]);
        const double az = a.ez * (2.0 * uc - a.u[iu - a.sz] - a.u[iu + a.sz]);
        a.R[(int64_t)b * a.nb + c] = a.h2 * a.f[a.fbase[b] + a.foff[c]] - (ax + ay + az);
    }
}

hipError_t launch_cube_resid(const CubeResidArgs &a, hipStream_t s)
{
    if (a.nblk <= 0) return hipSuccess;
    if (a.nb <= 0 || a.per <= 0) return hipErrorInvalidValue;
    const int grid = (a.nblk + a.per - 1) / a.per;
    hipLaunchKernelGGL(k_cube_resid, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace bs
