// Geometric cube blocks (section 2; the block Jacobi algorithm on GPUs).
//
// Blocks of more than 256 cells: step 1, the residual of every cell of a run
// of equally shaped blocks, is gathered into a block-major matrix
// R[block][cell] (cells of a block numbered x fastest); step 2, the product
// with the precomputed block inverse, is the FP64 matrix-core product
// R Ainv^T, whose epilogue applies step 3 (the update) through the same
// offset tables.
//
// Blocks of 65 to 256 cells: all three steps in one kernel, the residuals
// formed into LDS and the inverse read from memory (k_cube_big).
//
// Small blocks (up to 64 cells): all three steps in one kernel.  The inverse
// (at most 64 x 64) sits in LDS and each wavefront forms its blocks'
// residuals in registers, multiplies them by the inverse on the matrix cores
// and writes the updated cells: u and f are read once and the result written
// once, with no residual matrix in HBM.
#include <cstdint>

#include "bs_internal.h"

namespace bs {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

}  // namespace

// A workgroup owns `per` consecutive blocks (256 / nb of them for blocks of
// up to 256 cells, else one); its threads walk the per * nb cells with the
// cell index fastest, so the x-runs of a block are read with consecutive
// lanes and R is written contiguously.  Workgroups map XCD-contiguously:
// neighbouring blocks share cache lines and faces in one L2.
__global__ void __launch_bounds__(256) k_cube_resid(CubeArgs a)
{
    const int b0 = xcd_block(blockIdx.x, gridDim.x) * a.per;
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

hipError_t launch_cube_resid(const CubeArgs &a, hipStream_t s)
{
    if (a.nblk <= 0) return hipSuccess;
    if (a.nb <= 0 || a.per <= 0) return hipErrorInvalidValue;
    const int grid = (a.nblk + a.per - 1) / a.per;
    hipLaunchKernelGGL(k_cube_resid, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Fused small blocks: NP = nb rounded up to 16, 32 or 64.  A workgroup takes
// one chunk (up to 64 consecutive blocks of one group's list; the group gives
// the inverse, offsets and stencil weights, so one launch covers every group
// of the same NP).  Wavefront w owns blocks 16w..16w+15 (rows of the product) and forms their
// residuals straight into the matrix-core operand layout: lane l holds the
// residual of cell k + l/16 of block l%16 for k = 0, 4, ..., NP-4 -- the A
// operand of v_mfma_f64_16x16x4 -- so residuals never touch LDS or HBM; only
// the inverse (Bs[k][n] = Ainv[n][k], zero outside nb x nb) and the cell
// offsets are staged in LDS.  With consecutive blocks along x, one load
// instruction reads 16 blocks x 4 cells of a row: for 4-cell block edges a
// contiguous x-run of 64 cells.  All loads use in-range (clamped) indices;
// padding cells and blocks past the end give zero through selects, so a
// batch's loads are in flight together.  Result layout as in the plane
// products: register r holds row 4r + l/16, column l%16; the update reads u
// from the registers the residual loaded it into (through an exact identity
// product), so the epilogue only stores.
// Workgroups are mapped XCD-contiguously, so neighbouring blocks (which read
// each other's faces) share an L2.
// RL: the update takes u from a second load in the epilogue instead of the
// identity product (frees 32 AGPRs: four waves per SIMD instead of three for
// NP = 64); measured faster only for 4^3 Jacobi (0.191 against 0.207 ms per
// sweep on 64 patches of 64^3), slower for every smaller block and for the
// in-place schemes, so the launcher takes it only there.
template <int NP, bool RL>
__global__ void __launch_bounds__(256) k_cube_small(CubeBatchArgs ba_)
{
    __shared__ double Bs[NP][NP + 1];
    __shared__ int32_t So[2][NP];   // u and f offsets of each cell (cell 0's past nb)
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int l16 = lane & 15, lk = lane >> 4;
    const CubeChunk ch = ba_.chunks[xcd_block(blockIdx.x, gridDim.x)];
    const CubeGroupDev &g = ba_.groups[ch.group];
    struct {
        const double *u, *f;
        double *dst;
        int64_t sy, sz;
        double ex, ey, ez, h2, omega;
    } a = {ba_.u, ba_.f, ba_.dst, g.sy, g.sz, g.ex, g.ey, g.ez, g.h2, ba_.omega};
    const int nb = g.nb;
    const int b0 = ch.first, bend = ch.end;
    const int64_t *ubase = g.ubase[ba_.list], *fbase = g.fbase[ba_.list];

#pragma unroll
    for (int e = tid; e < NP * NP; e += 256) {
        const int n = e / NP, k = e % NP;
        Bs[k][n] = (n < nb && k < nb) ? g.ainv[n * nb + k] : 0.0;
    }
    if (tid < NP) {
        So[0][tid] = g.uoff[tid < nb ? tid : 0];
        So[1][tid] = g.foff[tid < nb ? tid : 0];
    }
    const int ba = b0 + w * 16 + l16;            // this lane's block for the operand
    const bool bok = ba < bend;
    const int64_t ub = ubase[bok ? ba : b0], fb = fbase[bok ? ba : b0];
    __syncthreads();

    // Operands in batches of four (the 32 loads of a batch are issued before
    // any is consumed), each multiplied into the result as soon as it is
    // formed.  A second product with the identity, exact (one term u * 1 per
    // output, the rest zeros), re-expresses the loaded centre values in the
    // result layout, so the update needs no second load of u.
    dbl4 acc[NP / 16], accu[NP / 16];
#pragma unroll
    for (int j = 0; j < NP / 16; ++j) {
        acc[j] = dbl4{0.0, 0.0, 0.0, 0.0};
        accu[j] = dbl4{0.0, 0.0, 0.0, 0.0};
    }
#pragma unroll
    for (int t0 = 0; t0 < NP / 4; t0 += 4) {
        double v[4][8];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = 4 * (t0 + q) + lk;
            if (NP == 16 && 4 * (t0 + q) >= nb) {   // rows wholly past a block of <= 12 cells (uniform)
                for (int m = 0; m < 8; ++m) v[q][m] = 0.0;
                continue;
            }
            const int64_t iu = ub + So[0][c];
            v[q][0] = a.u[iu];
            v[q][1] = a.u[iu - 1];
            v[q][2] = a.u[iu + 1];
            v[q][3] = a.u[iu - a.sy];
            v[q][4] = a.u[iu + a.sy];
            v[q][5] = a.u[iu - a.sz];
            v[q][6] = a.u[iu + a.sz];
            v[q][7] = a.f[fb + So[1][c]];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int t = t0 + q;
            if (NP == 16 && 4 * t >= nb) break;   // zero operand rows (uniform)
            const int c = 4 * t + lk;
            const double uc = v[q][0];
            const double ax = a.ex * (2.0 * uc - v[q][1] - v[q][2]);
            const double ay = a.ey * (2.0 * uc - v[q][3] - v[q][4]);
            const double az = a.ez * (2.0 * uc - v[q][5] - v[q][6]);
            const double r = (bok && c < nb) ? a.h2 * v[q][7] - (ax + ay + az) : 0.0;
#pragma unroll
            for (int j = 0; j < NP / 16; ++j) {
                acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(r, Bs[c][j * 16 + l16], acc[j], 0, 0, 0);
                if constexpr (!RL)
                    accu[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(uc, c == j * 16 + l16 ? 1.0 : 0.0, accu[j], 0, 0,
                                                                   0);
            }
        }
    }

    // result register r of a lane: block 4r + l/16 of the wavefront, whose
    // base the operand lane 4r + l/16 holds
    if constexpr (RL) {
        // every old value of the chunk is read before any new one is stored
        double uo[4][NP / 16];
        int64_t bases[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            bases[r] = __shfl(ub, 4 * r + lk);
#pragma unroll
            for (int j = 0; j < NP / 16; ++j) uo[r][j] = a.u[bases[r] + So[0][j * 16 + l16]];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const bool ok = b0 + w * 16 + 4 * r + lk < bend;
#pragma unroll
            for (int j = 0; j < NP / 16; ++j)
                if (ok && j * 16 + l16 < nb) a.dst[bases[r] + So[0][j * 16 + l16]] = fma(a.omega, acc[j][r], uo[r][j]);
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int m = 4 * r + lk;
        const int64_t base = __shfl(ub, m);
        const bool ok = b0 + w * 16 + m < bend;
#pragma unroll
        for (int j = 0; j < NP / 16; ++j)
            if (ok && j * 16 + l16 < nb) a.dst[base + So[0][j * 16 + l16]] = fma(a.omega, acc[j][r], accu[j][r]);
    }
}

// Fused large blocks (65 to 256 cells): NP = nb rounded up to 128 or 256.  A
// workgroup of eight wavefronts owns 32 consecutive blocks of one group's
// list and all NP columns of their product with the inverse, so each
// residual is formed once and every cell of its blocks is read before any is
// written (in place, Gauss-Seidel); wavefront w computes 32 x (NP / 8) result
// columns as two row blocks of v_mfma_f64_16x16x4.  (Splitting the columns of
// a chunk over two workgroups, as 512-cell blocks would need for two
// workgroups per compute unit, lets one workgroup write cells of a block that
// the other still reads in place.)  The
// contraction runs over the cells 16 at a time: the 512 threads form the 32
// blocks' residuals of those 16 cells (one each, into LDS in the operand
// layout), and every wavefront reads its slice of the inverse straight from
// memory (the block matrix is symmetric, so row k of the stored inverse is
// its column k: 16 consecutive columns are one 128-byte run; all workgroups
// share it through L2).  The next step's residual inputs and inverse slice are
// loaded while the current step's products run.  Epilogue: dst = u + omega du
// through the offset tables, as the small-block kernel.
template <int NP>
__global__ void __launch_bounds__(512) k_cube_big(CubeBatchArgs ba_)
{
    constexpr int NW = NP / 8;      // result columns per wavefront
    constexpr int JB = NW / 16;     // 16-column blocks per wavefront
    constexpr int BK = 16;          // cells per step: one residual per thread
    constexpr int KS = BK / 4;      // matrix-core steps per step
    __shared__ double As[2][BK][33];   // [buffer][cell of the step][block]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int l16 = lane & 15, lk = lane >> 4;
    const CubeChunk ch = ba_.chunks[xcd_block(blockIdx.x, gridDim.x)];
    const CubeGroupDev &g = ba_.groups[ch.group];
    const double *u = ba_.u, *f = ba_.f;
    const int nb = g.nb, b0 = ch.first, bend = ch.end;
    const int64_t sy = g.sy, sz = g.sz;
    const double ex = g.ex, ey = g.ey, ez = g.ez, h2 = g.h2;
    const int64_t *ubase = g.ubase[ba_.list], *fbase = g.fbase[ba_.list];
    const double *ainv = g.ainv;

    // residual role: block rb (0..31), cell BK kt + rc of the step
    const int rb = tid / BK, rc = tid % BK;
    const bool rbok = b0 + rb < bend;
    const int64_t rub = ubase[rbok ? b0 + rb : b0], rfb = fbase[rbok ? b0 + rb : b0];
    const int nk = (nb + BK - 1) / BK;
    double v[8];
    auto rload = [&](int kt) {
        const int c = BK * kt + rc;
        const int cc = c < nb ? c : nb - 1;   // in-range offsets for every lane
        const int64_t iu = rub + g.uoff[cc];
        v[0] = u[iu];
        v[1] = u[iu - 1];
        v[2] = u[iu + 1];
        v[3] = u[iu - sy];
        v[4] = u[iu + sy];
        v[5] = u[iu - sz];
        v[6] = u[iu + sz];
        v[7] = f[rfb + g.foff[cc]];
    };
    auto rstore = [&](int kt, int buf) {
        const int c = BK * kt + rc;
        const double uc = v[0];
        const double ax = ex * (2.0 * uc - v[1] - v[2]);
        const double ay = ey * (2.0 * uc - v[3] - v[4]);
        const double az = ez * (2.0 * uc - v[5] - v[6]);
        As[buf][rc][rb] = (rbok && c < nb) ? h2 * v[7] - (ax + ay + az) : 0.0;
    };
    // inverse slice of a step: lane (l16, lk) holds Ainv[k][n] for k = BK kt +
    // 4 s + lk, n = w NW + 16 j + l16 (zero outside nb x nb)
    double bq[KS][JB];
    auto bload = [&](int kt, double (&o)[KS][JB]) {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int k = BK * kt + 4 * s + lk;
#pragma unroll
            for (int j = 0; j < JB; ++j) {
                const int n = w * NW + 16 * j + l16;
                const double x = ainv[(int64_t)(k < nb ? k : nb - 1) * nb + (n < nb ? n : nb - 1)];
                o[s][j] = (k < nb && n < nb) ? x : 0.0;
            }
        }
    };
    dbl4 acc[2][JB];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int j = 0; j < JB; ++j) acc[r][j] = dbl4{0.0, 0.0, 0.0, 0.0};

    rload(0);
    bload(0, bq);
    rstore(0, 0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        double bn[KS][JB];
        const bool more = kt + 1 < nk;
        if (more) {   // the next step's inputs, in flight during this step's products
            rload(kt + 1);
            bload(kt + 1, bn);
        }
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const double a0 = As[cur][4 * s + lk][l16], a1 = As[cur][4 * s + lk][16 + l16];
#pragma unroll
            for (int j = 0; j < JB; ++j) {
                acc[0][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bq[s][j], acc[0][j], 0, 0, 0);
                acc[1][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bq[s][j], acc[1][j], 0, 0, 0);
            }
        }
        if (more) {
            rstore(kt + 1, cur ^ 1);
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int j = 0; j < JB; ++j) bq[s][j] = bn[s][j];
        }
        __syncthreads();
    }

    // result register r of a lane: block 16 hb + 4 r + l/16, cell column
    // column n = w NW + 16 j + l16
#pragma unroll
    for (int hb = 0; hb < 2; ++hb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = 16 * hb + 4 * r + lk;
            const bool ok = b0 + m < bend;
            const int64_t base = ubase[ok ? b0 + m : b0];
            double uo[JB];
            int64_t at[JB];
#pragma unroll
            for (int j = 0; j < JB; ++j) {   // all the centre values first, then the stores
                const int n = w * NW + 16 * j + l16;
                at[j] = base + g.uoff[n < nb ? n : nb - 1];
                uo[j] = u[at[j]];
            }
#pragma unroll
            for (int j = 0; j < JB; ++j) {
                const int n = w * NW + 16 * j + l16;
                if (ok && n < nb) ba_.dst[at[j]] = fma(ba_.omega, acc[hb][j][r], uo[j]);
            }
        }
}

hipError_t launch_cube_big(const CubeBatchArgs &a, int nchunks, int np, hipStream_t s)
{
    if (nchunks <= 0) return hipSuccess;
    const dim3 grid(nchunks);
    if (np == 128) hipLaunchKernelGGL(k_cube_big<128>, grid, dim3(512), 0, s, a);
    else if (np == 256) hipLaunchKernelGGL(k_cube_big<256>, grid, dim3(512), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_cube_small(const CubeBatchArgs &a, int nchunks, int np, hipStream_t s)
{
    if (nchunks <= 0) return hipSuccess;
    const dim3 grid(nchunks);
    if (np == 16) hipLaunchKernelGGL((k_cube_small<16, false>), grid, dim3(256), 0, s, a);
    else if (np == 32) hipLaunchKernelGGL((k_cube_small<32, false>), grid, dim3(256), 0, s, a);
    else if (np == 64 && a.list == 1) hipLaunchKernelGGL((k_cube_small<64, true>), grid, dim3(256), 0, s, a);   // Jacobi
    else if (np == 64) hipLaunchKernelGGL((k_cube_small<64, false>), grid, dim3(256), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace bs
