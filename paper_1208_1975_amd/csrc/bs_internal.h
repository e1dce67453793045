// Internal definitions shared by the library's host code and HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace bs {

// Chunk counts a line may be split into (one wavefront per chunk).  A line of
// n cells split for P_req chunks uses chunks of Lr = ceil(n / P_req) cells,
// P = ceil(n / Lr) <= P_req chunks, the last one Llast = n - (P-1) Lr long.
constexpr int kNumPOpt = 5;
constexpr int kPOpts[kNumPOpt] = {1, 2, 4, 8, 16};
constexpr int kMaxChunkLen = 64;   // largest Lr a kernel instantiation holds in registers
constexpr int kXregMaxN = 64;      // longest x-line of the register x-line kernel (16 lanes x 4 cells)

struct LineTabRef {
    int64_t off;   // offset in doubles into the table buffer, -1 if not built
    int32_t Lr, P, Llast, pad;
};

// Line table layout (doubles), chunk length Lr, P chunks:
//   g[Lr]   forward-elimination multipliers  eps_a / m_{t-1}   (g[0] = 0)
//   q[Lr]   reciprocal pivots                1 / m_t
//   evF[Lr], ewF[Lr]  eps_a * T^{-1} e_0 and eps_a * T^{-1} e_{Lr-1}, full chunks
//   evT[Lr], ewT[Lr]  the same for the last chunk (length Llast), zero padded
//   Kb[P][2P]  row of the inverse interface system giving the previous
//              chunk's last correction (zero row for chunk 0)
//   Ka[P][2P]  row giving the next chunk's first correction (zero for the last)
__host__ __device__ inline int line_table_size(int Lr, int P) { return 6 * Lr + 4 * P * P; }

// Plane table (per patch, per normal axis): orthonormal DST-I bases of the two
// in-plane axes (a < b) and the eigenvalue grid of the plane block.
struct PlaneTabRef {
    int64_t off;       // offset in doubles, -1 if not built
    int32_t na, nb;    // in-plane sizes, na = lower axis
};

struct PatchDesc {
    int32_t n[3];          // nx, ny, nz
    int32_t bc;            // extrapolated faces: bit 2a = low face of axis a, bit 2a+1 = high face
    int64_t uoff, foff;    // element offsets of this patch in u and f
    double eps[3];
    double h2;
    LineTabRef line[3][kNumPOpt];
    PlaneTabRef plane[3];
};

// One unit of work for a launch: (patch, tile, colour).
struct WorkItem {
    int32_t patch, tile, colour, pad;
};

// Arguments of the line-relaxation kernels.
struct LineArgs {
    const double *src;      // u read (old iterate)
    double *dst;            // written (== src for the Gauss-Seidel schemes)
    const double *f;
    const PatchDesc *pd;
    const double *tab;
    const WorkItem *items;
    int32_t axis;
    int32_t popt;           // index into kPOpts of the table set in use
    int32_t tx;             // lanes per row along the fast free axis (strided kernel)
    int32_t colour_mode;    // 0: every line; 1: only lines of the item's colour
    int32_t nitems;         // work items; a workgroup takes items blockIdx.x, +gridDim.x, ...
    int32_t rhs_mode;       // 0: right-hand side = residual h^2 f - A src; 1: = src itself (f unused)
    int32_t out_mode;       // 0: dst = src + omega du; 1: dst = du (the block solve alone);
                            // 2 (y/z lines, colour mode 0): dst = src + omega du and dst2 = du
    double omega;
    const float *tab32;     // FP32 copy of tab (same offsets)
    int32_t f32;            // 1: block solve in FP32 (residual and update stay FP64)
    int32_t f_stream;       // 1: colour mode 0 reads f with nontemporal loads (data beyond the Infinity Cache)
    int32_t direct;         // 1: colour mode 0 on y/z lines in the direct form dst = M^{-1}(omega b + (1 - omega) M src)
    double *dst2;           // out_mode 2: receives du
};
constexpr int64_t kMallBytes = 256ll << 20;   // MI355X Infinity Cache

// Residual / adjoint tile (one workgroup): columns x0.., y0.. of a patch
// marched along z over planes z0 .. z1 - 1.
struct ResidTile {
    int32_t patch, x0, y0, z0, z1;
};
constexpr int kResidPlanes = 64;      // planes per tile, halved while a patch set has too few tiles
constexpr int kResidMinTiles = 1024;  // about four workgroups per CU

struct ResidArgs {
    const double *u;
    const double *f;
    double *r;              // may be null
    double *partial;        // per-tile partial sums of r^2 (may be null)
    const PatchDesc *pd;
    const ResidTile *tiles;
    float *e32;                   // optional FP32 copy of r (f layout), may be null
    unsigned short *e16;          // optional BF16 copy of r (bit patterns), may be null
    float *r32;                   // optional FP32 r (f layout; the BF16 plane defect's input), may be null
};

// Host launchers (defined in the .hip files).
// grid: workgroups launched (each drains items blockIdx.x, +grid, ... < a.nitems)
hipError_t launch_line_strided(const LineArgs &a, int grid, int Lmax, int nwaves, size_t lds, hipStream_t s);
hipError_t launch_line_x(const LineArgs &a, int grid, int Lmax, int nwaves, size_t lds, hipStream_t s);
hipError_t launch_line_xr(const LineArgs &a, int grid, int nwaves, hipStream_t s);
// x-lines of up to 64 cells marched along z: items of rows x planes (a.tx =
// planes per item); colour_mode 0 (Jacobi) or 2 (chaotic GS).
hipError_t launch_line_xz(const LineArgs &a, int grid, int nwaves, hipStream_t s);
// Chaotic GS on y/z lines with omega = 1, two x-cells per lane (colour-0 lines,
// then colour-1 lines, one solve each); items of 128 x-cells by one row.
hipError_t launch_line_pair(const LineArgs &a, int grid, int Lmax, int nwaves, hipStream_t s);
hipError_t prepare_pair_kernels();
size_t pair_lds_bytes(int Lmax, int nwaves);
int line_xz_occupancy(int nwaves, int cm, int f32);
// Rows of one z-marching x-line item.
__host__ __device__ inline int xz_item_rows(int nx, int nwaves) { return nwaves * 4 * (16 / ((nx + 3) >> 2)); }
hipError_t prepare_line_kernels();
// Workgroups per compute unit that a line-kernel configuration can hold at once.
int line_occupancy(int axis, int Lmax, int nwaves, size_t lds, int colour_mode, int f32);
int line_xr_occupancy(int nwaves, int f32);
hipError_t launch_residual(const ResidArgs &a, int ntiles, hipStream_t s);
hipError_t launch_residual_final(const double *partial, const int32_t *patch_first_block,
                                 int npatch, double *out, hipStream_t s);
hipError_t launch_ghost_copy(const double *src, double *dst, const PatchDesc *pd, int npatch,
                             hipStream_t s);
hipError_t launch_interior_copy(const double *src, double *dst, const PatchDesc *pd, int npatch,
                                hipStream_t s);


// n / d for 0 <= n < 2^31 and d >= 1, given rd = 1.0 / d: the double product
// is within 1e-6 of the quotient, so one correction step makes it exact (a
// 32-bit integer division is some forty instructions on the GPU).
__device__ __forceinline__ int div_rd(int n, int d, double rd)
{
    int q = static_cast<int>(static_cast<double>(n) * rd);
    const int r = n - q * d;
    q += r >= d ? 1 : 0;
    q -= r < 0 ? 1 : 0;
    return q;
}

// Logical block of workgroup b out of nb: the hardware hands workgroup b to
// XCD b mod 8, so each XCD receives a contiguous range of logical blocks and
// neighbouring cells share that XCD's L2.  A bijection on [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int full = nb & ~7;
    if (b >= full) return b;
    return (b & 7) * (full >> 3) + (b >> 3);
}

// Geometric cube blocks (k_cube.hip), nblk equally shaped blocks of nb cells;
// cell c of block b is u[ubase[b] + uoff[c]] and f[fbase[b] + foff[c]].
//   launch_cube_resid: residuals into R[block][cell] (any nb).
struct CubeArgs {
    const double *u;
    const double *f;
    double *R;
    const int64_t *ubase, *fbase;
    const int32_t *uoff, *foff;
    int32_t nb, nblk, per;      // cells per block, blocks, blocks per workgroup
    int64_t sy, sz;             // u strides of y and z
    double ex, ey, ez, h2;
};
constexpr int kCubeSmallCells = 64;
hipError_t launch_cube_resid(const CubeArgs &a, hipStream_t s);

//   launch_cube_small: blocks of nb <= 64 cells of any number of groups in one
//   launch, fused (residuals, product with the inverse ainv (nb x nb,
//   row-major), update dst = u + omega du): one workgroup per chunk of at most
//   64 consecutive blocks of one group's list; np = 16, 32 or 64, the same
//   rounding of nb for every group of the launch.
struct CubeGroupDev {
    const double *ainv;
    const int32_t *uoff, *foff;
    const int64_t *ubase[2], *fbase[2];   // [0] colour-major list, [1] colour-free (Jacobi) list
    int32_t nb, pad;
    int64_t sy, sz;
    double ex, ey, ez, h2;
};
struct CubeChunk {
    int32_t group, first, end, pad;      // blocks [first, end) of the group's list
};
struct CubeBatchArgs {
    const double *u;
    double *dst;
    const double *f;
    const CubeGroupDev *groups;
    const CubeChunk *chunks;
    int32_t list;                        // index into ubase / fbase
    double omega;
};
hipError_t launch_cube_small(const CubeBatchArgs &a, int nchunks, int np, hipStream_t s);
//   launch_cube_big: blocks of 65..256 cells, fused likewise: one workgroup of
//   512 threads per chunk of at most 32 consecutive blocks; np = 128 or 256
//   (nb rounded up); the stored inverse must be symmetric.  Larger blocks
//   take launch_cube_resid and the FP64 product with the gather epilogue.
constexpr int kCubeBigChunk = 32;
hipError_t launch_cube_big(const CubeBatchArgs &a, int nchunks, int np, hipStream_t s);

// Ghost updates (k_ghost.hip).  One face operation copies the m1 x m2 cells
// of a layer: dst[d0 + a*d1 + b*d2] = sign * u[s0 + a*s1 + b*s2] (element
// offsets into the patch set's u).  Exchange between face-adjacent patches is
// a copy (sign +1) of the neighbour's first interior layer into a ghost layer;
// an extrapolated face is its own interior layer negated (sign -1).
struct FaceOp {
    int64_t d0, s0;
    int32_t d1, d2, s1, s2;
    int32_t m1, m2;
    double sign;
};
// A launch item: cells [first, first + count) of op `op` (in a-fastest order).
struct FaceItem {
    int32_t op, first, count, pad;
};
constexpr int kFaceItemCells = 2048;
hipError_t launch_face_ops(double *u, const FaceOp *ops, const FaceItem *items, int nitems, hipStream_t s);

// Lines next to an extrapolated face parallel to them: their block carries the
// folded ghosts on its whole diagonal, so they are solved one line per thread
// (Thomas with on-the-fly pivots) instead of by the chunked kernels.  p, q:
// the line's indices along the two other axes (lower axis first).
__host__ __device__ inline bool offline_extrap(int bc, int b, int p, int nb, int c, int q, int nc)
{
    return (((bc >> (2 * b)) & 1) && p == 0) || (((bc >> (2 * b + 1)) & 1) && p == nb - 1) ||
           (((bc >> (2 * c)) & 1) && q == 0) || (((bc >> (2 * c + 1)) & 1) && q == nc - 1);
}
struct BLineItem {
    int32_t patch, p, q, colour;
};
struct BLineArgs {
    const double *src;
    double *dst;
    const double *f;
    const PatchDesc *pd;
    const BLineItem *items;
    double *scratch;          // 2 * maxlen * nlines doubles: [2t + 1][line] residual, then eliminated rhs
    double *fac;              // 2 * maxlen * nlines doubles: [2t][line] multiplier eps_a / m_{t-1}, [2t + 1][line] 1 / m_t
    int32_t axis, nitems, nlines, first;   // items [first, first + nitems) of nlines
    double omega;
};
// Two launches: the lines' residuals one cell per thread, then the solves one
// line per thread (maxlen: the longest line of the set along the axis).
hipError_t launch_bline(const BLineArgs &a, int maxlen, hipStream_t s);
// The lines' LU factors (they depend on eps and the faces only), once per
// patch set and axis: one line per thread, every item of a.items.
hipError_t launch_bline_factors(const BLineArgs &a, hipStream_t s);

// Multigrid transfers (k_mg.hip), per patch: pf / pc the fine / coarse
// descriptors, max_cells the largest coarse (restriction) or fine
// (prolongation) patch.
//   restriction:   fc = mean of the 2x2x2 fine values of d / h_fine^2 (f layouts)
//   prolongation:  uf += trilinear interpolation of uc (u layouts); beyond a
//                  face in bc the coarse value is the reflected one, negated
hipError_t launch_restrict(const double *d, double *fc, const PatchDesc *pf, const PatchDesc *pc, int npatch,
                           int64_t max_cells, hipStream_t s);
hipError_t launch_prolong_add(const double *uc, double *uf, const PatchDesc *pf, const PatchDesc *pc, int npatch,
                              int64_t max_cells, int bc, hipStream_t s);

// Adjoint of damped Jacobi line sweeps (k_adjoint.hip).
hipError_t launch_fill(double *x, int64_t n, double v, hipStream_t s);
hipError_t launch_adj_init(const double *gK, double *gbar, const PatchDesc *pd, int npatch, hipStream_t s);
// spans: bit b set when the blocks span axis b (lines along a: 1 << a;
// planes normal to c: the other two bits), which decides dM/deps_b.
hipError_t launch_adj_step(const double *lam, const double *U, const double *w, double *gbar, double *gf,
                           double *acc, const PatchDesc *pd, const ResidTile *tiles, int ntiles, int spans,
                           double omega, hipStream_t s);
// Interior of a u-layout field into f layout (dst[f cell] = src[u cell]).
hipError_t launch_u_to_f(const double *src, double *dst, const PatchDesc *pd, int npatch, hipStream_t s);
hipError_t launch_eps_final(const double *acc, const int32_t *first_block, int npatch, double omega, double *out,
                            hipStream_t s);

}  // namespace bs
