// Line-block relaxation kernels (FP64): one sweep of every line along an axis.
//
// Per line (section 2, Algorithm 1; Algorithm 2's three steps):
//   1. block residual r = h^2 f - A u on the line's cells, from the current u
//      (off-line neighbours and ghosts included);
//   2. exact solve of the line block tridiag(-eps_a, d, -eps_a) du = r;
//   3. update dst = src + omega du.
//
// The exact solve is split across wavefronts: the line is cut into P chunks of
// Lr cells, each wavefront solves its chunk's tridiagonal block with
// precomputed LU factors (registers only), and the chunks are coupled exactly
// through the interface values: with y = T_chunk^{-1} r_chunk and the
// precomputed spikes v = T^{-1} e_0, w = T^{-1} e_last,
//   du_chunk = y + beta_prev * eps_a v + alpha_next * eps_a w,
// where beta_prev / alpha_next (the neighbouring chunks' end corrections) come
// from one row each of the precomputed inverse of the 2P x 2P interface
// system.  This is an exact reformulation of the tridiagonal solve (partition
// method), not an approximation.
#include <type_traits>

#include "bs_internal.h"
#include "line_dev.h"

namespace bs {

// ---------------------------------------------------------------------------
// y- and z-lines.  Lanes run along x (coalesced), a tile is tx lanes along x
// by 64/tx along the other free axis; wavefront p of the workgroup holds
// chunk p of all 64 lines.  With colour_mode, a tile holds lines of one
// colour only ((i + o) parity), which makes x stride 2.
//
// Register economy decides the speed of this kernel: a patch is addressed
// with wave-uniform base pointers and 32-bit byte offsets (one VGPR per
// address), the chunk factors and interface rows are wave-uniform and come
// through the scalar cache (read as constant memory), and u waits for the
// update in LDS (chunks of up to 16 cells; longer chunks read it again from
// memory).  The chunk ends take two LDS buffers, so consecutive items need
// no trailing barrier.
// ---------------------------------------------------------------------------

template <int L, int CM, bool F32, bool UCL>
__device__ __forceinline__ void line_strided_item(const LineArgs &a, const double *__restrict__ tabs,
                                                  const float *__restrict__ tabs32, const WorkItem it, double *ends,
                                                  double *ends2, double *ucs);

// Whether the update form keeps u in LDS for the update: 64 lanes x L cells
// per wavefront, at most 128 KiB (16 wavefronts of 16-cell chunks, or 8 of
// 32); longer chunks on more wavefronts read u again from memory.
template <int L, int MAXT, int CM>
constexpr bool uc_in_lds()
{
    return CM < 4 && (L <= 16 || (L == 32 && MAXT <= 512));
}

// A workgroup drains work items blockIdx.x, blockIdx.x + gridDim.x, ...: one
// item per workgroup when the grid covers the list, a persistent grid otherwise.
// LDS: the chunk values of u (L per lane, each lane reads back only its own)
// followed by two buffers of chunk ends.  CM: the kernel mode (0 all lines,
// 1 one colour per launch, 2 in-tile two-colour; 3 = 0 with f read
// nontemporally; 4 and 5 = 0 and 3 in the direct form below).  F32: the block
// solve in FP32 (residual and update stay FP64).
//
// Direct form of damped block Jacobi (modes 4, 5): with the line block M and
// b = h^2 f plus the off-line neighbour and line-end ghost terms, the update
// u + omega M^{-1}(b - M u) equals M^{-1}(omega b + (1 - omega) M u).  The
// kernel forms that right-hand side while loading (M u needs only the line's
// own cells, already loaded for the residual) and stores the solve's result
// as it is, so u never waits for the update: no LDS for it, and half the
// registers per cell of the long-chunk form that reads u again.  A line end
// at an extrapolated face (ghost = -u_0, folded into M's diagonal) takes the
// ghost's coefficient omega eps_a - eps_a instead of omega eps_a.
// The direct form with 32-cell chunks is held to 128 VGPRs (four waves per
// SIMD: two 8-wave workgroups per CU, one loading while the other solves).
template <int L, int MAXT, int CM, bool F32>
__global__ void __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu((CM >= 4 && L == 32) ? 4 : 1)))
k_line_strided(LineArgs a, const double *__restrict__ tabs, const float *__restrict__ tabs32)
{
    extern __shared__ double smem[];
    const int nw = blockDim.x >> 6;
    double *ucs = smem;
    constexpr bool UCL = uc_in_lds<L, MAXT, CM>();
    double *endb = smem + (UCL ? L * 64 * nw : 0);
    int buf = 0;
    for (int i = blockIdx.x; i < a.nitems; i += gridDim.x) {
        const WorkItem it = a.items[i];
        if (it.patch < 0) continue;   // padding of the dispatch order
        line_strided_item<L, CM, F32, UCL>(a, tabs, tabs32, it, endb + buf * (2 * 64 * nw),
                                           endb + (buf ^ 1) * (2 * 64 * nw), ucs);
        // one barrier per item alternates the buffers; the in-tile two-colour
        // mode uses both in every item behind two barriers
        if (CM != 2) buf ^= 1;
    }
}

template <int L, int CM, bool F32, bool UCL>
__device__ __forceinline__ void line_strided_item(const LineArgs &a, const double *__restrict__ tabs,
                                                  const float *__restrict__ tabs32, const WorkItem it, double *ends,
                                                  double *ends2, double *ucs)
{
    using T = typename std::conditional<F32, float, double>::type;
    const int nthr = blockDim.x;
    // the update form keeps u in LDS for the update when it fits (UCL,
    // uc_in_lds); otherwise it reads u again from memory
    constexpr bool kDirect = CM >= 4;
    constexpr bool kUcLds = UCL;
    constexpr bool kNtF = CM == 3 || CM == 5;
    const PatchDesc *pd = a.pd + it.patch;
    const int axis = a.axis;          // 1 or 2
    const int oaxis = 3 - axis;       // the other free axis
    const int nx = pd->n[0], ny = pd->n[1];
    const int no = pd->n[oaxis];
    const uint32_t sx = nx + 2, sy = sx * (uint32_t)(ny + 2);
    const uint32_t Sa = axis == 2 ? sy : sx;           // u strides (elements)
    const uint32_t So = axis == 2 ? sx : sy;
    const uint32_t Fa = axis == 2 ? (uint32_t)nx * ny : (uint32_t)nx;   // f strides
    const uint32_t Fo = axis == 2 ? (uint32_t)nx : (uint32_t)nx * ny;
    const double ex = pd->eps[0], ea = pd->eps[axis], eo = pd->eps[oaxis];
    const double d = 2.0 * (pd->eps[0] + pd->eps[1] + pd->eps[2]);
    const double h2 = pd->h2;
    const LineTabRef tr = pd->line[axis][a.popt];
    const int Lr = tr.Lr, P = tr.P, Llast = tr.Llast;
    const T *tab;
    if constexpr (F32)
        tab = tabs32 + tr.off;
    else
        tab = tabs + tr.off;

    const int lane = threadIdx.x & 63;
    const int p = uniform_wave();
    const int tx = a.tx, tyo = 64 / tx;
    const int li = lane % tx, lo = lane / tx;
    int i, o;
    if (CM == 1) {
        const int half = (nx + 1) >> 1;
        const int nti = (half + tx - 1) / tx;
        o = (it.tile / nti) * tyo + lo;
        i = 2 * ((it.tile % nti) * tx + li) + ((o + it.colour) & 1);
    } else {
        const int nti = (nx + tx - 1) / tx;
        o = (it.tile / nti) * tyo + lo;
        i = (it.tile % nti) * tx + li;
    }
    // lines next to an extrapolated face parallel to them are solved by the
    // boundary-line kernel (their block has a raised diagonal): skipped here
    const bool valid = (i < nx) && (o < no) && (p < P) && !offline_extrap(pd->bc, 0, i, nx, oaxis, o, no);
    // Inactive lanes and chunks read clamped, in-patch addresses so that every
    // load can be issued without a branch; their results are never stored.
    const int ic = i < nx ? i : nx - 1;
    const int oc = o < no ? o : no - 1;
    const int pc = p < P ? p : P - 1;
    const int Lp = (pc == P - 1) ? Llast : Lr;
    const int t0 = pc * Lr;
    // x-neighbours come from the adjacent lanes (DPP) unless the lane is at a
    // row edge of the tile or the patch, or lanes are colour-strided.  A lane
    // that needs one side from memory gets it with the batched loads; a lane
    // that needs both (colour-strided, or a one-lane row) takes one more load.
    const bool need_l = CM == 1 || li == 0;
    const bool need_r = CM == 1 || li == tx - 1 || i >= nx - 1;
    const bool both = need_l && need_r;

    const char *ub = reinterpret_cast<const char *>(a.src + pd->uoff);
    const char *fbase = reinterpret_cast<const char *>(a.f + pd->foff);
    const char *ubm = ub - 8u * So, *ubp = ub + 8u * So;   // the o-neighbours share u's offsets
    // byte offsets of this lane's first chunk cell in u and f
    const uint32_t cu = 8u * ((uint32_t)(ic + 1) + (uint32_t)(t0 + 1) * Sa + (uint32_t)(oc + 1) * So);
    const uint32_t cf = 8u * ((uint32_t)ic + (uint32_t)t0 * Fa + (uint32_t)oc * Fo);
    const uint32_t Sa8 = 8u * Sa, Fa8 = 8u * Fa;
    const uint32_t xo = need_l ? 0u - 8u : 8u;
    // Loads are issued in batches of B cells, each batch before any of its
    // values is used (the scheduling barriers keep the compiler from sinking
    // loads next to their uses).
    constexpr int B = L < 4 ? L : 4;
    double r[L];
    const double ulo = ldb(ub, cu - Sa8);
    const double uhi = ldb(ub, cu + (uint32_t)Lp * Sa8);
    // direct form: the residual's coefficients scaled by omega, (1 - omega) M u
    // added; in-line neighbours weigh (omega - 1) eps_a, a line-end ghost
    // omega eps_a (minus eps_a at an extrapolated end)
    const double om = a.omega;
    const double cx = kDirect ? om * ex : ex, co = kDirect ? om * eo : eo, ch2 = kDirect ? om * h2 : h2;
    const double cd = kDirect ? (1.0 - om) * d : -d;
    const double cn = kDirect ? (om - 1.0) * ea : ea;
    const double clo = (kDirect && t0 == 0) ? fma(om, ea, ((pd->bc >> (2 * axis)) & 1) ? -ea : 0.0) : cn;
    const double chi = (kDirect && pc == P - 1) ? fma(om, ea, ((pd->bc >> (2 * axis + 1)) & 1) ? -ea : 0.0) : cn;
    if (!kDirect && a.rhs_mode) {
#pragma unroll
        for (int t = 0; t < L; ++t) {
            r[t] = ldb(ub, cu + (uint32_t)(t < Lp ? t : Lp - 1) * Sa8);
            if (kUcLds) ucs[t * nthr + threadIdx.x] = r[t];
        }
    } else {
        // r = h^2 f + eps_o (o-neighbours) + eps_x (x-neighbours) + eps_a
        // (line neighbours) - d u, finished cell by cell as soon as the next
        // centre value has arrived, so only B + 1 centre values stay live
        // (the direct form's right-hand side the same way, with its own
        // coefficients)
        double uprev = ulo, ucur = 0.0, rpend = 0.0;
#pragma unroll
        for (int tb = 0; tb < L; tb += B) {
            double ub4[B], fb[B], om[B], op[B], xa[B];
#pragma unroll
            for (int k = 0; k < B; ++k) {
                const int t = tb + k;
                const uint32_t tt = (uint32_t)(t < Lp ? t : Lp - 1);
                const uint32_t c = cu + tt * Sa8;
                ub4[k] = ldb(ub, c);
                // CM 3 (Jacobi on data larger than the 256 MiB Infinity Cache):
                // f with a nontemporal load (measured 117 -> 102 us per 256^3
                // sweep; data that fits the cache, and the in-place schemes,
                // are slower with it)
                if constexpr (kNtF)
                    fb[k] = __builtin_nontemporal_load(reinterpret_cast<const double *>(fbase + (cf + tt * Fa8)));
                else
                    fb[k] = ldb(fbase, cf + tt * Fa8);
                om[k] = ldb(ubm, c);
                op[k] = ldb(ubp, c);
                xa[k] = ldb(ub, c + xo);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < B; ++k) {
                const int t = tb + k;
                if (kUcLds) ucs[t * nthr + threadIdx.x] = ub4[k];
                const double left = lane_shift<-1>(ub4[k]);
                const double right = lane_shift<+1>(ub4[k]);
                const double xs = (need_l ? xa[k] : left) + (need_r ? (need_l ? 0.0 : xa[k]) : right);
                const double rt = fma(cd, ub4[k], fma(cx, xs, fma(ch2, fb[k], co * (om[k] + op[k]))));
                // cell t-1 is complete now that u_t is known (beyond Lp the
                // upper neighbour is the chunk's far neighbour uhi)
                if (t > 0) {
                    if constexpr (kDirect)
                        r[t - 1] = fma(t == 1 ? clo : cn, uprev, fma(t < Lp ? cn : chi, t < Lp ? ub4[k] : uhi, rpend));
                    else
                        r[t - 1] = fma(ea, uprev + (t < Lp ? ub4[k] : uhi), rpend);
                }
                uprev = ucur;
                ucur = ub4[k];
                rpend = rt;
                if (t == 0) uprev = ulo;
            }
            // keep the next batch's loads below this point (bounded registers)
            asm volatile("" ::: "memory");
        }
        if constexpr (kDirect)
            r[L - 1] = fma(cn, uprev, fma(chi, uhi, rpend));
        else
            r[L - 1] = fma(ea, uprev + uhi, rpend);
        if (__builtin_amdgcn_ballot_w64(both) != 0) {
#pragma unroll
            for (int tb = 0; tb < L; tb += B) {
                double xb[B];
#pragma unroll
                for (int k = 0; k < B; ++k)
                    xb[k] = ldb(ub, cu + (uint32_t)((tb + k) < Lp ? (tb + k) : Lp - 1) * Sa8 + 8u);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int k = 0; k < B; ++k) r[tb + k] = fma(cx, both ? xb[k] : 0.0, r[tb + k]);
            }
        }
    }
    T rs[L];
#pragma unroll
    for (int t = 0; t < L; ++t) rs[t] = static_cast<T>(r[t]);
    T y0, yl;
    chunk_solve_u<L, T>(rs, Lp, tab, tab + Lr, static_cast<T>(ea), y0, yl);
    ends[(p * 64 + lane) * 2 + 0] = y0;
    ends[(p * 64 + lane) * 2 + 1] = yl;
    __syncthreads();   // every chunk's ends are in LDS; all reads of the tile's lines precede any write
    double uo[kUcLds ? 1 : L];
    if (!kUcLds && !kDirect && a.out_mode != 1) {
#pragma unroll
        for (int t = 0; t < L; ++t) uo[kUcLds ? 0 : t] = ldb(ub, cu + (uint32_t)(t < Lp ? t : Lp - 1) * Sa8);
    }
    T bprev, anext;
    interface_terms_k<T>(as_const(tab), ends, Lr, P, pc, lane, bprev, anext);
    const __attribute__((address_space(4))) T *ev = as_const(tab) + (pc == P - 1 ? 4 * Lr : 2 * Lr);
    const __attribute__((address_space(4))) T *ew = ev + Lr;
    char *db = reinterpret_cast<char *>(a.dst + pd->uoff);
    if (CM == 2) {
        // In-tile two-colour (chaotic GS): the solve above is exact for the
        // colour-0 lines ((i + o) even).  Every lane takes u + omega du (for
        // colour-1 lines that is the part of their solve due to the residual
        // as loaded; the line solve is linear), and the colour-1 lines then
        // solve for the residual change caused by their updated colour-0
        // neighbours inside the tile.  Neighbours in other tiles are read as
        // they were (the asynchronous part of the scheme).
        const bool red = ((i + o) & 1) == 0;
        const bool in_dn = lo > 0, in_up = lo < tyo - 1 && o + 1 < no;
#pragma unroll
        for (int t = 0; t < L; ++t) {
            const double du = static_cast<double>(fma(anext, ew[t], fma(bprev, ev[t], rs[t])));
            if (kUcLds) {
                double *us = ucs + t * nthr + threadIdx.x;
                *us = fma(om, du, *us);
            } else {
                uo[kUcLds ? 0 : t] = fma(om, du, uo[kUcLds ? 0 : t]);
            }
            const double dl = (red && valid) ? om * du : 0.0;
            const double cl = lane_shift<-1>(dl), cr = lane_shift<+1>(dl);
            double c = ex * ((need_l ? 0.0 : cl) + (need_r ? 0.0 : cr));
            if (tyo > 1) {
                const double cd = lane_get(dl, lane - tx < 0 ? lane : lane - tx);
                const double cu2 = lane_get(dl, lane + tx > 63 ? lane : lane + tx);
                c = fma(eo, (in_dn ? cd : 0.0) + (in_up ? cu2 : 0.0), c);
            }
            rs[t] = static_cast<T>((!red && t < Lp) ? c : 0.0);
        }
        // reload the factors rather than holding them in scalar registers
        // across both solves
        const T *tab2 = tab;
        asm volatile("" : "+s"(tab2));
        chunk_solve_u<L, T>(rs, Lp, tab2, tab2 + Lr, static_cast<T>(ea), y0, yl);
        ends2[(p * 64 + lane) * 2 + 0] = y0;
        ends2[(p * 64 + lane) * 2 + 1] = yl;
        __syncthreads();
        interface_terms_k<T>(as_const(tab2), ends2, Lr, P, pc, lane, bprev, anext);
        const __attribute__((address_space(4))) T *ev2 = as_const(tab2) + (pc == P - 1 ? 4 * Lr : 2 * Lr);
        const __attribute__((address_space(4))) T *ew2 = ev2 + Lr;
        if (valid) {
#pragma unroll
            for (int t = 0; t < L; ++t) {
                if (t < Lp) {
                    const double du = static_cast<double>(fma(anext, ew2[t], fma(bprev, ev2[t], rs[t])));
                    *reinterpret_cast<double *>(db + (cu + (uint32_t)t * Sa8)) =
                        fma(om, du, kUcLds ? ucs[t * nthr + threadIdx.x] : uo[kUcLds ? 0 : t]);
                }
            }
        }
        return;
    }
    if (valid) {
        // out_mode 2 (update form only): du itself to dst2 as well
        char *db2 = reinterpret_cast<char *>((a.out_mode == 2 ? a.dst2 : a.dst) + pd->uoff);
#pragma unroll
        for (int t = 0; t < L; ++t) {
            if (t < Lp) {
                const double du = static_cast<double>(fma(anext, ew[t], fma(bprev, ev[t], rs[t])));
                *reinterpret_cast<double *>(db + (cu + (uint32_t)t * Sa8)) =
                    (kDirect || a.out_mode == 1)
                        ? du
                        : fma(om, du, kUcLds ? ucs[t * nthr + threadIdx.x] : uo[kUcLds ? 0 : t]);
                if (!kDirect && a.out_mode == 2) *reinterpret_cast<double *>(db2 + (cu + (uint32_t)t * Sa8)) = du;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// x-lines (contiguous).  A workgroup owns 64 rows (lines); the residual of the
// tile is formed cooperatively with x-coalesced loads into LDS, each lane then
// solves its row's chunk from LDS in registers, and the update is written back
// coalesced.  With colour_mode the tile holds rows of one colour ((j+k) parity).
// ---------------------------------------------------------------------------
template <int L, int MAXT, bool F32>
__device__ __forceinline__ void line_x_item(const LineArgs &a, const float *__restrict__ tabs32, const WorkItem it,
                                            double *smem);

// F32: the block solve in FP32 (factors from the FP32 table copy, read
// through the scalar cache); residual and update stay FP64.
template <int L, int MAXT, bool F32>
__global__ void __launch_bounds__(MAXT) k_line_x(LineArgs a, const float *__restrict__ tabs32)
{
    extern __shared__ double smem[];
    for (int i = blockIdx.x; i < a.nitems; i += gridDim.x) {
        const WorkItem it = a.items[i];
        if (it.patch < 0) continue;   // padding of the dispatch order
        line_x_item<L, MAXT, F32>(a, tabs32, it, smem);
        __syncthreads();
    }
}

template <int L, int MAXT, bool F32>
__device__ __forceinline__ void line_x_item(const LineArgs &a, const float *__restrict__ tabs32, const WorkItem it,
                                            double *smem)
{
    const PatchDesc *pd = a.pd + it.patch;
    const int nx = pd->n[0], ny = pd->n[1], nz = pd->n[2];
    const int64_t sx = nx + 2, sy = sx * (int64_t)(ny + 2);
    const double ex = pd->eps[0], ey = pd->eps[1], ez = pd->eps[2];
    const double d = 2.0 * (ex + ey + ez);
    const double h2 = pd->h2;
    const LineTabRef tr = pd->line[0][a.popt];
    const int Lr = tr.Lr, P = tr.P, Llast = tr.Llast;
    const int tsz = line_table_size(Lr, P);
    const int sd = nx | 1;                 // odd row stride in LDS (bank spread)
    const double rnx = 1.0 / nx;
    const int nw = blockDim.x >> 6;

    double *tab = smem;
    double *ends = tab + ((tsz + 1) & ~1);
    double *rb = ends + 2 * 64 * nw;
    int64_t *rowu = reinterpret_cast<int64_t *>(rb + 64 * sd);   // per row: u offset of cell (0,j,k), -1 if outside
    int64_t *rowf = rowu + 64;
    for (int t = threadIdx.x; t < tsz; t += blockDim.x) tab[t] = a.tab[tr.off + t];
    if (threadIdx.x < 64) {
        const int rho = it.tile * 64 + (int)threadIdx.x;
        int j, k;
        if (a.colour_mode == 1) {
            const int M = (ny + 1) >> 1;
            k = rho / M;
            j = 2 * (rho % M) + ((k + it.colour) & 1);
        } else {
            k = rho / ny;
            j = rho % ny;
        }
        // rows next to an extrapolated y or z face belong to the boundary-line kernel
        const bool in = j < ny && k < nz && !offline_extrap(pd->bc, 1, j, ny, 2, k, nz);
        rowu[threadIdx.x] = in ? pd->uoff + (int64_t)(k + 1) * sy + (int64_t)(j + 1) * sx + 1 : -1;
        rowf[threadIdx.x] = in ? pd->foff + ((int64_t)k * ny + j) * nx : -1;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int w = uniform_wave();
    const double *s = a.src;
    const int ncell = 64 * nx;

    // phase 1: residuals of the tile into LDS (x-coalesced); four cells per
    // thread per round, rows outside the patch read a clamped in-patch row
    const int64_t safe_u = pd->uoff + sy + sx + 1;
    const int64_t safe_f = pd->foff;
    for (int i0 = threadIdx.x; i0 < ncell; i0 += 4 * (int)blockDim.x) {
        double res[4];
        int at[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int idx = i0 + m * (int)blockDim.x;
            const int idc = idx < ncell ? idx : ncell - 1;
            const int row = div_rd(idc, nx, rnx), i = idc - row * nx;
            const int64_t bu = rowu[row];
            at[m] = (idx < ncell && bu >= 0) ? row * sd + i : -1;
            const int64_t c = (bu >= 0 ? bu : safe_u) + i;
            const int64_t fc = (bu >= 0 ? rowf[row] : safe_f) + i;
            if (a.rhs_mode) {
                res[m] = s[c];
            } else {
                const double nb = ex * (s[c - 1] + s[c + 1]) + ey * (s[c - sx] + s[c + sx]) + ez * (s[c - sy] + s[c + sy]);
                res[m] = fma(-d, s[c], fma(h2, a.f[fc], nb));
            }
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
            if (at[m] >= 0) rb[at[m]] = res[m];
    }
    __syncthreads();

    // phase 2: lane = row, wavefront = chunk
    const int p = w;
    const bool valid = (rowu[lane] >= 0) && (p < P);
    const int Lp = (p == P - 1) ? Llast : Lr;
    const int t0 = p * Lr;
    using T = typename std::conditional<F32, float, double>::type;
    const T *tabT;
    if constexpr (F32)
        tabT = tabs32 + tr.off;
    else
        tabT = tab;
    T r[L];
    T y0 = 0, yl = 0;
    if (valid) {
#pragma unroll
        for (int t = 0; t < L; ++t)
            if (t < Lp) r[t] = static_cast<T>(rb[lane * sd + t0 + t]);
        if constexpr (F32)
            chunk_solve_u<L, T>(r, Lp, tabT, tabT + Lr, static_cast<T>(ex), y0, yl);
        else
            chunk_solve<L>(r, Lp, Lr, tab, tab + Lr, ex, y0, yl);
    }
    ends[(p * 64 + lane) * 2 + 0] = y0;
    ends[(p * 64 + lane) * 2 + 1] = yl;
    __syncthreads();
    if (valid) {
        T bprev, anext;
        interface_terms<T>(tabT, ends, Lr, P, p, lane, bprev, anext);
        const T *ev = tabT + (p == P - 1 ? 4 * Lr : 2 * Lr);
        const T *ew = ev + Lr;
#pragma unroll
        for (int t = 0; t < L; ++t)
            if (t < Lp) rb[lane * sd + t0 + t] = static_cast<double>(fma(anext, ew[t], fma(bprev, ev[t], r[t])));
    }
    __syncthreads();
    if (a.colour_mode == 2) {
        // In-tile two-colour (chaotic GS): the solve above is exact for the
        // colour-0 rows ((j + k) even); the colour-1 rows solve again for the
        // residual change caused by their updated colour-0 neighbours in this
        // tile (rows rho +- 1 along y, rho +- ny along z) and add it (the line
        // solve is linear).  Neighbours in other tiles are read as they were.
        const int rho = it.tile * 64 + lane;
        const int j = rho % ny, k = rho / ny;
        const bool black = ((j + k) & 1) != 0;
        const double om = a.omega;
        auto nbr = [&](int row, bool ok) -> int { return (ok && row >= 0 && row < 64 && rowu[row] >= 0) ? row : -1; };
        const int rjm = nbr(lane - 1, j > 0), rjp = nbr(lane + 1, j + 1 < ny);
        const int rkm = nbr(lane - ny, k > 0), rkp = nbr(lane + ny, k + 1 < nz);
        T r2[L];
        T z0 = 0, zl = 0;
        if (valid) {
#pragma unroll
            for (int t = 0; t < L; ++t) {
                double c = 0.0;
                if (black && t < Lp) {
                    const int x = t0 + t;
                    const double dy = (rjm >= 0 ? rb[rjm * sd + x] : 0.0) + (rjp >= 0 ? rb[rjp * sd + x] : 0.0);
                    const double dz = (rkm >= 0 ? rb[rkm * sd + x] : 0.0) + (rkp >= 0 ? rb[rkp * sd + x] : 0.0);
                    c = om * fma(ey, dy, ez * dz);
                }
                r2[t] = static_cast<T>(c);
            }
            if constexpr (F32)
                chunk_solve_u<L, T>(r2, Lp, tabT, tabT + Lr, static_cast<T>(ex), z0, zl);
            else
                chunk_solve<L>(r2, Lp, Lr, tab, tab + Lr, ex, z0, zl);
        }
        ends[(p * 64 + lane) * 2 + 0] = z0;
        ends[(p * 64 + lane) * 2 + 1] = zl;
        __syncthreads();   // every colour-0 value above was read before any colour-1 row changes
        if (valid && black) {
            T bprev, anext;
            interface_terms<T>(tabT, ends, Lr, P, p, lane, bprev, anext);
            const T *ev = tabT + (p == P - 1 ? 4 * Lr : 2 * Lr);
            const T *ew = ev + Lr;
#pragma unroll
            for (int t = 0; t < L; ++t)
                if (t < Lp) rb[lane * sd + t0 + t] += static_cast<double>(fma(anext, ew[t], fma(bprev, ev[t], r2[t])));
        }
        __syncthreads();
    }

    // phase 3: coalesced update (all reads of the tile happened before the barriers)
    const double om = a.omega;
    for (int i0 = threadIdx.x; i0 < ncell; i0 += 4 * (int)blockDim.x) {
        double val[4];
        int64_t dst[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int idx = i0 + m * (int)blockDim.x;
            const int idc = idx < ncell ? idx : ncell - 1;
            const int row = div_rd(idc, nx, rnx), i = idc - row * nx;
            const int64_t bu = rowu[row];
            dst[m] = (idx < ncell && bu >= 0) ? bu + i : -1;
            val[m] = a.out_mode ? rb[row * sd + i] : fma(om, rb[row * sd + i], s[(bu >= 0 ? bu : safe_u) + i]);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
            if (dst[m] >= 0) a.dst[dst[m]] = val[m];
    }
}

template <int L, int MAXT, bool F32>
static void launch_strided_p(const LineArgs &a, int grid, int nwaves, size_t lds, hipStream_t s)
{
    const dim3 g(grid), b(64 * nwaves);
    switch (a.colour_mode) {
    case 0:
        if constexpr (!F32) {
            if (a.direct) {
                if (a.f_stream)
                    hipLaunchKernelGGL((k_line_strided<L, MAXT, 5, false>), g, b, lds, s, a, a.tab, a.tab32);
                else
                    hipLaunchKernelGGL((k_line_strided<L, MAXT, 4, false>), g, b, lds, s, a, a.tab, a.tab32);
                break;
            }
        }
        if (a.f_stream) {
            hipLaunchKernelGGL((k_line_strided<L, MAXT, 3, F32>), g, b, lds, s, a, a.tab, a.tab32);
        } else {
            hipLaunchKernelGGL((k_line_strided<L, MAXT, 0, F32>), g, b, lds, s, a, a.tab, a.tab32);
        }
        break;
    case 1: hipLaunchKernelGGL((k_line_strided<L, MAXT, 1, F32>), g, b, lds, s, a, a.tab, a.tab32); break;
    default: hipLaunchKernelGGL((k_line_strided<L, MAXT, 2, F32>), g, b, lds, s, a, a.tab, a.tab32); break;
    }
}

template <int L, int MAXT>
static hipError_t launch_strided_t(const LineArgs &a, int grid, int nwaves, size_t lds, hipStream_t s)
{
    if (a.colour_mode < 0 || a.colour_mode > 2) return hipErrorInvalidValue;
    if (a.f32)
        launch_strided_p<L, MAXT, true>(a, grid, nwaves, lds, s);
    else
        launch_strided_p<L, MAXT, false>(a, grid, nwaves, lds, s);
    return hipGetLastError();
}

template <int L, int MAXT>
static hipError_t launch_x_t(const LineArgs &a, int grid, int nwaves, size_t lds, hipStream_t s)
{
    if (a.f32)
        hipLaunchKernelGGL((k_line_x<L, MAXT, true>), dim3(grid), dim3(64 * nwaves), lds, s, a, a.tab32);
    else
        hipLaunchKernelGGL((k_line_x<L, MAXT, false>), dim3(grid), dim3(64 * nwaves), lds, s, a, a.tab32);
    return hipGetLastError();
}

// The thread bound of an instantiation is the smallest of 256/512/1024 that
// holds the workgroup, so a small workgroup may use more registers per lane.
#define BS_DISPATCH(FN)                                                                  \
    template <int L>                                                                     \
    static hipError_t FN##_b(const LineArgs &a, int nitems, int nwaves, size_t lds,     \
                             hipStream_t s)                                              \
    {                                                                                    \
        const int t = 64 * nwaves;                                                       \
        if (t <= 256) return FN<L, 256>(a, nitems, nwaves, lds, s);                      \
        if (t <= 512) return FN<L, 512>(a, nitems, nwaves, lds, s);                      \
        if (t <= 1024) return FN<L, 1024>(a, nitems, nwaves, lds, s);                    \
        return hipErrorInvalidValue;                                                     \
    }
BS_DISPATCH(launch_strided_t)
BS_DISPATCH(launch_x_t)
#undef BS_DISPATCH

// Allow the large-LDS line kernels (x-lines of up to 256 cells) once per
// process, so that no attribute call ever happens inside a graph capture.
template <int L, bool F32>
static hipError_t allow_all_p()
{
    hipError_t e = hipSuccess;
    const void *ks[] = {reinterpret_cast<const void *>(k_line_x<L, 256, F32>),
                        reinterpret_cast<const void *>(k_line_x<L, 512, F32>),
                        reinterpret_cast<const void *>(k_line_x<L, 1024, F32>),
                        reinterpret_cast<const void *>(k_line_strided<L, 256, 0, F32>),
                        reinterpret_cast<const void *>(k_line_strided<L, 512, 0, F32>),
                        reinterpret_cast<const void *>(k_line_strided<L, 1024, 0, F32>),
                        reinterpret_cast<const void *>(k_line_strided<L, 256, 1, F32>),
                        reinterpret_cast<const void *>(k_line_strided<L, 512, 1, F32>),
                        reinterpret_cast<const void *>(k_line_strided<L, 1024, 1, F32>),
                        reinterpret_cast<const void *>(k_line_strided<L, 256, 2, F32>),
                        reinterpret_cast<const void *>(k_line_strided<L, 512, 2, F32>),
                        reinterpret_cast<const void *>(k_line_strided<L, 1024, 2, F32>),
                        reinterpret_cast<const void *>(k_line_strided<L, 256, 3, F32>),
                        reinterpret_cast<const void *>(k_line_strided<L, 512, 3, F32>),
                        reinterpret_cast<const void *>(k_line_strided<L, 1024, 3, F32>)};
    for (const void *k : ks) {
        hipError_t r = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (r != hipSuccess) e = r;
    }
    return e;
}

template <int L>
static hipError_t allow_all_t()
{
    hipError_t e = allow_all_p<L, false>();
    return e == hipSuccess ? allow_all_p<L, true>() : e;
}

hipError_t prepare_line_kernels()
{
    static hipError_t done = hipErrorNotInitialized;
    if (done == hipSuccess) return done;
    hipError_t e = allow_all_t<8>();
    if (e == hipSuccess) e = allow_all_t<16>();
    if (e == hipSuccess) e = allow_all_t<32>();
    if (e == hipSuccess) e = allow_all_t<64>();
    done = e;
    return e;
}

// Workgroups of one line-kernel instantiation that a compute unit holds at
// once (registers, LDS and waves permitting); 1 if the query fails.
template <typename K>
static int occupancy_of(K kern, int threads, size_t lds)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, threads, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return n > 0 ? n : 1;
}

template <int L, int MAXT>
static int line_occupancy_t(int axis, int threads, size_t lds, int colour_mode, int f32)
{
    if (axis == 0)
        return f32 ? occupancy_of(k_line_x<L, MAXT, true>, threads, lds)
                   : occupancy_of(k_line_x<L, MAXT, false>, threads, lds);
    // the chaotic mode is the one whose dispatch depends on it
    if (colour_mode == 2)
        return f32 ? occupancy_of(k_line_strided<L, MAXT, 2, true>, threads, lds)
                   : occupancy_of(k_line_strided<L, MAXT, 2, false>, threads, lds);
    if (colour_mode == 1)
        return f32 ? occupancy_of(k_line_strided<L, MAXT, 1, true>, threads, lds)
                   : occupancy_of(k_line_strided<L, MAXT, 1, false>, threads, lds);
    return f32 ? occupancy_of(k_line_strided<L, MAXT, 0, true>, threads, lds)
               : occupancy_of(k_line_strided<L, MAXT, 0, false>, threads, lds);
}

template <int L>
static int line_occupancy_b(int axis, int nwaves, size_t lds, int colour_mode, int f32)
{
    const int t = 64 * nwaves;
    if (t <= 256) return line_occupancy_t<L, 256>(axis, t, lds, colour_mode, f32);
    if (t <= 512) return line_occupancy_t<L, 512>(axis, t, lds, colour_mode, f32);
    return line_occupancy_t<L, 1024>(axis, t, lds, colour_mode, f32);
}

int line_occupancy(int axis, int Lmax, int nwaves, size_t lds, int colour_mode, int f32)
{
    switch (Lmax) {
    case 8: return line_occupancy_b<8>(axis, nwaves, lds, colour_mode, f32);
    case 16: return line_occupancy_b<16>(axis, nwaves, lds, colour_mode, f32);
    case 32: return line_occupancy_b<32>(axis, nwaves, lds, colour_mode, f32);
    default: return line_occupancy_b<64>(axis, nwaves, lds, colour_mode, f32);
    }
}

hipError_t launch_line_strided(const LineArgs &a, int nitems, int Lmax, int nwaves, size_t lds,
                               hipStream_t s)
{
    switch (Lmax) {
    case 8: return launch_strided_t_b<8>(a, nitems, nwaves, lds, s);
    case 16: return launch_strided_t_b<16>(a, nitems, nwaves, lds, s);
    case 32: return launch_strided_t_b<32>(a, nitems, nwaves, lds, s);
    case 64: return launch_strided_t_b<64>(a, nitems, nwaves, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_line_x(const LineArgs &a, int nitems, int Lmax, int nwaves, size_t lds, hipStream_t s)
{
    switch (Lmax) {
    case 8: return launch_x_t_b<8>(a, nitems, nwaves, lds, s);
    case 16: return launch_x_t_b<16>(a, nitems, nwaves, lds, s);
    case 32: return launch_x_t_b<32>(a, nitems, nwaves, lds, s);
    case 64: return launch_x_t_b<64>(a, nitems, nwaves, lds, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace bs
