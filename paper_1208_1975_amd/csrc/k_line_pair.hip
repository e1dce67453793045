// Chaotic block Gauss-Seidel on y- and z-lines with omega = 1, two x-cells
// per lane.
//
// The in-tile two-colour order of the chaotic sweep (colour (i + o) mod 2,
// colour 0 first) needs every line solved once with its colour-1
// neighbours' old values and every colour-1 line once with its colour-0
// neighbours' new values.  Here a lane holds the adjacent cells i = 2l and
// 2l + 1 of a row, one of each colour, so the tile (128 x-cells of one row o)
// is solved in two passes over full wavefronts: the colour-0 lines, then the
// colour-1 lines, each pass one exact line solve per lane (the partition
// method of k_line.hip: chunk solves with precomputed LU factors coupled
// through the interface system).
//
// With omega = 1 the update needs no old value of the line itself:
// u_new = M^{-1} b with b = h^2 f plus the off-line neighbour terms (and the
// ghosts at the line's two ends), the form of eq. (blockiteration1), the same
// map as u + M^{-1} r.  So the colour-0 pass forms b from the old colour-1
// cells, and the colour-1 pass adds the new colour-0 neighbours, held in
// registers (own cell) or taken from the adjacent lane (DPP).  Neighbours in
// other tiles (the tile's two x-edges and the rows o +- 1) are read as they
// are found, the asynchronous part of the scheme.  The colour-0 results wait
// in LDS, and both cells of a lane are stored together at the end.
#include "bs_internal.h"
#include "line_dev.h"

namespace bs {

template <int L>
__device__ __forceinline__ void line_pair_item(const LineArgs &a, const double *__restrict__ tabs, const WorkItem it,
                                               double *ends, double *ends2, double *v0s);

// LDS: the colour-0 results (L per lane) and two buffers of chunk ends.
template <int L, int MAXT>
__global__ void __launch_bounds__(MAXT) k_line_pair(LineArgs a, const double *__restrict__ tabs)
{
    extern __shared__ double smem[];
    const int nw = blockDim.x >> 6;
    double *v0s = smem;
    double *endb = smem + L * 64 * nw;
    for (int i = blockIdx.x; i < a.nitems; i += gridDim.x) {
        const WorkItem it = a.items[i];
        if (it.patch < 0) continue;   // padding of the dispatch order
        line_pair_item<L>(a, tabs, it, endb, endb + 2 * 64 * nw, v0s);
        __syncthreads();              // the next item reuses the LDS buffers
    }
}

template <int L>
__device__ __forceinline__ void line_pair_item(const LineArgs &a, const double *__restrict__ tabs, const WorkItem it,
                                               double *ends, double *ends2, double *v0s)
{
    const PatchDesc *pd = a.pd + it.patch;
    const int axis = a.axis;          // 1 or 2
    const int oaxis = 3 - axis;       // the other free axis
    const int nx = pd->n[0], ny = pd->n[1];
    const int no = pd->n[oaxis];
    const uint32_t sx = nx + 2, sy = sx * (uint32_t)(ny + 2);
    const uint32_t Sa = axis == 2 ? sy : sx;
    const uint32_t So = axis == 2 ? sx : sy;
    const uint32_t Fa = axis == 2 ? (uint32_t)nx * ny : (uint32_t)nx;
    const uint32_t Fo = axis == 2 ? (uint32_t)nx : (uint32_t)nx * ny;
    const double ex = pd->eps[0], ea = pd->eps[axis], eo = pd->eps[oaxis];
    const double h2 = pd->h2;
    // extrapolated line ends are folded into the line tables, not into b
    const double elo = ((pd->bc >> (2 * axis)) & 1) ? 0.0 : ea;
    const double ehi = ((pd->bc >> (2 * axis + 1)) & 1) ? 0.0 : ea;
    const LineTabRef tr = pd->line[axis][a.popt];
    const int Lr = tr.Lr, P = tr.P, Llast = tr.Llast;
    const double *tab = tabs + tr.off;
    const int nthr = blockDim.x;

    const int lane = threadIdx.x & 63;
    const int p = uniform_wave();
    const int nti = (nx + 127) >> 7;
    const int o = it.tile / nti;                          // wave-uniform row
    const int ia = ((it.tile - o * nti) << 7) + 2 * lane;  // the lane's cells ia, ia + 1
    const bool va = ia < nx, vb = ia + 1 < nx;
    const int pc = p < P ? p : P - 1;
    const int Lp = (pc == P - 1) ? Llast : Lr;
    const int t0 = pc * Lr;
    const bool chunk_ok = p < P;
    // colour-0 cell of the pair: ia when o is even, ia + 1 when o is odd
    const bool odd = (o & 1) != 0;
    // in-patch addresses for every lane (clamped; results of invalid cells are
    // not stored): a's cell, b's cell in u (the ghost x = nx when b is past the
    // row, so that it serves as a's right neighbour) and in f
    const int iac = va ? ia : nx - 1;
    const int ibu = ia + 1 < nx ? ia + 1 : nx;
    const int ibf = ia + 1 < nx ? ia + 1 : nx - 1;
    const char *ub = reinterpret_cast<const char *>(a.src + pd->uoff);
    const char *fbase = reinterpret_cast<const char *>(a.f + pd->foff);
    const uint32_t rowu = (uint32_t)(t0 + 1) * Sa + (uint32_t)(o + 1) * So;
    const uint32_t rowf = (uint32_t)t0 * Fa + (uint32_t)o * Fo;
    const uint32_t cua = 8u * (rowu + (uint32_t)(iac + 1)), cub = 8u * (rowu + (uint32_t)(ibu + 1));
    const uint32_t cfa = 8u * (rowf + (uint32_t)iac), cfb = 8u * (rowf + (uint32_t)ibf);
    const uint32_t Sa8 = 8u * Sa, So8 = 8u * So, Fa8 = 8u * Fa;
    // neighbours across the tile's x-edges: the cell left of a (lane 0) and
    // the cell right of b (the last lane, or the ghost x = nx)
    const bool edge_l = lane == 0, edge_r = lane == 63 || ia + 2 >= nx;
    const uint32_t cxr = 8u * (rowu + (uint32_t)(ia + 3 <= nx + 1 ? ia + 3 : nx + 1));

    // the ghosts beyond the line's two ends (global indices -1 and na): loaded
    // by every chunk from in-patch addresses, used by the first / last one
    const double glo_a = ldb(ub, cua - Sa8), glo_b = ldb(ub, cub - Sa8);
    const double ghi_a = ldb(ub, cua + (uint32_t)Lp * Sa8), ghi_b = ldb(ub, cub + (uint32_t)Lp * Sa8);
    const double wlo = t0 == 0 ? elo : 0.0, whi = pc == P - 1 ? ehi : 0.0;
    // the o-neighbours through shifted base pointers with the cells' offsets
    const char *ubm = ub - So8, *ubp = ub + So8;
    constexpr int B = 2;
    // b0: the colour-0 right-hand side (registers); the colour-1 right-hand
    // side without its in-tile x terms waits in the LDS slots that later hold
    // the colour-0 results
    double b0[L];
#pragma unroll
    for (int tb = 0; tb < L; tb += B) {
        double ua[B], ubv[B], fa[B], fb2[B], oma[B], omb[B], opa[B], opb[B], xl[B], xr[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const uint32_t tt = (uint32_t)((tb + k) < Lp ? (tb + k) : Lp - 1);
            const uint32_t ca = cua + tt * Sa8, cb = cub + tt * Sa8;
            ua[k] = ldb(ub, ca);
            ubv[k] = ldb(ub, cb);
            fa[k] = ldb(fbase, cfa + tt * Fa8);
            fb2[k] = ldb(fbase, cfb + tt * Fa8);
            oma[k] = ldb(ubm, ca);
            omb[k] = ldb(ubm, cb);
            opa[k] = ldb(ubp, ca);
            opb[k] = ldb(ubp, cb);
            xl[k] = ldb(ub, ca - 8u);
            xr[k] = ldb(ub, cxr + tt * Sa8);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int t = tb + k;
            // the cell left of ia (lane - 1's second cell) and right of ia + 1
            // (lane + 1's first cell); edge lanes read theirs from memory
            // the moves run under full EXEC: the empty asm pins their results
            // before the selects, which the compiler may otherwise turn into
            // branches around them
            double sl = lane_shift<-1>(ubv[k]), sr = lane_shift<+1>(ua[k]);
            asm volatile("" : "+v"(sl), "+v"(sr));
            const double lft = edge_l ? xl[k] : sl;
            const double rgt = edge_r ? xr[k] : sr;
            // line-axis ghosts at the line's two ends
            const double wl = t == 0 ? wlo : 0.0, wh = t == Lp - 1 ? whi : 0.0;
            const double ga = fma(wl, glo_a, wh * ghi_a), gb = fma(wl, glo_b, wh * ghi_b);
            const double rest_a = fma(h2, fa[k], fma(eo, oma[k] + opa[k], ga));
            const double rest_b = fma(h2, fb2[k], fma(eo, omb[k] + opb[k], gb));
            // colour-0 cell: old colour-1 x-neighbours; colour-1 cell: its
            // neighbour across a tile edge as found now, the in-tile colour-0
            // neighbours after the first solve
            const double bc0 = odd ? fma(ex, ua[k] + rgt, rest_b) : fma(ex, lft + ubv[k], rest_a);
            // (in an odd row whose last cell is a lane's first one, that
            // cell's right neighbour is the ghost x = nx, loaded as b's cell)
            const double far = odd ? (edge_l ? xl[k] : 0.0) + (vb ? 0.0 : ubv[k]) : (edge_r ? xr[k] : 0.0);
            const bool in = t < Lp;
            b0[t] = in ? bc0 : 0.0;
            v0s[t * nthr + threadIdx.x] = in ? fma(ex, far, odd ? rest_a : rest_b) : 0.0;
        }
        asm volatile("" ::: "memory");
    }
    const bool c0_ok = chunk_ok && (odd ? vb : va);
    const bool c1_ok = chunk_ok && (odd ? va : vb);
#pragma unroll
    for (int t = 0; t < L; ++t) b0[t] = c0_ok ? b0[t] : 0.0;

    // colour 0: solve and couple the chunks
    double y0, yl;
    chunk_solve_u<L, double>(b0, Lp, tab, tab + Lr, ea, y0, yl);
    ends[(p * 64 + lane) * 2 + 0] = y0;
    ends[(p * 64 + lane) * 2 + 1] = yl;
    __syncthreads();
    double bprev, anext;
    interface_terms_k<double>(as_const(tab), ends, Lr, P, pc, lane, bprev, anext);
    const __attribute__((address_space(4))) double *ev = as_const(tab) + (pc == P - 1 ? 4 * Lr : 2 * Lr);
    const __attribute__((address_space(4))) double *ew = ev + Lr;
    // colour-1 right-hand side: the new colour-0 x-neighbours in the tile (own
    // cell, and the adjacent lane's unless across a tile edge)
    const bool far_edge = odd ? edge_l : edge_r;
    double s1[L];
#pragma unroll
    for (int t = 0; t < L; ++t) {
        const double v0 = fma(anext, ew[t], fma(bprev, ev[t], b0[t]));
        s1[t] = v0s[t * nthr + threadIdx.x];   // each lane reads back only its own slots
        v0s[t * nthr + threadIdx.x] = v0;
        double nl = lane_shift<-1>(v0), nr = lane_shift<+1>(v0);
        asm volatile("" : "+v"(nl), "+v"(nr));
        const double other = far_edge ? 0.0 : (odd ? nl : nr);
        s1[t] = (c1_ok && t < Lp) ? fma(ex, v0 + other, s1[t]) : 0.0;
    }
    // colour 1: solve and couple (the second end buffer: no barrier needed
    // before its writes)
    const double *tab2 = tab;
    asm volatile("" : "+s"(tab2));
    chunk_solve_u<L, double>(s1, Lp, tab2, tab2 + Lr, ea, y0, yl);
    ends2[(p * 64 + lane) * 2 + 0] = y0;
    ends2[(p * 64 + lane) * 2 + 1] = yl;
    __syncthreads();
    interface_terms_k<double>(as_const(tab2), ends2, Lr, P, pc, lane, bprev, anext);
    const __attribute__((address_space(4))) double *ev2 = as_const(tab2) + (pc == P - 1 ? 4 * Lr : 2 * Lr);
    const __attribute__((address_space(4))) double *ew2 = ev2 + Lr;
    char *db = reinterpret_cast<char *>(a.dst + pd->uoff);
    if (chunk_ok) {
#pragma unroll
        for (int t = 0; t < L; ++t) {
            if (t < Lp) {
                const double v1 = fma(anext, ew2[t], fma(bprev, ev2[t], s1[t]));
                const double v0 = v0s[t * nthr + threadIdx.x];
                const double nva = odd ? v1 : v0, nvb = odd ? v0 : v1;
                if (va) *reinterpret_cast<double *>(db + cua + (uint32_t)t * Sa8) = nva;
                if (vb) *reinterpret_cast<double *>(db + cub + (uint32_t)t * Sa8) = nvb;
            }
        }
    }
}

template <int L, int MAXT>
static hipError_t launch_pair_t(const LineArgs &a, int grid, int nwaves, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((k_line_pair<L, MAXT>), dim3(grid), dim3(64 * nwaves), lds, s, a, a.tab);
    return hipGetLastError();
}

template <int L>
static hipError_t launch_pair_l(const LineArgs &a, int grid, int nwaves, size_t lds, hipStream_t s)
{
    const int t = 64 * nwaves;
    if (t <= 256) return launch_pair_t<L, 256>(a, grid, nwaves, lds, s);
    if (t <= 512) return launch_pair_t<L, 512>(a, grid, nwaves, lds, s);
    // 32-cell chunks: at most eight wavefronts (registers and LDS)
    if constexpr (L <= 16) return launch_pair_t<L, 1024>(a, grid, nwaves, lds, s);
    return hipErrorInvalidValue;
}

template <int L, int MAXT>
static hipError_t allow_pair_t()
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_line_pair<L, MAXT>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

hipError_t prepare_pair_kernels()
{
    static hipError_t done = hipErrorNotInitialized;
    if (done == hipSuccess) return done;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = allow_pair_t<8, 256>();
    if (e == hipSuccess) e = allow_pair_t<8, 512>();
    if (e == hipSuccess) e = allow_pair_t<8, 1024>();
    if (e == hipSuccess) e = allow_pair_t<16, 256>();
    if (e == hipSuccess) e = allow_pair_t<16, 512>();
    if (e == hipSuccess) e = allow_pair_t<16, 1024>();
    if (e == hipSuccess) e = allow_pair_t<32, 256>();
    if (e == hipSuccess) e = allow_pair_t<32, 512>();
    done = e;
    return e;
}

size_t pair_lds_bytes(int Lmax, int nwaves)
{
    return static_cast<size_t>(Lmax + 4) * 64 * static_cast<size_t>(nwaves) * sizeof(double);
}

hipError_t launch_line_pair(const LineArgs &a, int grid, int Lmax, int nwaves, hipStream_t s)
{
    if (a.colour_mode != 2 || a.rhs_mode || a.out_mode || a.f32 || a.axis == 0) return hipErrorInvalidValue;
    const size_t lds = pair_lds_bytes(Lmax, nwaves);
    switch (Lmax) {
    case 8: return launch_pair_l<8>(a, grid, nwaves, lds, s);
    case 16: return launch_pair_l<16>(a, grid, nwaves, lds, s);
    case 32: return launch_pair_l<32>(a, grid, nwaves, lds, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace bs
