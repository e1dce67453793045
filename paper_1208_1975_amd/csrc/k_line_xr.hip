// x-line relaxation with the lines held in registers (lines of up to 64 cells).
//
// Lanes run along x: a line of nx cells occupies ge = ceil(nx / 4) lanes of
// one 16-lane DPP row, four consecutive cells per lane, so loads and stores
// are x-contiguous and the tile needs no transposition through LDS.  A row of
// 16 lanes holds 16 / ge lines, a wavefront four rows of lanes.
//
// Per line (section 2, Algorithm 2's three steps): block residual from the
// current u, exact solve of tridiag(-eps_x, d, -eps_x), update.  The solve is
// the Thomas algorithm with the line's own LU factors (pivots m_t, m_0 = d,
// m_t = d - eps_x^2 / m_{t-1}); its two first-order recurrences
//     z_t = r_t + (eps_x / m_{t-1}) z_{t-1}      forward elimination
//     x_t = (z_t + eps_x x_{t+1}) / m_t          back substitution
// run over each lane's four cells from a zero carry, and the carries between
// the lanes of a line come from a log-step scan of the affine maps
// carry_out = b + a carry_in across the lanes (DPP row shifts by 1, 2, 4, 8).
// The multipliers a (products of the recurrence coefficients over a lane's
// cells, and their scan partial products) depend only on the patch and are
// formed once per work item.  This is the same LU solve, reassociated.
//
// Chaotic GS (colour mode 2) updates the tile's rows of colour 0 ((j + k)
// even) first and then, after a workgroup barrier (which makes those stores
// visible to the workgroup), the rows of colour 1, which read the new values;
// rows of other tiles are read as they are found.
#include <type_traits>

#include "bs_internal.h"

namespace bs {

namespace {

template <int CTRL>
__device__ __forceinline__ double dpp64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

// Value of lane l - S (from_left) or l + S (from_right) of the same 16-lane
// row; zero where that lane is outside the row.
template <int S, typename T>
__device__ __forceinline__ T from_left(T v)
{
    if constexpr (std::is_same<T, float>::value)
        return dpp32<0x110 + S>(v);   // row_shr:S
    else
        return dpp64<0x110 + S>(v);
}

template <int S, typename T>
__device__ __forceinline__ T from_right(T v)
{
    if constexpr (std::is_same<T, float>::value)
        return dpp32<0x100 + S>(v);   // row_shl:S
    else
        return dpp64<0x100 + S>(v);
}

__device__ __forceinline__ double ldb(const char *base, uint32_t off)
{
    return *reinterpret_cast<const double *>(base + off);
}

}  // namespace

template <bool F32>
__global__ void __launch_bounds__(256) k_line_xr(LineArgs a)
{
    using T = typename std::conditional<F32, float, double>::type;
    __shared__ int rows[64];     // colour mode 2: the tile's rows, colour 0 first
    __shared__ int ncnt[2];
    // per position g of a lane in its line: g_t, q_t of its four cells, the
    // forward and backward scan multipliers of steps 1, 2, 4, 8 (zero where
    // the partner lane is not in the line), and 1/0 flags for a left / right
    // neighbour lane.  Every select below that feeds on a DPP result is free of
    // loads, so the compiler keeps the cross-lane moves under full EXEC.
    __shared__ T xt[18][16];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int nw = blockDim.x >> 6;
    const int cm = a.colour_mode;

    for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
        const WorkItem it = a.items[item];
        if (it.patch < 0) continue;   // padding of the dispatch order
        const PatchDesc *pd = a.pd + it.patch;
        const int nx = pd->n[0], ny = pd->n[1], nz = pd->n[2];
        const uint32_t sx = nx + 2, sy = sx * (uint32_t)(ny + 2);
        const double ex = pd->eps[0], ey = pd->eps[1], ez = pd->eps[2];
        const double d = 2.0 * (ex + ey + ez);
        const double h2 = pd->h2;
        const int64_t toff = pd->line[0][0].off;   // one chunk: the line's own LU factors

        // lane -> (line slot, position in the line)
        const int ge = (nx + 3) >> 2;   // lanes per line
        const int lpr = 16 / ge;        // lines per 16-lane row
        const int lpw = 4 * lpr;        // lines per wavefront and pass
        const int q16 = lane & 15;
        const int seg = q16 / ge;
        const int g = q16 - seg * ge;
        const int slot = (lane >> 4) * lpr + seg;
        const bool lane_ok = seg < lpr;
        const int i0 = 4 * g;
        const int Lp = nx - i0 < 4 ? nx - i0 : 4;   // >= 1: g < ge
        const bool need_l = g == 0, need_r = g == ge - 1;

        const T ext = static_cast<T>(ex);
        if (w == 0) {
            // lanes 0..15: the factors of position g = lane (g_t = eps_x / m_{t-1},
            // q_t = 1 / m_t) and the carry multipliers of the two scans
            const T *tab;
            if constexpr (F32)
                tab = a.tab32 + toff;
            else
                tab = a.tab + toff;
            const int gg = lane & 15, ii = 4 * gg;
            const int Lg = nx - ii < 4 ? nx - ii : 4;
            T gv[4], qq[4];
            T pf = 1, pb = 1;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int idx = ii + t < nx ? ii + t : nx - 1;
                gv[t] = tab[idx];
                qq[t] = tab[nx + idx];
                pf = t < Lg ? pf * gv[t] : pf;
                pb = t < Lg ? pb * (ext * qq[t]) : pb;
            }
            // Hillis-Steele partial products: step s combines lane g with g - s
            // (forward) or g + s (backward)
            const T af1 = pf;
            const T l1 = from_left<1>(af1);
            const T af2 = gg >= 1 ? af1 * l1 : af1;
            const T l2 = from_left<2>(af2);
            const T af4 = gg >= 2 ? af2 * l2 : af2;
            const T l4 = from_left<4>(af4);
            const T af8 = gg >= 4 ? af4 * l4 : af4;
            const T ab1 = pb;
            const T r1 = from_right<1>(ab1);
            const T ab2 = gg + 1 < ge ? ab1 * r1 : ab1;
            const T r2 = from_right<2>(ab2);
            const T ab4 = gg + 2 < ge ? ab2 * r2 : ab2;
            const T r4 = from_right<4>(ab4);
            const T ab8 = gg + 4 < ge ? ab4 * r4 : ab4;
            if (lane < 16) {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    xt[t][gg] = gv[t];
                    xt[4 + t][gg] = qq[t];
                }
                xt[8][gg] = gg >= 1 ? af1 : T(0);
                xt[9][gg] = gg >= 2 ? af2 : T(0);
                xt[10][gg] = gg >= 4 ? af4 : T(0);
                xt[11][gg] = gg >= 8 ? af8 : T(0);
                xt[12][gg] = gg + 1 < ge ? ab1 : T(0);
                xt[13][gg] = gg + 2 < ge ? ab2 : T(0);
                xt[14][gg] = gg + 4 < ge ? ab4 : T(0);
                xt[15][gg] = gg + 8 < ge ? ab8 : T(0);
                xt[16][gg] = gg >= 1 ? T(1) : T(0);
                xt[17][gg] = gg + 1 < ge ? T(1) : T(0);
            }
        }

        int nph = 1;
        if (cm == 2) {
            if (w == 0) {
                const int rho = it.tile * 64 + lane;
                const int k = rho / ny, j = rho - k * ny;
                const bool in = k < nz;
                const bool c1 = ((j + k) & 1) != 0;
                const uint64_t m0 = __builtin_amdgcn_ballot_w64(in && !c1);
                const uint64_t m1 = __builtin_amdgcn_ballot_w64(in && c1);
                const int n0 = __popcll(m0);
                const uint64_t below = (1ull << lane) - 1ull;
                if (in) rows[c1 ? n0 + __popcll(m1 & below) : __popcll(m0 & below)] = lane;
                if (lane == 0) {
                    ncnt[0] = n0;
                    ncnt[1] = __popcll(m1);
                }
            }
            nph = 2;
        }
        __syncthreads();   // factor table (and row list) complete

        const char *ub = reinterpret_cast<const char *>(a.src + pd->uoff);
        const char *fb = reinterpret_cast<const char *>(a.f + pd->foff);
        char *db = reinterpret_cast<char *>(a.dst + pd->uoff);
        const double om = a.omega;

        for (int ph = 0; ph < nph; ++ph) {
            const int first = (cm == 2 && ph == 1) ? ncnt[0] : 0;
            const int count = cm == 2 ? ncnt[ph] : 64;
            for (int base = w * lpw; base < count; base += nw * lpw) {
                asm volatile("" ::: "memory");   // table reads stay inside the pass
                const int m = base + slot;
                const bool row_ok = lane_ok && m < count;
                const int rt = row_ok ? (cm == 2 ? rows[first + m] : m) : 0;
                const int rho = it.tile * 64 + rt;
                int j, k;
                if (cm == 1) {
                    const int M = (ny + 1) >> 1;
                    k = rho / M;
                    j = 2 * (rho - k * M) + ((k + it.colour) & 1);
                } else {
                    k = rho / ny;
                    j = rho - k * ny;
                }
                // rows next to an extrapolated y or z face: the boundary-line kernel
                const bool in = row_ok && j < ny && k < nz && !offline_extrap(pd->bc, 1, j, ny, 2, k, nz);
                const int jc = in ? j : 0, kc = in ? k : 0;
                // byte offsets of this lane's first cell in u and f
                const uint32_t cu = 8u * ((uint32_t)(kc + 1) * sy + (uint32_t)(jc + 1) * sx + 1u + (uint32_t)i0);
                const uint32_t cf = 8u * (((uint32_t)kc * ny + (uint32_t)jc) * nx + (uint32_t)i0);
                const uint32_t sx8 = 8u * sx, sy8 = 8u * sy;

                double uc[4], rr[4];
                if (a.rhs_mode) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        uc[t] = ldb(ub, cu + 8u * (uint32_t)(t < Lp ? t : Lp - 1));
                        rr[t] = uc[t];
                    }
                } else {
                    double fv[4], ym[4], yp[4], zm[4], zp[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const uint32_t c = cu + 8u * (uint32_t)(t < Lp ? t : Lp - 1);
                        uc[t] = ldb(ub, c);
                        fv[t] = ldb(fb, cf + 8u * (uint32_t)(t < Lp ? t : Lp - 1));
                        ym[t] = ldb(ub, c - sx8);
                        yp[t] = ldb(ub, c + sx8);
                        zm[t] = ldb(ub, c - sy8);
                        zp[t] = ldb(ub, c + sy8);
                    }
                    // the line's end neighbours are ghosts; a one-lane line needs both
                    const double xa = ldb(ub, need_l ? cu - 8u : cu + 8u * (uint32_t)Lp);
                    const double xb = ge == 1 ? ldb(ub, cu + 8u * (uint32_t)Lp) : 0.0;
                    const double prev_last = from_left<1>(uc[3]);
                    const double next_first = from_right<1>(uc[0]);
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const double left = t == 0 ? (need_l ? xa : prev_last) : uc[t - 1];
                        const double right =
                            t == Lp - 1 ? (need_r ? (need_l ? xb : xa) : next_first) : uc[t < 3 ? t + 1 : 3];
                        const double nb = fma(ex, left + right, fma(ey, ym[t] + yp[t], ez * (zm[t] + zp[t])));
                        rr[t] = fma(-d, uc[t], fma(h2, fv[t], nb));
                    }
                }

                // forward elimination: lane-local from a zero carry, then the carries
                T z[4];
                T b = 0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const T v = fma(xt[t][g], b, static_cast<T>(rr[t]));
                    z[t] = (in && t < Lp) ? v : T(0);
                    b = t < Lp ? z[t] : b;
                }
                b = fma(xt[8][g], from_left<1>(b), b);
                if (ge > 2) b = fma(xt[9][g], from_left<2>(b), b);
                if (ge > 4) b = fma(xt[10][g], from_left<4>(b), b);
                if (ge > 8) b = fma(xt[11][g], from_left<8>(b), b);
                const T zin = xt[16][g] * from_left<1>(b);
                T pr = 1;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    pr *= xt[t][g];
                    z[t] = t < Lp ? fma(pr, zin, z[t]) : T(0);
                }

                // back substitution: lane-local from a zero carry, then the carries
                T x[4];
                T B = 0;
                T qt[4];
#pragma unroll
                for (int t = 3; t >= 0; --t) {
                    qt[t] = xt[4 + t][g];
                    const T v = fma(ext, B, z[t]) * qt[t];
                    x[t] = t < Lp ? v : T(0);
                    B = t < Lp ? v : B;
                }
                B = fma(xt[12][g], from_right<1>(B), B);
                if (ge > 2) B = fma(xt[13][g], from_right<2>(B), B);
                if (ge > 4) B = fma(xt[14][g], from_right<4>(B), B);
                if (ge > 8) B = fma(xt[15][g], from_right<8>(B), B);
                const T xout = xt[17][g] * from_right<1>(B);
                T pq = 1;
#pragma unroll
                for (int t = 3; t >= 0; --t) {
                    const T pn = pq * (ext * qt[t]);
                    pq = t < Lp ? pn : pq;
                    x[t] = fma(pq, xout, x[t]);
                }

                if (in) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        if (t < Lp) {
                            const double du = static_cast<double>(x[t]);
                            *reinterpret_cast<double *>(db + cu + 8u * (uint32_t)t) =
                                a.out_mode ? du : fma(om, du, uc[t]);
                        }
                    }
                }
            }
            if (cm == 2 && ph == 0) __syncthreads();   // colour 0 stored before colour 1 reads
        }
        __syncthreads();   // the next item rewrites the tables
    }
}

int line_xr_occupancy(int nwaves, int f32)
{
    int n = 0;
    const hipError_t e = f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_line_xr<true>, 64 * nwaves, 0)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_line_xr<false>, 64 * nwaves, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return n > 0 ? n : 1;
}

hipError_t launch_line_xr(const LineArgs &a, int grid, int nwaves, hipStream_t s)
{
    if (nwaves < 1 || nwaves > 4) return hipErrorInvalidValue;
    if (a.f32)
        hipLaunchKernelGGL(k_line_xr<true>, dim3(grid), dim3(64 * nwaves), 0, s, a);
    else
        hipLaunchKernelGGL(k_line_xr<false>, dim3(grid), dim3(64 * nwaves), 0, s, a);
    return hipGetLastError();
}

}  // namespace bs
