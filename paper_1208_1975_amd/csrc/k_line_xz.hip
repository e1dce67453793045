// x-line relaxation marching along z (lines of up to 64 cells).
//
// A work item is a block of R consecutive rows j (the x-lines of those rows)
// by a range of planes k, marched in increasing k.  Within a plane the lines
// lie as in the register x-line kernel: a line of nx cells across
// ge = ceil(nx / 4) lanes of a 16-lane DPP row, four cells per lane, so loads
// and stores are x-contiguous, and the exact solve is the Thomas algorithm
// reassociated into lane-local recurrences plus a log-step scan of the
// carries (see k_line_xr.hip).  What marching adds: each lane keeps its line's
// cells of planes k-1, k and k+1 in registers, so the z-neighbours of a line
// are never fetched again and every u value is read from memory about once
// per sweep (the y-neighbour rows are the block's own rows of the same plane,
// which the cache holds, except at the block's two edge rows).
//
// Per line (section 2, Algorithm 2's three steps): block residual from the
// current u, exact solve of tridiag(-eps_x, d, -eps_x), update.
//   Jacobi: every line of the plane from the old iterate into the second
//     vector; the registers keep the old values for the next plane.
//   Chaotic GS: in place; within a plane the lines of colour 0 ((j + k) even)
//     first, then, after a workgroup barrier that makes their stores visible,
//     the lines of colour 1 with their updated y-neighbours; the plane below
//     is already updated (its new values are the ones kept in registers) and
//     the plane above is not: one of the orders an asynchronous sweep may
//     take, with lexicographic order along z.  Rows and planes of other items
//     are read as they are found.
#include <type_traits>

#include "bs_internal.h"

namespace bs {

namespace {

template <int CTRL>
__device__ __forceinline__ double xz_dpp64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ float xz_dpp32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

// Value of lane l - S (left) or l + S (right) of the same 16-lane row; zero
// where that lane is outside the row.
template <int S, typename T>
__device__ __forceinline__ T xz_left(T v)
{
    if constexpr (std::is_same<T, float>::value)
        return xz_dpp32<0x110 + S>(v);   // row_shr:S
    else
        return xz_dpp64<0x110 + S>(v);
}

template <int S, typename T>
__device__ __forceinline__ T xz_right(T v)
{
    if constexpr (std::is_same<T, float>::value)
        return xz_dpp32<0x100 + S>(v);   // row_shl:S
    else
        return xz_dpp64<0x100 + S>(v);
}

__device__ __forceinline__ double xz_ld(const char *base, uint32_t off)
{
    return *reinterpret_cast<const double *>(base + off);
}

}  // namespace

// CM: 0 Jacobi (src -> dst), 2 chaotic GS (in place).  a.tx carries the
// planes per item.
template <int CM, bool F32>
__global__ void __launch_bounds__(256) k_line_xz(LineArgs a)
{
    using T = typename std::conditional<F32, float, double>::type;
    __shared__ T xt[18][16];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int nw = blockDim.x >> 6;
    const int zc = a.tx;

    for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
        const WorkItem it = a.items[item];
        if (it.patch < 0) continue;   // padding of the dispatch order
        const PatchDesc *pd = a.pd + it.patch;
        const int nx = pd->n[0], ny = pd->n[1], nz = pd->n[2];
        const uint32_t sx = nx + 2, sy = sx * (uint32_t)(ny + 2);
        const double ex = pd->eps[0], ey = pd->eps[1], ez = pd->eps[2];
        const double d = 2.0 * (ex + ey + ez);
        const double h2 = pd->h2;
        const int bc = pd->bc;
        const int64_t toff = pd->line[0][0].off;   // one chunk: the line's own LU factors

        const int ge = (nx + 3) >> 2;   // lanes per line
        const int lpr = 16 / ge;        // lines per 16-lane row
        const int R = nw * 4 * lpr;     // rows per item
        const int q16 = lane & 15;
        const int seg = q16 / ge;
        const int g = q16 - seg * ge;
        const bool lane_ok = seg < lpr;
        const int i0 = 4 * g;
        const int Lp = nx - i0 < 4 ? nx - i0 : 4;   // >= 1: g < ge
        const bool need_l = g == 0, need_r = g == ge - 1;
        const int nty = (ny + R - 1) / R;
        const int ty = it.tile % nty, tz = it.tile / nty;
        const int j = ty * R + w * (4 * lpr) + (lane >> 4) * lpr + seg;
        const bool row_ok = lane_ok && j < ny;
        const int jc = row_ok ? j : (j < ny ? j : ny - 1);
        const int z0 = tz * zc, z1 = z0 + zc < nz ? z0 + zc : nz;

        const T ext = static_cast<T>(ex);
        __syncthreads();   // the previous item's table reads are done
        if (w == 0) {
            // lanes 0..15: the factors of position g = lane and the carry
            // multipliers of the two scans (as in the register x-line kernel)
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
            const T af1 = pf;
            const T l1 = xz_left<1>(af1);
            const T af2 = gg >= 1 ? af1 * l1 : af1;
            const T l2 = xz_left<2>(af2);
            const T af4 = gg >= 2 ? af2 * l2 : af2;
            const T l4 = xz_left<4>(af4);
            const T af8 = gg >= 4 ? af4 * l4 : af4;
            const T ab1 = pb;
            const T r1 = xz_right<1>(ab1);
            const T ab2 = gg + 1 < ge ? ab1 * r1 : ab1;
            const T r2 = xz_right<2>(ab2);
            const T ab4 = gg + 2 < ge ? ab2 * r2 : ab2;
            const T r4 = xz_right<4>(ab4);
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
        __syncthreads();   // factor table complete

        const char *ub = reinterpret_cast<const char *>(a.src + pd->uoff);
        const char *fb = reinterpret_cast<const char *>(a.f + pd->foff);
        char *db = reinterpret_cast<char *>(a.dst + pd->uoff);
        const double om = a.omega;
        const uint32_t sx8 = 8u * sx, sy8 = 8u * sy;
        // byte offset of this lane's first cell in row jc of plane -1 (the ghost plane)
        const uint32_t col = 8u * ((uint32_t)(jc + 1) * sx + 1u + (uint32_t)i0);
        auto cell = [&](int t) -> uint32_t { return 8u * (uint32_t)(t < Lp ? t : Lp - 1); };

        double prv[4], cur[4], nxt[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            prv[t] = xz_ld(ub, col + (uint32_t)z0 * sy8 + cell(t));
            cur[t] = xz_ld(ub, col + (uint32_t)(z0 + 1) * sy8 + cell(t));
            nxt[t] = xz_ld(ub, col + (uint32_t)(z0 + 2) * sy8 + cell(t));
        }
        for (int k = z0; k < z1; ++k) {
            const uint32_t pc = col + (uint32_t)(k + 1) * sy8;   // plane k
            const uint32_t fc = 8u * (((uint32_t)k * ny + (uint32_t)jc) * nx + (uint32_t)i0);
            // the next plane's values are fetched a step ahead (the ghost plane
            // at the end, clamped)
            const int kn = k + 3 <= nz + 1 ? k + 3 : nz + 1;
            double nn[4], fv[4], ym[4], yp[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                nn[t] = xz_ld(ub, col + (uint32_t)kn * sy8 + cell(t));
                fv[t] = xz_ld(fb, fc + cell(t));
                ym[t] = xz_ld(ub, pc - sx8 + cell(t));
                yp[t] = xz_ld(ub, pc + sx8 + cell(t));
            }
            const double xa = xz_ld(ub, need_l ? pc - 8u : pc + 8u * (uint32_t)Lp);
            const double xb = ge == 1 ? xz_ld(ub, pc + 8u * (uint32_t)Lp) : 0.0;
            // lines next to an extrapolated y or z face: the boundary-line kernel
            const bool in = row_ok && !offline_extrap(bc, 1, j, ny, 2, k, nz);
            const int nph = CM == 2 ? 2 : 1;
            double upd[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) upd[t] = cur[t];
            for (int ph = 0; ph < nph; ++ph) {
                const bool act = in && (CM != 2 || (((j + k) & 1) == ph));
                if (CM == 2 && ph == 1) {
                    __syncthreads();   // colour-0 stores of this plane are visible
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        ym[t] = xz_ld(ub, pc - sx8 + cell(t));
                        yp[t] = xz_ld(ub, pc + sx8 + cell(t));
                    }
                }
                double rr[4];
                const double prev_last = xz_left<1>(cur[3]);
                const double next_first = xz_right<1>(cur[0]);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const double left = t == 0 ? (need_l ? xa : prev_last) : cur[t - 1];
                    const double right = t == Lp - 1 ? (need_r ? (need_l ? xb : xa) : next_first) : cur[t < 3 ? t + 1 : 3];
                    const double nb = fma(ex, left + right, fma(ey, ym[t] + yp[t], ez * (prv[t] + nxt[t])));
                    rr[t] = fma(-d, cur[t], fma(h2, fv[t], nb));
                }
                // forward elimination: lane-local from a zero carry, then the carries
                T z[4];
                T b = 0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const T v = fma(xt[t][g], b, static_cast<T>(rr[t]));
                    z[t] = (act && t < Lp) ? v : T(0);
                    b = t < Lp ? z[t] : b;
                }
                b = fma(xt[8][g], xz_left<1>(b), b);
                if (ge > 2) b = fma(xt[9][g], xz_left<2>(b), b);
                if (ge > 4) b = fma(xt[10][g], xz_left<4>(b), b);
                if (ge > 8) b = fma(xt[11][g], xz_left<8>(b), b);
                const T zin = xt[16][g] * xz_left<1>(b);
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
                B = fma(xt[12][g], xz_right<1>(B), B);
                if (ge > 2) B = fma(xt[13][g], xz_right<2>(B), B);
                if (ge > 4) B = fma(xt[14][g], xz_right<4>(B), B);
                if (ge > 8) B = fma(xt[15][g], xz_right<8>(B), B);
                const T xout = xt[17][g] * xz_right<1>(B);
                T pq = 1;
#pragma unroll
                for (int t = 3; t >= 0; --t) {
                    const T pn = pq * (ext * qt[t]);
                    pq = t < Lp ? pn : pq;
                    x[t] = fma(pq, xout, x[t]);
                }
                if (act) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const double v = fma(om, static_cast<double>(x[t]), cur[t]);
                        upd[t] = v;
                        if (t < Lp) *reinterpret_cast<double *>(db + pc + 8u * (uint32_t)t) = v;
                    }
                }
            }
            // next plane: Jacobi keeps the old values of this plane for its
            // z-neighbour term, chaotic GS the new ones
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                prv[t] = CM == 2 ? upd[t] : cur[t];
                cur[t] = nxt[t];
                nxt[t] = nn[t];
            }
        }
    }
}

hipError_t launch_line_xz(const LineArgs &a, int grid, int nwaves, hipStream_t s)
{
    if (nwaves < 1 || nwaves > 4) return hipErrorInvalidValue;
    if (a.colour_mode != 0 && a.colour_mode != 2) return hipErrorInvalidValue;
    const dim3 g(grid), b(64 * nwaves);
    if (a.colour_mode == 0) {
        if (a.f32)
            hipLaunchKernelGGL((k_line_xz<0, true>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((k_line_xz<0, false>), g, b, 0, s, a);
    } else {
        if (a.f32)
            hipLaunchKernelGGL((k_line_xz<2, true>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((k_line_xz<2, false>), g, b, 0, s, a);
    }
    return hipGetLastError();
}

int line_xz_occupancy(int nwaves, int cm, int f32)
{
    int n = 0;
    hipError_t e;
    if (cm == 0)
        e = f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_line_xz<0, true>, 64 * nwaves, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_line_xz<0, false>, 64 * nwaves, 0);
    else
        e = f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_line_xz<2, true>, 64 * nwaves, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_line_xz<2, false>, 64 * nwaves, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return n > 0 ? n : 1;
}

}  // namespace bs
