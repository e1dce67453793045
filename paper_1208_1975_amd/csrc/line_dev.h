// Device helpers shared by the line-relaxation kernels: the chunk solve with
// precomputed LU factors, lane shifts, and the interface coupling of the
// partition method (k_line.hip describes the method).
#pragma once

#include "bs_internal.h"

namespace bs {

__device__ __forceinline__ int uniform_wave()
{
    return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
}

// Chunk solve in registers: r (length Lp <= L; entries t >= Lp are ignored)
// -> y = T^{-1} r with the LU factors g (multipliers) and q (reciprocal
// pivots), both Lr long, held in LDS.  Branch-free: entries past Lp are forced
// to zero, which keeps the back substitution exact for t < Lp.
template <int L>
__device__ __forceinline__ void chunk_solve(double (&r)[L], int Lp, int Lr, const double *g, const double *q,
                                            double ea, double &y0, double &yl)
{
    double zprev = 0.0;
#pragma unroll
    for (int t = 0; t < L; ++t) {
        const double z = fma(g[t < Lr ? t : Lr - 1], zprev, r[t]);
        r[t] = (t < Lp) ? z : 0.0;
        zprev = r[t];
    }
    double ynext = 0.0;
    yl = 0.0;
#pragma unroll
    for (int t = L - 1; t >= 0; --t) {
        const double y = fma(ea, ynext, r[t]) * q[t < Lr ? t : Lr - 1];
        r[t] = y;
        ynext = y;
        yl = (t == Lp - 1) ? y : yl;
    }
    y0 = r[0];
}

// The same solve with the factors read at constant indices from a
// wave-uniform table (scalar loads, fetched in bulk).  Entries g[t], q[t] for
// t >= Lr read the following table entries, which are finite; their results
// are discarded exactly as above (the table holds at least 3 Lr > Lr + L - 1
// entries because L < 2 Lr).
template <int L, typename T>
__device__ __forceinline__ void chunk_solve_u(T (&r)[L], int Lp, const T *__restrict__ g, const T *__restrict__ q,
                                              T ea, T &y0, T &yl)
{
    T zprev = 0;
#pragma unroll
    for (int t = 0; t < L; ++t) {
        const T z = fma(g[t], zprev, r[t]);
        r[t] = (t < Lp) ? z : T(0);
        zprev = r[t];
    }
    asm volatile("" ::: "memory");   // q is fetched after g is consumed
    T ynext = 0;
    yl = 0;
#pragma unroll
    for (int t = L - 1; t >= 0; --t) {
        const T y = fma(ea, ynext, r[t]) * q[t];
        r[t] = y;
        ynext = y;
        yl = (t == Lp - 1) ? y : yl;
    }
    y0 = r[0];
}

// Neighbour of a lane's value along the wavefront (DPP wave shift by one lane):
// dir < 0 gives lane l the value of lane l-1, dir > 0 that of lane l+1.
template <int DIR>
__device__ __forceinline__ double lane_shift(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    constexpr int ctrl = DIR < 0 ? 0x138 : 0x130;   // wave_shr:1 / wave_shl:1
    const int lo2 = __builtin_amdgcn_update_dpp(0, lo, ctrl, 0xf, 0xf, false);
    const int hi2 = __builtin_amdgcn_update_dpp(0, hi, ctrl, 0xf, 0xf, false);
    return __hiloint2double(hi2, lo2);
}

// Value of lane `src` (any lane of the wavefront, through the LDS crossbar).
__device__ __forceinline__ double lane_get(double v, int src)
{
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Interface coupling: every chunk's wavefront reads the ends of all chunks of
// its line from LDS and forms the two corrections it needs.
template <typename T>
__device__ __forceinline__ void interface_terms(const T *tab, const double *ends, int Lr, int P, int p, int lane,
                                                T &bprev, T &anext)
{
    const T *Kb = tab + 6 * Lr + p * 2 * P;
    const T *Ka = tab + 6 * Lr + 2 * P * P + p * 2 * P;
    bprev = 0;
    anext = 0;
    for (int jj = 0; jj < 2 * P; ++jj) {
        const T Y = static_cast<T>(ends[((jj >> 1) * 64 + lane) * 2 + (jj & 1)]);
        bprev = fma(Kb[jj], Y, bprev);
        anext = fma(Ka[jj], Y, anext);
    }
}

// The same for a table in memory no kernel writes, read as constant memory:
// the rows are wave-uniform, so they come through the scalar cache.
template <typename T>
__device__ __forceinline__ void interface_terms_k(const __attribute__((address_space(4))) T *tab, const double *ends,
                                                  int Lr, int P, int p, int lane, T &bprev, T &anext)
{
    const __attribute__((address_space(4))) T *Kb = tab + 6 * Lr + p * 2 * P;
    const __attribute__((address_space(4))) T *Ka = tab + 6 * Lr + 2 * P * P + p * 2 * P;
    bprev = 0;
    anext = 0;
    for (int jj = 0; jj < 2 * P; ++jj) {
        const T Y = static_cast<T>(ends[((jj >> 1) * 64 + lane) * 2 + (jj & 1)]);
        bprev = fma(Kb[jj], Y, bprev);
        anext = fma(Ka[jj], Y, anext);
    }
}

template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *as_const(const T *p)
{
    return (const __attribute__((address_space(4))) T *)p;
}

__device__ __forceinline__ double ldb(const char *base, uint32_t off)
{
    return *reinterpret_cast<const double *>(base + off);
}

}  // namespace bs
