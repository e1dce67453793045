// Mixed-precision plane solves, FP32 form, and the FP64 helpers of both mixed
// forms: the four fast-diagonalisation products in FP32 on the matrix cores
// (v_mfma_f32_16x16x4_f32) while the residual, the defect of the refinement
// and the update stay in FP64.  For the plane block M_P and residual R
// (FP64), the correction D solves M_P D = R by
//   D_0 = M~^{-1} R,  D_{j+1} = D_j + M~^{-1}(R - M_P D_j)   (j < refine)
// with M~^{-1} the low-precision transform chain, M_P D_j applied in FP64,
// and finally u += omega D in FP64.  (The BF16 products are in k_plane_bf16.)
#include <cstdint>

#include "bs_internal.h"
#include "plane.h"

namespace bs {

namespace {

typedef float flt4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 32;

}  // namespace

// C_b = A_b B_b with FP32 operands (v_mfma_f32_16x16x4_f32), FP32
// accumulation.  A 64 x 64 block of C per workgroup (four wavefronts, 32 x 32
// each); K advances BK at a time through two LDS buffers, the next tile
// fetched into registers while the current one feeds the matrix cores.
// BT: B given [n][k] (transposed on its way into LDS).  FOLD 1 / 2: the
// contraction runs over A's rows / B's k-rows folded about the middle of a
// length-Kfull axis, x'[k] = x[k] + fsign x[Kfull-1-k] (x[k] alone where
// k = Kfull-1-k): with the other operand the even or odd half of a DST-I
// basis (S[n-1-i][j] = (-1)^j S[i][j]), one half of the product at half the
// flops; its rows or columns are the logical rows / columns m row_s + row_o /
// n col_s + col_o of C.
// The fetch is branch-free (clamped in-range addresses, zeroing deferred to
// the LDS store), so those loads stay in flight during the products; VEC:
// aligned rows whose lengths are multiples of 4, one 16-byte load per quad.
template <int EPI, bool VEC, int BT, int FOLD>
__global__ void __launch_bounds__(256) k_gemm_mixed(GemmMixedArgs g)
{
    __shared__ __attribute__((aligned(16))) float As[2][BK][BM + 4];
    __shared__ __attribute__((aligned(16))) float Bs[2][BK][BN + 4];
    // tiles numbered n fastest, then m, then the batch, each XCD taking a
    // contiguous range: the column tiles that read the same rows of A share
    // one XCD's L2
    const int nt = (g.N + BN - 1) / BN, mt = (g.M + BM - 1) / BM;
    const int t = xcd_block(blockIdx.x, gridDim.x);
    const int tn = t % nt, tr = t / nt;
    const int b = tr / mt;
    const int m0 = (tr - b * mt) * BM, n0 = tn * BN;
    const float *A = g.A + (int64_t)b * g.sA;
    const float *B = g.B + (int64_t)b * g.sB;
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int l16 = lane & 15, lk = lane >> 4;
    auto ld4 = [](const float *row, int c0, int lim) -> float4 {   // c0 a multiple of 4
        if constexpr (VEC) {
            return *reinterpret_cast<const float4 *>(row + (c0 < lim ? c0 : lim - 4));
        } else {
            float4 v;
            v.x = row[c0 < lim ? c0 : lim - 1];
            v.y = row[c0 + 1 < lim ? c0 + 1 : lim - 1];
            v.z = row[c0 + 2 < lim ? c0 + 2 : lim - 1];
            v.w = row[c0 + 3 < lim ? c0 + 3 : lim - 1];
            return v;
        }
    };
    auto keep4 = [](float4 v, int c0, int lim, bool row_ok) -> float4 {
        v.x = row_ok && c0 < lim ? v.x : 0.f;
        v.y = row_ok && c0 + 1 < lim ? v.y : 0.f;
        v.z = row_ok && c0 + 2 < lim ? v.z : 0.f;
        v.w = row_ok && c0 + 3 < lim ? v.w : 0.f;
        return v;
    };

    flt4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};

    const int Kf = g.Kfull;
    const float fs = (float)g.fsign;
    // the mirrored entries Kf-1-k of k = c0 .. c0+3 (in that order) of a row
    // (FOLD 1) -- one 16-byte load of the quad Kf-4-c0 .. Kf-1-c0, reversed,
    // when aligned -- and the folding of a loaded quad
    auto ldm4 = [&](const float *row, int c0) -> float4 {
        if constexpr (VEC) {
            const int b = Kf - 4 - c0;
            const float4 v = *reinterpret_cast<const float4 *>(row + (b >= 0 ? b : 0));
            return float4{v.w, v.z, v.y, v.x};
        } else {
            float4 v;
            v.x = row[Kf - 1 - c0 >= 0 ? Kf - 1 - c0 : 0];
            v.y = row[Kf - 2 - c0 >= 0 ? Kf - 2 - c0 : 0];
            v.z = row[Kf - 3 - c0 >= 0 ? Kf - 3 - c0 : 0];
            v.w = row[Kf - 4 - c0 >= 0 ? Kf - 4 - c0 : 0];
            return v;
        }
    };
    auto fold4 = [&](float4 v, float4 m, int c0) -> float4 {   // entries k = c0 .. c0+3
        v.x = (c0 < g.K && Kf - 1 - c0 != c0) ? fmaf(fs, m.x, v.x) : v.x;
        v.y = (c0 + 1 < g.K && Kf - 2 - c0 != c0 + 1) ? fmaf(fs, m.y, v.y) : v.y;
        v.z = (c0 + 2 < g.K && Kf - 3 - c0 != c0 + 2) ? fmaf(fs, m.z, v.z) : v.z;
        v.w = (c0 + 3 < g.K && Kf - 4 - c0 != c0 + 3) ? fmaf(fs, m.w, v.w) : v.w;
        return v;
    };

    // A tile BM x BK: quad c -> row c / 8, k offset (c % 8) * 4; B tile BK x BN:
    // quad c -> k row c / 16, n offset (c % 16) * 4, or (BT) n row c / 8, k
    // offset (c % 8) * 4 (two quads a thread)
    float4 ra[2], rb[2], rm[2];   // rm: the mirrored quad (A for FOLD 1, B for FOLD 2)
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int c = tid + 256 * q;
            const int r = c >> 3, kc = (c & 7) * 4;
            const int gr = m0 + r;
            const float *arow = A + (int64_t)(gr < g.M ? gr : g.M - 1) * g.lda;
            ra[q] = ld4(arow, k0 + kc, g.K);
            if constexpr (FOLD == 1) rm[q] = ldm4(arow, k0 + kc);
            if constexpr (BT) {
                const int gn = n0 + r;
                rb[q] = ld4(B + (int64_t)(gn < g.N ? gn : g.N - 1) * g.ldb, k0 + kc, g.K);
            } else {
                const int kr = c >> 4, nc = (c & 15) * 4;
                const int gk = k0 + kr, gkc = gk < g.K ? gk : g.K - 1;
                rb[q] = ld4(B + (int64_t)gkc * g.ldb, n0 + nc, g.N);
                if constexpr (FOLD == 2) rm[q] = ld4(B + (int64_t)(Kf - 1 - gkc) * g.ldb, n0 + nc, g.N);
            }
        }
    };
    auto stash = [&](int buf, int k0) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int c = tid + 256 * q;
            const int r = c >> 3, kc = (c & 7) * 4;
            float4 a4 = ra[q];
            if constexpr (FOLD == 1) a4 = fold4(a4, rm[q], k0 + kc);
            a4 = keep4(a4, k0 + kc, g.K, m0 + r < g.M);
            As[buf][kc][r] = a4.x;
            As[buf][kc + 1][r] = a4.y;
            As[buf][kc + 2][r] = a4.z;
            As[buf][kc + 3][r] = a4.w;
            if constexpr (BT) {
                const float4 b4 = keep4(rb[q], k0 + kc, g.K, n0 + r < g.N);
                Bs[buf][kc][r] = b4.x;
                Bs[buf][kc + 1][r] = b4.y;
                Bs[buf][kc + 2][r] = b4.z;
                Bs[buf][kc + 3][r] = b4.w;
            } else {
                const int kr = c >> 4, nc = (c & 15) * 4;
                const int gk = k0 + kr;
                float4 b4 = rb[q];
                if constexpr (FOLD == 2) {
                    const bool use = gk < g.K && Kf - 1 - gk != gk;
                    b4.x = use ? fmaf(fs, rm[q].x, b4.x) : b4.x;
                    b4.y = use ? fmaf(fs, rm[q].y, b4.y) : b4.y;
                    b4.z = use ? fmaf(fs, rm[q].z, b4.z) : b4.z;
                    b4.w = use ? fmaf(fs, rm[q].w, b4.w) : b4.w;
                }
                *reinterpret_cast<float4 *>(&Bs[buf][kr][nc]) = keep4(b4, n0 + nc, g.N, gk < g.K);
            }
        }
    };

    const int nk = (g.K + BK - 1) / BK;
    fetch(0);
    stash(0, 0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) fetch((kt + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            float af[2], bfr[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) af[i] = As[cur][kk + lk][wm * 32 + i * 16 + l16];
#pragma unroll
            for (int j = 0; j < 2; ++j) bfr[j] = Bs[cur][kk + lk][wn * 32 + j * 16 + l16];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
        if (kt + 1 < nk) stash(cur ^ 1, (kt + 1) * BK);
        __syncthreads();
    }

    // D layout of the FP32 16x16 block: register r of a lane holds row
    // 4*(lane/16) + r, column lane%16 (checked by the layout test).  Per block,
    // the values the four outputs of a lane read (scale, D, u) are loaded
    // before any of their stores, so they are in flight together.
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            double in1[4], in2[4];
            bool ok[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int pm = m0 + wm * 32 + i * 16 + (g.dlayout ? r * 4 + lk : lk * 4 + r);
                const int pn = n0 + wn * 32 + j * 16 + l16;
                const int row = pm * g.row_s + g.row_o, col = pn * g.col_s + g.col_o;   // logical
                bool o = pm < g.M && pn < g.N;
                if (EPI == kEpiUpdate || EPI == kEpiUpdateAcc)
                    o = o && !(g.ncolour >= 0 && ((col + g.colour_shift) & 1) != g.ncolour);
                ok[r] = o;
                const int rr = o ? row : 0, cc = o ? col : 0;   // in-range addresses for every lane
                const int64_t ci = (int64_t)b * g.sC + (int64_t)rr * g.ldc + cc;
                in1[r] = 0.0;
                in2[r] = 0.0;
                if (EPI == kEpiScale) in1[r] = g.scale[(int64_t)b * g.sc_b + (int64_t)rr * g.sc_m + (int64_t)cc * g.sc_n];
                if (EPI == kEpiUpdateAcc || (EPI == kEpiD64 && g.accumulate)) in1[r] = g.D[ci];
                if (EPI == kEpiUpdate || EPI == kEpiUpdateAcc)
                    in2[r] = g.usrc[g.u0 + (int64_t)b * g.u_b + (int64_t)rr * g.u_m + (int64_t)cc * g.u_n];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (!ok[r]) continue;
                const int row = (m0 + wm * 32 + i * 16 + (g.dlayout ? r * 4 + lk : lk * 4 + r)) * g.row_s + g.row_o;
                const int col = (n0 + wn * 32 + j * 16 + l16) * g.col_s + g.col_o;
                const float v = acc[i][j][r];
                const int64_t ci = (int64_t)b * g.sC + (int64_t)row * g.ldc + col;
                if (EPI == kEpiStore) {
                    g.C[ci] = v;
                } else if (EPI == kEpiScale) {
                    g.C[ci] = v * static_cast<float>(in1[r]);
                } else if (EPI == kEpiD64) {
                    g.D[ci] = g.accumulate ? in1[r] + (double)v : (double)v;
                } else {
                    const int64_t u = g.u0 + (int64_t)b * g.u_b + (int64_t)row * g.u_m + (int64_t)col * g.u_n;
                    const double du = EPI == kEpiUpdateAcc ? in1[r] + (double)v : (double)v;
                    g.udst[u] = fma(g.omega, du, in2[r]);
                }
            }
        }
}

__device__ __forceinline__ void put_lowp(float *E, int64_t c, double v) { E[c] = (float)v; }
__device__ __forceinline__ void put_lowp(unsigned short *E, int64_t c, double v)
{
    E[c] = __builtin_bit_cast(unsigned short, static_cast<__bf16>(v));
}

// V consecutive values of a row from p (V = 1, or 4 from a 4-element-aligned
// p: one 16-byte load of floats, two of doubles).
template <int V, typename S>
__device__ __forceinline__ void ld_row(const S *p, double (&o)[V])
{
    if constexpr (V == 1) {
        o[0] = (double)p[0];
    } else if constexpr (sizeof(S) == 4) {
        const float4 q = *reinterpret_cast<const float4 *>(p);
        o[0] = q.x; o[1] = q.y; o[2] = q.z; o[3] = q.w;
    } else {
        const double2 q0 = *reinterpret_cast<const double2 *>(p), q1 = *reinterpret_cast<const double2 *>(p + 2);
        o[0] = q0.x; o[1] = q0.y; o[2] = q1.x; o[3] = q1.y;
    }
}

// E = low-precision (R - M_P D) on every cell of one patch (D may be null:
// E = R), M_P the plane block with normal NORMAL: d D - eps_a (in-plane
// neighbours along a) - eps_b (along b), zero beyond the plane's edges,
// formed in FP64 from R and D stored as S (double, or float for the BF16
// chain).  T: float, or unsigned short holding BF16 (rounded from FP64
// directly).  A thread takes V consecutive cells of one x-row (V = 4 when
// the rows are multiples of four cells and the fields 16-byte aligned, so
// every load is one vector load); the neighbour loads are unconditional
// (clamped addresses, zero weights beyond the plane's edges), so they are all
// in flight together.
template <typename S, typename T, int NORMAL, int V>
__global__ void __launch_bounds__(256) k_plane_defect(const S *R, const S *D, T *E, int nx, int ny, int nz,
                                                      double ex, double ey, double ez, double rnx, double rny)
{
    const int n = nx * ny * nz;   // < 2^31: patches are below 4 GiB
    const int c = (blockIdx.x * 256 + threadIdx.x) * V;
    if (c >= n) return;
    double v[V];
    ld_row<V>(R + c, v);
    if (D) {
        const int jk = div_rd(c, nx, rnx);
        const int i = c - jk * nx;
        const int k = div_rd(jk, ny, rny);
        const int j = jk - k * ny;
        const int64_t pl = (int64_t)nx * ny;
        double dc[V], md[V];
        ld_row<V>(D + c, dc);
        const double d = 2.0 * (ex + ey + ez);
#pragma unroll
        for (int e = 0; e < V; ++e) md[e] = d * dc[e];
        if (NORMAL != 0) {
            const double l = (double)D[i > 0 ? c - 1 : c], r = (double)D[i + V < nx ? c + V : c];
            const double wl = i > 0 ? ex : 0.0, wr = i + V < nx ? ex : 0.0;
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const double xl = e == 0 ? wl * l : ex * dc[e > 0 ? e - 1 : 0];
                const double xr = e == V - 1 ? wr * r : ex * dc[e < V - 1 ? e + 1 : 0];
                md[e] -= xl + xr;
            }
        }
        if (NORMAL != 1) {
            double a[V], b[V];
            ld_row<V>(D + (j > 0 ? c - nx : c), a);
            ld_row<V>(D + (j < ny - 1 ? c + nx : c), b);
            const double wa = j > 0 ? ey : 0.0, wb = j < ny - 1 ? ey : 0.0;
#pragma unroll
            for (int e = 0; e < V; ++e) md[e] -= wa * a[e] + wb * b[e];
        }
        if (NORMAL != 2) {
            double a[V], b[V];
            ld_row<V>(D + (k > 0 ? c - pl : c), a);
            ld_row<V>(D + (k < nz - 1 ? c + pl : c), b);
            const double wa = k > 0 ? ez : 0.0, wb = k < nz - 1 ? ez : 0.0;
#pragma unroll
            for (int e = 0; e < V; ++e) md[e] -= wa * a[e] + wb * b[e];
        }
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] -= md[e];
    }
    if constexpr (V == 4 && sizeof(T) == 2) {   // four BF16 values: one 8-byte store
        uint2 w;
        w.x = __builtin_bit_cast(unsigned short, static_cast<__bf16>(v[0])) |
              ((uint32_t)__builtin_bit_cast(unsigned short, static_cast<__bf16>(v[1])) << 16);
        w.y = __builtin_bit_cast(unsigned short, static_cast<__bf16>(v[2])) |
              ((uint32_t)__builtin_bit_cast(unsigned short, static_cast<__bf16>(v[3])) << 16);
        *reinterpret_cast<uint2 *>(E + c) = w;
    } else if constexpr (V == 4) {             // four floats: one 16-byte store
        *reinterpret_cast<float4 *>(E + c) = float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
    } else {
        put_lowp(E, c, v[0]);
    }
}

template <typename S, typename T, int V>
static void launch_defect_v(const S *R, const S *D, T *E, int nx, int ny, int nz, int normal, const double eps[3],
                            hipStream_t s)
{
    const int64_t n = (int64_t)nx * ny * nz;
    const dim3 grid((unsigned)((n / V + 255) / 256));
    const double rnx = 1.0 / nx, rny = 1.0 / ny;
    switch (normal) {
    case 0:
        hipLaunchKernelGGL((k_plane_defect<S, T, 0, V>), grid, dim3(256), 0, s, R, D, E, nx, ny, nz, eps[0],
                           eps[1], eps[2], rnx, rny);
        break;
    case 1:
        hipLaunchKernelGGL((k_plane_defect<S, T, 1, V>), grid, dim3(256), 0, s, R, D, E, nx, ny, nz, eps[0],
                           eps[1], eps[2], rnx, rny);
        break;
    default:
        hipLaunchKernelGGL((k_plane_defect<S, T, 2, V>), grid, dim3(256), 0, s, R, D, E, nx, ny, nz, eps[0],
                           eps[1], eps[2], rnx, rny);
        break;
    }
}

template <typename S, typename T>
static hipError_t launch_defect(const S *R, const S *D, T *E, int nx, int ny, int nz, int normal, const double eps[3],
                                hipStream_t s)
{
    const int64_t n = (int64_t)nx * ny * nz;
    if (n <= 0) return hipSuccess;
    const bool vec = nx % 4 == 0 && reinterpret_cast<uintptr_t>(R) % (4 * sizeof(S)) == 0 &&
                     reinterpret_cast<uintptr_t>(D) % (4 * sizeof(S)) == 0 &&
                     reinterpret_cast<uintptr_t>(E) % (4 * sizeof(T)) == 0;
    if (vec)
        launch_defect_v<S, T, 4>(R, D, E, nx, ny, nz, normal, eps, s);
    else
        launch_defect_v<S, T, 1>(R, D, E, nx, ny, nz, normal, eps, s);
    return hipGetLastError();
}

template <bool VEC, int BT, int FOLD>
static hipError_t launch_mixed_f(const GemmMixedArgs &g, int epi, dim3 grid, hipStream_t s)
{
    switch (epi) {
    case kEpiStore: hipLaunchKernelGGL((k_gemm_mixed<kEpiStore, VEC, BT, FOLD>), grid, dim3(256), 0, s, g); break;
    case kEpiScale: hipLaunchKernelGGL((k_gemm_mixed<kEpiScale, VEC, BT, FOLD>), grid, dim3(256), 0, s, g); break;
    case kEpiUpdate: hipLaunchKernelGGL((k_gemm_mixed<kEpiUpdate, VEC, BT, FOLD>), grid, dim3(256), 0, s, g); break;
    case kEpiD64: hipLaunchKernelGGL((k_gemm_mixed<kEpiD64, VEC, BT, FOLD>), grid, dim3(256), 0, s, g); break;
    case kEpiUpdateAcc:
        hipLaunchKernelGGL((k_gemm_mixed<kEpiUpdateAcc, VEC, BT, FOLD>), grid, dim3(256), 0, s, g);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool VEC>
static hipError_t launch_mixed_v(const GemmMixedArgs &g, int epi, dim3 grid, hipStream_t s)
{
    if (g.b_trans && g.fold == 1) return launch_mixed_f<VEC, 1, 1>(g, epi, grid, s);
    if (!g.b_trans && g.fold == 2) return launch_mixed_f<VEC, 0, 2>(g, epi, grid, s);
    if (!g.b_trans && g.fold == 0) return launch_mixed_f<VEC, 0, 0>(g, epi, grid, s);
    return hipErrorInvalidValue;
}

hipError_t launch_gemm_mixed(const GemmMixedArgs &g0, int prec, int epi, hipStream_t s)
{
    if (prec != 1) return hipErrorInvalidValue;
    if (g0.M <= 0 || g0.N <= 0 || g0.K <= 0 || g0.batch <= 0) return hipSuccess;
    GemmMixedArgs g = g0;
    if (g.row_s == 0) { g.row_s = 1; g.row_o = 0; }
    if (g.col_s == 0) { g.col_s = 1; g.col_o = 0; }
    if (g.fold == 0) { g.Kfull = g.K; g.fsign = 1; }
    const dim3 grid((unsigned)(((g.N + BN - 1) / BN) * ((g.M + BM - 1) / BM) * g.batch));
    // 16-byte quads: aligned bases and strides, row lengths (K for A and for B
    // given [n][k], N for B given [k][n]) multiples of 4, and for A's mirrored
    // quads an axis length Kfull that is one too
    const bool vec = (reinterpret_cast<uintptr_t>(g.A) % 16 == 0) && (reinterpret_cast<uintptr_t>(g.B) % 16 == 0) &&
                     g.lda % 4 == 0 && g.ldb % 4 == 0 && g.sA % 4 == 0 && g.sB % 4 == 0 && g.K % 4 == 0 &&
                     (g.b_trans || g.N % 4 == 0) && (g.fold != 1 || g.Kfull % 4 == 0);
    return vec ? launch_mixed_v<true>(g, epi, grid, s) : launch_mixed_v<false>(g, epi, grid, s);
}

hipError_t launch_plane_defect(const double *R, const double *D, float *E, int nx, int ny, int nz, int normal,
                               const double eps[3], hipStream_t s)
{
    return launch_defect(R, D, E, nx, ny, nz, normal, eps, s);
}

hipError_t launch_plane_defect_bf16(const float *R, const float *D, unsigned short *E, int nx, int ny, int nz,
                                    int normal, const double eps[3], hipStream_t s)
{
    return launch_defect(R, D, E, nx, ny, nz, normal, eps, s);
}

}  // namespace bs
