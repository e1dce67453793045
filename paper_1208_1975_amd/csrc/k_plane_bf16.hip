// BF16 fast-diagonalisation products for the mixed-precision plane solve.
//
// The four products of M_P^{-1} E = S_b [(S_b E S_a) ./ Lambda] S_a run on
// v_mfma_f32_16x16x32_bf16 (BF16 operands, FP32 accumulation).  Operands and
// intermediate fields are stored in BF16: every product rounds its inputs to
// BF16 anyway, so storing them rounded changes no result and halves the bytes.
//
// Tiling: a workgroup of four wavefronts computes a 128 x 128 block of C, each
// wavefront a 64 x 64 quadrant as 4 x 4 blocks of 16 x 16; K advances 32 at a
// time through two LDS buffers (the next tile is fetched into registers while
// the current one feeds the matrix cores; one barrier per step).  In LDS both
// operands are k-contiguous rows (A as [m][k], B as [n][k]), so each MFMA
// operand of a lane -- eight consecutive k of one row or column -- is one
// 128-bit LDS read.  B arrives either already k-contiguous (the sine bases
// are symmetric, S = S^T, and fields that the previous product stored
// transposed) or as [k][n] (a field), which is transposed on its way into
// LDS.  The store epilogues can write C^T, so that the next product finds its
// field operand k-contiguous.
#include <cstdint>

#include "bs_internal.h"
#include "plane.h"

namespace bs {

namespace {

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16;

constexpr int TM = 128, TN = 128, TK = 32;
constexpr int PK = TK + 8;   // LDS row pitch in BF16 elements (80 bytes)

__device__ __forceinline__ u16 to_bf16(float v)
{
    const __bf16 h = static_cast<__bf16>(v);
    return __builtin_bit_cast(u16, h);
}

// Eight consecutive BF16 of a row starting at column c0 (zero beyond `lim`);
// `vec` allows one 16-byte load when the whole group is inside.
__device__ __forceinline__ uint4 load8(const u16 *row, int c0, int lim, bool vec)
{
    if (vec && c0 + 8 <= lim) return *reinterpret_cast<const uint4 *>(row + c0);
    u16 v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (c0 + e < lim) ? row[c0 + e] : (u16)0;
    uint4 r;
    r.x = v[0] | ((uint32_t)v[1] << 16);
    r.y = v[2] | ((uint32_t)v[3] << 16);
    r.z = v[4] | ((uint32_t)v[5] << 16);
    r.w = v[6] | ((uint32_t)v[7] << 16);
    return r;
}

}  // namespace

template <int EPI, int BT>
__global__ void __launch_bounds__(256) k_gemm_bf16(GemmBf16Args g)
{
    __shared__ __attribute__((aligned(16))) u16 As[2][TM * PK];
    __shared__ __attribute__((aligned(16))) u16 Bs[2][TN * PK];
    const int b = blockIdx.z;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const u16 *A = g.A + (int64_t)b * g.sA;
    const u16 *B = g.B + (int64_t)b * g.sB;
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int l16 = lane & 15, lk = lane >> 4;
    const bool avec = ((g.lda & 7) == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
    const bool bvec = ((g.ldb & 7) == 0) && ((reinterpret_cast<uintptr_t>(B) & 15) == 0);

    flt4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};

    uint4 ra[2], rb[2];
    // chunk c of the A tile: row c / 4, k offset (c % 4) * 8; of the B tile:
    // BT: row (n) c / 4, k offset (c % 4) * 8; otherwise k row c / 16, n offset (c % 16) * 8
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int c = tid + 256 * q;
            const int r = c >> 2, kc = (c & 3) * 8;
            const int gr = m0 + r;
            ra[q] = gr < g.M ? load8(A + (int64_t)gr * g.lda, k0 + kc, g.K, avec) : uint4{0, 0, 0, 0};
            if (BT) {
                const int gn = n0 + r;
                rb[q] = gn < g.N ? load8(B + (int64_t)gn * g.ldb, k0 + kc, g.K, bvec) : uint4{0, 0, 0, 0};
            } else {
                const int kr = c >> 4, nc = (c & 15) * 8;
                const int gk = k0 + kr;
                rb[q] = gk < g.K ? load8(B + (int64_t)gk * g.ldb, n0 + nc, g.N, bvec) : uint4{0, 0, 0, 0};
            }
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int c = tid + 256 * q;
            const int r = c >> 2, kc = (c & 3) * 8;
            *reinterpret_cast<uint4 *>(&As[buf][r * PK + kc]) = ra[q];
            if (BT) {
                *reinterpret_cast<uint4 *>(&Bs[buf][r * PK + kc]) = rb[q];
            } else {
                const int kr = c >> 4, nc = (c & 15) * 8;
                const uint32_t wv[4] = {rb[q].x, rb[q].y, rb[q].z, rb[q].w};
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    Bs[buf][(nc + e) * PK + kr] = (u16)((wv[e >> 1] >> (16 * (e & 1))) & 0xffff);
            }
        }
    };

    const int nk = (g.K + TK - 1) / TK;
    fetch(0);
    stash(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) fetch((kt + 1) * TK);
        bf16x8 af[4], bfr[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            af[i] = *reinterpret_cast<const bf16x8 *>(&As[cur][(wm * 64 + i * 16 + l16) * PK + 8 * lk]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            bfr[j] = *reinterpret_cast<const bf16x8 *>(&Bs[cur][(wn * 64 + j * 16 + l16) * PK + 8 * lk]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        if (kt + 1 < nk) stash(cur ^ 1);
        __syncthreads();
    }

    // register r of a lane holds row 4*(lane/16) + r, column lane%16 of its
    // 16 x 16 block (checked by the layout test)
    if ((EPI == kEpiStore || EPI == kEpiScale) && g.c_trans) {
        // C^T: a lane's four rows are consecutive in memory (one 8-byte store
        // when aligned and inside)
        const bool cvec = ((g.ldc & 3) == 0) && ((g.sC & 3) == 0) && ((reinterpret_cast<uintptr_t>(g.C) & 7) == 0);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row0 = m0 + wm * 64 + i * 16 + 4 * lk;
                const int col = n0 + wn * 64 + j * 16 + l16;
                if (col >= g.N) continue;
                u16 h[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float v = acc[i][j][r];
                    if (EPI == kEpiScale)
                        v *= g.scale[(int64_t)b * g.sc_b + (int64_t)(row0 + r < g.M ? row0 + r : 0) * g.sc_m +
                                     (int64_t)col * g.sc_n];
                    h[r] = to_bf16(v);
                }
                u16 *dst = g.C + (int64_t)b * g.sC + (int64_t)col * g.ldc + row0;
                if (cvec && row0 + 4 <= g.M) {
                    uint2 w2;
                    w2.x = h[0] | ((uint32_t)h[1] << 16);
                    w2.y = h[2] | ((uint32_t)h[3] << 16);
                    *reinterpret_cast<uint2 *>(dst) = w2;
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (row0 + r < g.M) dst[r] = h[r];
                }
            }
        return;
    }
    // The four outputs of a lane in one 16 x 16 block at a time: every value
    // they read (scale, D, u) is loaded before any of their stores, so those
    // loads are in flight together instead of one round trip per element.
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jh = 0; jh < 4; ++jh) {
            double in1[1][4], in2[1][4];
            bool ok[1][4];
#pragma unroll
            for (int jj = 0; jj < 1; ++jj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = m0 + wm * 64 + i * 16 + 4 * lk + r;
                    const int col = n0 + wn * 64 + (jh + jj) * 16 + l16;
                    bool o = row < g.M && col < g.N;
                    if (EPI == kEpiUpdate || EPI == kEpiUpdateAcc)
                        o = o && !(g.ncolour >= 0 && ((col + g.colour_shift) & 1) != g.ncolour);
                    ok[jj][r] = o;
                    const int rr = o ? row : 0, cc = o ? col : 0;   // in-range addresses for every lane
                    const int64_t ci = (int64_t)b * g.sC + (int64_t)rr * g.ldc + cc;
                    in1[jj][r] = 0.0;
                    in2[jj][r] = 0.0;
                    if (EPI == kEpiScale)
                        in1[jj][r] = g.scale[(int64_t)b * g.sc_b + (int64_t)rr * g.sc_m + (int64_t)cc * g.sc_n];
                    if (EPI == kEpiUpdateAcc || (EPI == kEpiD64 && g.accumulate)) in1[jj][r] = g.D[ci];
                    if (EPI == kEpiUpdate || EPI == kEpiUpdateAcc)
                        in2[jj][r] = g.usrc[g.u0 + (int64_t)b * g.u_b + (int64_t)rr * g.u_m + (int64_t)cc * g.u_n];
                }
#pragma unroll
            for (int jj = 0; jj < 1; ++jj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (!ok[jj][r]) continue;
                    const int row = m0 + wm * 64 + i * 16 + 4 * lk + r;
                    const int col = n0 + wn * 64 + (jh + jj) * 16 + l16;
                    const float v = acc[i][jh + jj][r];
                    const int64_t ci = (int64_t)b * g.sC + (int64_t)row * g.ldc + col;
                    if (EPI == kEpiStore) {
                        g.C[ci] = to_bf16(v);
                    } else if (EPI == kEpiScale) {
                        g.C[ci] = to_bf16(v * static_cast<float>(in1[jj][r]));
                    } else if (EPI == kEpiD64) {
                        g.D[ci] = g.accumulate ? in1[jj][r] + (double)v : (double)v;
                    } else {
                        const int64_t u = g.u0 + (int64_t)b * g.u_b + (int64_t)row * g.u_m + (int64_t)col * g.u_n;
                        const double du = EPI == kEpiUpdateAcc ? in1[jj][r] + (double)v : (double)v;
                        g.udst[u] = fma(g.omega, du, in2[jj][r]);
                    }
                }
        }
}

template <int BT>
static hipError_t launch_bf16_t(const GemmBf16Args &g, int epi, hipStream_t s)
{
    const dim3 grid((g.N + TN - 1) / TN, (g.M + TM - 1) / TM, g.batch);
    switch (epi) {
    case kEpiStore: hipLaunchKernelGGL((k_gemm_bf16<kEpiStore, BT>), grid, dim3(256), 0, s, g); break;
    case kEpiScale: hipLaunchKernelGGL((k_gemm_bf16<kEpiScale, BT>), grid, dim3(256), 0, s, g); break;
    case kEpiUpdate: hipLaunchKernelGGL((k_gemm_bf16<kEpiUpdate, BT>), grid, dim3(256), 0, s, g); break;
    case kEpiD64: hipLaunchKernelGGL((k_gemm_bf16<kEpiD64, BT>), grid, dim3(256), 0, s, g); break;
    case kEpiUpdateAcc: hipLaunchKernelGGL((k_gemm_bf16<kEpiUpdateAcc, BT>), grid, dim3(256), 0, s, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gemm_bf16(const GemmBf16Args &g, int b_trans, int epi, hipStream_t s)
{
    if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.batch <= 0) return hipSuccess;
    return b_trans ? launch_bf16_t<1>(g, epi, s) : launch_bf16_t<0>(g, epi, s);
}

}  // namespace bs
