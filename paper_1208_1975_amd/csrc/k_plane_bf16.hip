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
//
// The tiles of a launch are numbered n fastest, then m, then the batch, and
// each XCD takes a contiguous range of that numbering (xcd_block), so the
// column tiles that share one A row block run together on one XCD and read it
// once into that XCD's L2 (in the hardware's own order each of them sat on a
// different XCD and fetched the block again from memory).
#include <cstdint>
#include <type_traits>

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

}  // namespace

// Two ways to feed the matrix cores.
//
// Register staging (any shapes): operand chunks are loaded branch-free into
// registers (clamped, in-range addresses) and completed in stash (zeroed
// outside the operands), so the next step's loads stay in flight while the
// matrix cores work on the current one.  VEC: every row 16-byte aligned and
// every row length a multiple of 8, so a chunk is one 16-byte load.
//
// Direct staging (ASYNC; B given [n][k], 16-byte aligned rows, K a multiple
// of TK): global_load_lds writes each lane's 16 bytes straight into LDS, so
// the operand tiles of the next NS - 1 steps are in flight at once without
// holding registers.  A wave's load fills 1 KiB of LDS, lane l at byte 16 l:
// 16 rows of TK = 32 BF16 (64 bytes) with no padding; lane l takes row l / 4
// and slot l % 4, which holds the row's k-chunk (l % 4) ^ ((row / 2) % 4).
// That swizzle puts the 16-byte slots that one 8-lane phase of the MFMA
// operand reads (rows r..r+7, one chunk) and of the writes (two rows, four
// chunks each) in different bank groups.  Each step waits for its own tile
// (s_waitcnt vmcnt) and a workgroup barrier, then issues the tile NS - 1
// steps ahead into the buffer that every wave finished reading in the
// previous step.
constexpr int NS = 3;   // LDS stages of direct staging

template <int EPI, int BT, bool VEC, bool ASYNC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_gemm_bf16(GemmBf16Args g)
{
    // register staging's double buffer (a single row when direct staging
    // uses its own stage arrays)
    constexpr int NBUF = ASYNC ? 1 : 2;
    __shared__ __attribute__((aligned(16))) u16 As[NBUF][ASYNC ? 8 : TM * PK];
    __shared__ __attribute__((aligned(16))) u16 Bs[NBUF][ASYNC ? 8 : TN * PK];
    const int nt = (g.N + TN - 1) / TN, mt = (g.M + TM - 1) / TM;
    const int t = xcd_block(blockIdx.x, gridDim.x);
    const int tn = t % nt, tr = t / nt;
    const int b = tr / mt;
    const int m0 = (tr - b * mt) * TM, n0 = tn * TN;
    const u16 *A = g.A + (int64_t)b * g.sA;
    const u16 *B = g.B + (int64_t)b * g.sB;
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int l16 = lane & 15, lk = lane >> 4;
    // eight consecutive entries c0.. c0 + 7 (c0 a multiple of 8) of a row of
    // length lim, loaded from in-range addresses; keep8 zeroes those at or
    // beyond lim
    auto ld8 = [](const u16 *row, int c0, int lim) -> uint4 {
        if constexpr (VEC) {
            return *reinterpret_cast<const uint4 *>(row + (c0 < lim ? c0 : lim - 8));
        } else {
            u16 v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = row[c0 + e < lim ? c0 + e : lim - 1];
            uint4 r;
            r.x = v[0] | ((uint32_t)v[1] << 16);
            r.y = v[2] | ((uint32_t)v[3] << 16);
            r.z = v[4] | ((uint32_t)v[5] << 16);
            r.w = v[6] | ((uint32_t)v[7] << 16);
            return r;
        }
    };
    auto keep8 = [](uint4 v, int c0, int lim) -> uint4 {
        auto m = [&](int e) -> uint32_t {   // mask of the 32-bit word holding entries e, e + 1
            return (c0 + e < lim ? 0xffffu : 0u) | (c0 + e + 1 < lim ? 0xffff0000u : 0u);
        };
        return uint4{v.x & m(0), v.y & m(2), v.z & m(4), v.w & m(6)};
    };

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
            ra[q] = ld8(A + (int64_t)(gr < g.M ? gr : g.M - 1) * g.lda, k0 + kc, g.K);
            if (BT) {
                const int gn = n0 + r;
                rb[q] = ld8(B + (int64_t)(gn < g.N ? gn : g.N - 1) * g.ldb, k0 + kc, g.K);
            } else {
                const int kr = c >> 4, nc = (c & 15) * 8;
                const int gk = k0 + kr;
                rb[q] = ld8(B + (int64_t)(gk < g.K ? gk : g.K - 1) * g.ldb, n0 + nc, g.N);
            }
        }
    };
    auto stash = [&](int buf, int k0) {
        const uint4 z{0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int c = tid + 256 * q;
            const int r = c >> 2, kc = (c & 3) * 8;
            const int gr = m0 + r;
            *reinterpret_cast<uint4 *>(&As[buf][r * PK + kc]) = gr < g.M ? keep8(ra[q], k0 + kc, g.K) : z;
            if (BT) {
                const int gn = n0 + r;
                *reinterpret_cast<uint4 *>(&Bs[buf][r * PK + kc]) = gn < g.N ? keep8(rb[q], k0 + kc, g.K) : z;
            } else {
                const int kr = c >> 4, nc = (c & 15) * 8;
                const uint4 v = (k0 + kr) < g.K ? keep8(rb[q], n0 + nc, g.N) : z;
                const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    Bs[buf][(nc + e) * PK + kr] = (u16)((wv[e >> 1] >> (16 * (e & 1))) & 0xffff);
            }
        }
    };

    const int nk = (g.K + TK - 1) / TK;
    if constexpr (!ASYNC) {
        fetch(0);
        stash(0, 0);
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
            if (kt + 1 < nk) stash(cur ^ 1, (kt + 1) * TK);
            __syncthreads();
        }
    } else {
        // one named LDS array per stage and operand: the compiler then sees
        // that an operand read and the loads still in flight into the other
        // stages touch different objects, and adds no wait of its own
        __shared__ __attribute__((aligned(16))) u16 A0[TM * TK], A1[TM * TK], A2[TM * TK];
        __shared__ __attribute__((aligned(16))) u16 B0[TN * TK], B1[TN * TK], B2[TN * TK];
        static_assert(NS == 3, "three named stages");
        typedef __attribute__((address_space(3))) void lds_t;
        typedef const __attribute__((address_space(1))) void glb_t;
        auto abuf = [&](auto S) -> u16 * {
            if constexpr (decltype(S)::value == 0) return A0;
            else if constexpr (decltype(S)::value == 1) return A1;
            else return A2;
        };
        auto bbuf = [&](auto S) -> u16 * {
            if constexpr (decltype(S)::value == 0) return B0;
            else if constexpr (decltype(S)::value == 1) return B1;
            else return B2;
        };
        // this lane's rows and k-chunk in the wave's two 16-row loads of A and
        // of B (wave w fills rows 32 w .. 32 w + 31 of both tiles)
        const int rr = 32 * w + (lane >> 2);                 // + 16 h
        const int ka = ((lane & 3) ^ ((rr >> 1) & 3)) * 8;   // rr + 16 takes the same chunk
        const u16 *ga[2], *gb[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int gm = m0 + rr + 16 * h, gn = n0 + rr + 16 * h;
            ga[h] = A + (int64_t)(gm < g.M ? gm : g.M - 1) * g.lda + ka;
            gb[h] = B + (int64_t)(gn < g.N ? gn : g.N - 1) * g.ldb + ka;
        }
        auto issue = [&](auto S, int kt) {
            const int k0 = kt * TK;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                __builtin_amdgcn_global_load_lds((glb_t *)(ga[h] + k0), (lds_t *)(abuf(S) + (32 * w + 16 * h) * TK),
                                                 16, 0, 0);
                __builtin_amdgcn_global_load_lds((glb_t *)(gb[h] + k0), (lds_t *)(bbuf(S) + (32 * w + 16 * h) * TK),
                                                 16, 0, 0);
            }
        };
        // operand reads: row l16 of a 16-row block (a multiple of 16 from the
        // tile's start), k-chunk lk, at its swizzled slot
        const int sw = (lk ^ ((l16 >> 1) & 3)) * 8;
        // FULL: a step of the steady state (the next step's tile in flight and
        // the one after issued here), with no conditions, so that the loop
        // body has no branches for the compiler's wait analysis to merge
        auto step = [&](auto S, auto FULL, int kt) {
            constexpr int st = decltype(S)::value;
            constexpr bool full = decltype(FULL)::value;
            // this step's tile has landed (loads complete in order; the next
            // step's four loads may stay in flight), this wave's operand
            // reads of the previous step have returned (lgkmcnt(0)), and after
            // the barrier every wave's have: the previous step's buffer is
            // refilled next
            if (full || kt + 1 < nk)
                __builtin_amdgcn_s_waitcnt(0x74);   // vmcnt(4) lgkmcnt(0)
            else
                __builtin_amdgcn_s_waitcnt(0x70);   // vmcnt(0) lgkmcnt(0)
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            const u16 *As_ = abuf(S), *Bs_ = bbuf(S);
            bf16x8 af[4], bfr[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                af[i] = *reinterpret_cast<const bf16x8 *>(&As_[(wm * 64 + i * 16 + l16) * TK + sw]);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                bfr[j] = *reinterpret_cast<const bf16x8 *>(&Bs_[(wn * 64 + j * 16 + l16) * TK + sw]);
            // the tile two steps ahead, into the buffer all waves finished with
            // (issued after this step's operand reads)
            if (full || kt + 2 < nk) issue(std::integral_constant<int, (st + 2) % 3>{}, kt + 2);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        };
        using C0 = std::integral_constant<int, 0>;
        using C1 = std::integral_constant<int, 1>;
        using C2 = std::integral_constant<int, 2>;
        using Full = std::true_type;
        using Tail = std::false_type;
        issue(C0{}, 0);   // nk >= 2 (launch condition)
        issue(C1{}, 1);
        int kt = 0;
        for (; kt + 3 <= nk - 2; kt += 3) {   // steps kt .. kt + 2 all issue the tile two ahead
            step(C0{}, Full{}, kt);
            step(C1{}, Full{}, kt + 1);
            step(C2{}, Full{}, kt + 2);
        }
        // at most four steps remain (kt a multiple of three: stages 0, 1, 2, 0)
        if (kt < nk) step(C0{}, Tail{}, kt);
        if (kt + 1 < nk) step(C1{}, Tail{}, kt + 1);
        if (kt + 2 < nk) step(C2{}, Tail{}, kt + 2);
        if (kt + 3 < nk) step(C0{}, Tail{}, kt + 3);
    }

    // register r of a lane holds row 4*(lane/16) + r, column lane%16 of its
    // 16 x 16 block (checked by the layout test)
    if ((EPI == kEpiStore || EPI == kEpiScale) && g.c_trans) {
        // C^T: a lane's four rows are consecutive in memory (one 8-byte store
        // when aligned and inside)
        const bool cvec = ((g.ldc & 3) == 0) && ((g.sC & 3) == 0) && ((reinterpret_cast<uintptr_t>(g.C) & 7) == 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row0 = m0 + wm * 64 + i * 16 + 4 * lk;
            // the scale factors of the block row, loaded before its stores
            // (in-range addresses for every lane)
            float sc[4][4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int col = n0 + wn * 64 + j * 16 + l16;
                    sc[j][r] = EPI == kEpiScale ? g.scale[(int64_t)b * g.sc_b +
                                                          (int64_t)(row0 + r < g.M ? row0 + r : 0) * g.sc_m +
                                                          (int64_t)(col < g.N ? col : 0) * g.sc_n]
                                                : 1.0f;
                }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int col = n0 + wn * 64 + j * 16 + l16;
                if (col >= g.N) continue;
                u16 h[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float v = acc[i][j][r];
                    if (EPI == kEpiScale) v *= sc[j][r];
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
        }
        return;
    }
    // The outputs of a lane in JG 16 x 16 blocks at a time (a whole block row
    // for the epilogues that update u): every value they read (scale, D, u) is
    // loaded before any of their stores, so those loads are in flight together
    // instead of one round trip per element or per block.  (The D epilogue
    // keeps one block at a time: a block row there cost a wave per SIMD of
    // occupancy and ran slower, 765 against 630 us per 512^3 product.)
    constexpr int JG = (EPI == kEpiUpdate || EPI == kEpiUpdateAcc) ? 4 : (EPI == kEpiD64 ? 2 : 1);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jh = 0; jh < 4; jh += JG) {
            float in1[JG][4];   // scale factor or FP32 D
            double in2[JG][4];
            bool ok[JG][4];
#pragma unroll
            for (int jj = 0; jj < JG; ++jj)
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
                    in1[jj][r] = 0.0f;
                    in2[jj][r] = 0.0;
                    if (EPI == kEpiScale)
                        in1[jj][r] = g.scale[(int64_t)b * g.sc_b + (int64_t)rr * g.sc_m + (int64_t)cc * g.sc_n];
                    if (EPI == kEpiUpdateAcc || (EPI == kEpiD64 && g.accumulate)) in1[jj][r] = g.D[ci];
                    if (EPI == kEpiUpdate || EPI == kEpiUpdateAcc)
                        in2[jj][r] = g.usrc[g.u0 + (int64_t)b * g.u_b + (int64_t)rr * g.u_m + (int64_t)cc * g.u_n];
                }
#pragma unroll
            for (int jj = 0; jj < JG; ++jj)
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
                        g.C[ci] = to_bf16(v * in1[jj][r]);
                    } else if (EPI == kEpiD64) {
                        g.D[ci] = g.accumulate ? (float)((double)in1[jj][r] + (double)v) : v;
                    } else {
                        const int64_t u = g.u0 + (int64_t)b * g.u_b + (int64_t)row * g.u_m + (int64_t)col * g.u_n;
                        const double du = EPI == kEpiUpdateAcc ? (double)in1[jj][r] + (double)v : (double)v;
                        g.udst[u] = fma(g.omega, du, in2[jj][r]);
                    }
                }
        }
}

template <int BT, bool VEC, bool ASYNC>
static hipError_t launch_bf16_v(const GemmBf16Args &g, int epi, hipStream_t s)
{
    const dim3 grid((unsigned)(((g.N + TN - 1) / TN) * ((g.M + TM - 1) / TM) * g.batch));
    switch (epi) {
    case kEpiStore: hipLaunchKernelGGL((k_gemm_bf16<kEpiStore, BT, VEC, ASYNC>), grid, dim3(256), 0, s, g); break;
    case kEpiScale: hipLaunchKernelGGL((k_gemm_bf16<kEpiScale, BT, VEC, ASYNC>), grid, dim3(256), 0, s, g); break;
    case kEpiUpdate: hipLaunchKernelGGL((k_gemm_bf16<kEpiUpdate, BT, VEC, ASYNC>), grid, dim3(256), 0, s, g); break;
    case kEpiD64: hipLaunchKernelGGL((k_gemm_bf16<kEpiD64, BT, VEC, ASYNC>), grid, dim3(256), 0, s, g); break;
    case kEpiUpdateAcc:
        hipLaunchKernelGGL((k_gemm_bf16<kEpiUpdateAcc, BT, VEC, ASYNC>), grid, dim3(256), 0, s, g);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Direct staging on (1) or off (0), -1: whenever the shapes allow it.
static int g_bf16_async = -1;

template <int BT>
static hipError_t launch_bf16_t(const GemmBf16Args &g, int epi, hipStream_t s)
{
    // 16-byte chunks: aligned bases, strides that keep alignment, row lengths
    // (K for A and for B given [n][k], N for B given [k][n]) multiples of 8
    const bool vec = (reinterpret_cast<uintptr_t>(g.A) % 16 == 0) && (reinterpret_cast<uintptr_t>(g.B) % 16 == 0) &&
                     g.lda % 8 == 0 && g.ldb % 8 == 0 && g.sA % 8 == 0 && g.sB % 8 == 0 && g.K % 8 == 0 &&
                     (BT || g.N % 8 == 0);
    if constexpr (BT == 1) {
        if (vec && g.K % TK == 0 && g.K >= 2 * TK && g_bf16_async != 0)
            return launch_bf16_v<1, true, true>(g, epi, s);
    }
    return vec ? launch_bf16_v<BT, true, false>(g, epi, s) : launch_bf16_v<BT, false, false>(g, epi, s);
}

void set_bf16_async(int mode) { g_bf16_async = mode; }

hipError_t launch_gemm_bf16(const GemmBf16Args &g, int b_trans, int epi, hipStream_t s)
{
    if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.batch <= 0) return hipSuccess;
    return b_trans ? launch_bf16_t<1>(g, epi, s) : launch_bf16_t<0>(g, epi, s);
}

}  // namespace bs
