// Plane-block solves by fast diagonalisation: every plane block
//   M_P = d I - eps_a (shifts along a) - eps_b (shifts along b)
// equals (S_a (x) S_b) (Lambda) (S_a (x) S_b) with the orthonormal DST-I bases
// S_a, S_b of the two in-plane axes and Lambda_pq = sigma_a,p + sigma_b,q +
// 2 eps_c, so M_P^{-1} R = S_b [ (S_b R S_a) ./ Lambda ] S_a.  The four
// transforms are batched dense products -- the one dense contraction of the
// method -- and run on the FP64 matrix cores (v_mfma_f64_16x16x4).
//
// One strided batched kernel C_b = A_b B_b (row-major, either operand may be
// shared across the batch with a zero batch stride) serves every plane
// orientation; its epilogue either stores C, stores C scaled elementwise by a
// table (the inverse eigenvalue grid), or writes dst = src + omega C straight
// into the padded u layout (the block update; for cube blocks through a
// per-row / per-column offset table).
#include <cstdint>

#include "bs_internal.h"
#include "plane.h"

namespace bs {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int kThreads = 512;   // eight wavefronts: 2 (rows) x 4 (columns) of 64 x 32

}  // namespace

// A 128 x 128 block of C per workgroup (eight wavefronts, 64 x 32 each as
// 4 x 2 blocks of 16 x 16: twice the flops per byte fetched from L2 of a
// 64 x 64 block, which L2 bandwidth holds back); K advances BK at a time
// through two LDS buffers, the next tile fetched into registers while the
// current one feeds the matrix cores (one barrier per step).
//
// Operand tiles are fetched branch-free: indices are clamped into range and
// out-of-range values replaced by zero with selects, so all of a step's loads
// are in flight together (conditional loads made the compiler wait for each
// one in turn).  VEC: both operands' rows are 16-byte aligned with even
// lengths (and an even folded axis), so pairs are single 16-byte loads.
template <int EPI, int BT, int FOLD, bool VEC>
__global__ void __launch_bounds__(kThreads) k_gemm_f64(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) double As[2][BK][BM + 2];
    __shared__ __attribute__((aligned(16))) double Bs[2][BK][BN + 2];
    // tiles numbered n fastest, then m, then the batch, each XCD taking a
    // contiguous range: the column tiles that read the same rows of A run
    // together on one XCD and share its L2
    const int nt = (g.N + BN - 1) / BN, mt = (g.M + BM - 1) / BM;
    const int t = xcd_block(blockIdx.x, gridDim.x);
    const int tn = t % nt, tr = t / nt;
    const int b = tr / mt;
    const int m0 = (tr - b * mt) * BM, n0 = tn * BN;
    const double *A = g.A + (int64_t)b * g.sA;
    const double *B = g.B + (int64_t)b * g.sB;
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int wm = w >> 2, wn = w & 3;
    const int l16 = lane & 15, lk = lane >> 4;
    // Raw operand pairs of the next step are loaded in fetch (clamped, in-range
    // addresses only) and completed in stash -- zeroed outside the operands,
    // mirrored halves added -- so the loads stay in flight while the matrix
    // cores work on the current step.
    auto ld2 = [](const double *row, int c0, int lim) -> double2 {   // c0 even
        if constexpr (VEC) {
            return *reinterpret_cast<const double2 *>(row + (c0 < lim ? c0 : lim - 2));
        } else {
            double2 v;
            v.x = row[c0 < lim ? c0 : lim - 1];
            v.y = row[c0 + 1 < lim ? c0 + 1 : lim - 1];
            return v;
        }
    };
    auto keep = [](double2 v, int c0, int lim) -> double2 {
        v.x = c0 < lim ? v.x : 0.0;
        v.y = c0 + 1 < lim ? v.y : 0.0;
        return v;
    };
    const int Kf = g.Kfull;
    const double fs = (double)g.fsign;
    double2 la[2], lb[2], lm[2];   // A pair, B pair, mirrored pair (A for FOLD 1, B for FOLD 2)
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int c = tid + kThreads * q;
            const int r = c >> 3, kc = (c & 7) * 2;
            const int gr = m0 + r;
            const double *arow = A + (int64_t)(gr < g.M ? gr : g.M - 1) * g.lda;
            la[q] = ld2(arow, k0 + kc, g.K);
            if (FOLD == 1) {
                const int k1 = k0 + kc, k2 = k1 + 1;
                if constexpr (VEC) {
                    // mirrored pair (Kf-2-k1, Kf-1-k1): one aligned 16-byte load (even Kf has no middle)
                    lm[q] = *reinterpret_cast<const double2 *>(arow + (Kf - 2 - (k1 < g.K ? k1 : g.K - 2)));
                } else {
                    lm[q].x = arow[Kf - 1 - (k1 < g.K ? k1 : g.K - 1)];
                    lm[q].y = arow[Kf - 1 - (k2 < g.K ? k2 : g.K - 1)];
                }
            }
            if (BT) {
                const int gn = n0 + r;
                lb[q] = ld2(B + (int64_t)(gn < g.N ? gn : g.N - 1) * g.ldb, k0 + kc, g.K);
            } else {
                const int kr = c >> 6, nc = (c & 63) * 2;
                const int gk = k0 + kr, gkc = gk < g.K ? gk : g.K - 1;
                lb[q] = ld2(B + (int64_t)gkc * g.ldb, n0 + nc, g.N);
                if (FOLD == 2) lm[q] = ld2(B + (int64_t)(Kf - 1 - gkc) * g.ldb, n0 + nc, g.N);
            }
        }
    };
    auto stash = [&](int buf, int k0) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int c = tid + kThreads * q;
            const int r = c >> 3, kc = (c & 7) * 2;
            const int gr = m0 + r;
            const int k1 = k0 + kc, k2 = k1 + 1;
            double2 a2 = keep(la[q], k1, g.K);
            if (FOLD == 1) {
                const double mx = VEC ? lm[q].y : lm[q].x, my = VEC ? lm[q].x : lm[q].y;
                a2.x = (k1 < g.K && Kf - 1 - k1 != k1) ? fma(fs, mx, a2.x) : a2.x;
                a2.y = (k2 < g.K && Kf - 1 - k2 != k2) ? fma(fs, my, a2.y) : a2.y;
            }
            As[buf][kc][r] = gr < g.M ? a2.x : 0.0;
            As[buf][kc + 1][r] = gr < g.M ? a2.y : 0.0;
            if (BT) {
                const int gn = n0 + r;
                const double2 b2 = keep(lb[q], k1, g.K);
                Bs[buf][kc][r] = gn < g.N ? b2.x : 0.0;
                Bs[buf][kc + 1][r] = gn < g.N ? b2.y : 0.0;
            } else {
                const int kr = c >> 6, nc = (c & 63) * 2;
                const int gk = k0 + kr;
                double2 b2 = keep(lb[q], n0 + nc, g.N);
                if (FOLD == 2) {
                    const double2 m = keep(lm[q], n0 + nc, g.N);
                    const bool use = Kf - 1 - gk != gk;
                    b2.x = use ? fma(fs, m.x, b2.x) : b2.x;
                    b2.y = use ? fma(fs, m.y, b2.y) : b2.y;
                }
                Bs[buf][kr][nc] = gk < g.K ? b2.x : 0.0;
                Bs[buf][kr][nc + 1] = gk < g.K ? b2.y : 0.0;
            }
        }
    };

    dbl4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

    const int nk = (g.K + BK - 1) / BK;
    fetch(0);
    stash(0, 0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) fetch((kt + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            double af[4], bf[2];
#pragma unroll
            for (int i = 0; i < 4; ++i) af[i] = As[cur][kk + lk][wm * 64 + i * 16 + l16];
#pragma unroll
            for (int j = 0; j < 2; ++j) bf[j] = Bs[cur][kk + lk][wn * 32 + j * 16 + l16];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        if (kt + 1 < nk) stash(cur ^ 1, (kt + 1) * BK);
        __syncthreads();
    }

    // D layout of the FP64 16x16 block: register r of a lane holds row
    // 4*r + lane/16, column lane%16 (checked by the layout test).  Per block,
    // the values the four outputs of a lane read (scale or u) are loaded
    // before any of their stores, so they are in flight together.
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            double in[4];
            bool ok[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int pr = m0 + wm * 64 + i * 16 + r * 4 + lk;
                const int pcl = n0 + wn * 32 + j * 16 + l16;
                bool o = pr < g.M && pcl < g.N;
                const int row = o ? (g.row_s ? pr * g.row_s + g.row_o : pr) : 0;
                const int col = o ? (g.row_s ? pcl * g.col_s + g.col_o : pcl) : 0;
                if (EPI == kEpiUpdate) o = o && !(g.ncolour >= 0 && ((col + g.colour_shift) & 1) != g.ncolour);
                ok[r] = o;
                in[r] = 0.0;
                if (EPI == kEpiScale)
                    in[r] = g.scale[(int64_t)b * g.sc_b + (int64_t)(o ? row : 0) * g.sc_m + (int64_t)(o ? col : 0) * g.sc_n];
                if (EPI == kEpiUpdate)
                    in[r] = g.usrc[g.u0 + (int64_t)b * g.u_b + (int64_t)(o ? row : 0) * g.u_m + (int64_t)(o ? col : 0) * g.u_n];
                if (EPI == kEpiGather) in[r] = g.usrc[o ? g.ebase[pr] + g.eoff[pcl] : g.ebase[0]];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (!ok[r]) continue;
                const int pr = m0 + wm * 64 + i * 16 + r * 4 + lk;
                const int pcl = n0 + wn * 32 + j * 16 + l16;
                const int row = g.row_s ? pr * g.row_s + g.row_o : pr;
                const int col = g.row_s ? pcl * g.col_s + g.col_o : pcl;
                const double v = acc[i][j][r];
                if (EPI == kEpiStore) {
                    g.C[(int64_t)b * g.sC + (int64_t)row * g.ldc + col] = v;
                } else if (EPI == kEpiScale) {
                    g.C[(int64_t)b * g.sC + (int64_t)row * g.ldc + col] = v * in[r];
                } else if (EPI == kEpiGather) {
                    g.udst[g.ebase[pr] + g.eoff[pcl]] = fma(g.omega, v, in[r]);
                } else {
                    const int64_t u = g.u0 + (int64_t)b * g.u_b + (int64_t)row * g.u_m + (int64_t)col * g.u_n;
                    g.udst[u] = fma(g.omega, v, in[r]);
                }
            }
        }
}

template <int BT, int FOLD, bool VEC>
static hipError_t launch_f64_v(const GemmArgs &g, int epi, hipStream_t s)
{
    const dim3 grid((unsigned)(((g.N + BN - 1) / BN) * ((g.M + BM - 1) / BM) * g.batch));
    switch (epi) {
    case kEpiStore: hipLaunchKernelGGL((k_gemm_f64<kEpiStore, BT, FOLD, VEC>), grid, dim3(kThreads), 0, s, g); break;
    case kEpiScale: hipLaunchKernelGGL((k_gemm_f64<kEpiScale, BT, FOLD, VEC>), grid, dim3(kThreads), 0, s, g); break;
    case kEpiUpdate: hipLaunchKernelGGL((k_gemm_f64<kEpiUpdate, BT, FOLD, VEC>), grid, dim3(kThreads), 0, s, g); break;
    case kEpiGather:
        if constexpr (BT == 1 && FOLD == 0) {
            hipLaunchKernelGGL((k_gemm_f64<kEpiGather, BT, FOLD, VEC>), grid, dim3(kThreads), 0, s, g);
            break;
        } else {
            return hipErrorInvalidValue;
        }
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int BT, int FOLD>
static hipError_t launch_f64_t(const GemmArgs &g, int epi, hipStream_t s)
{
    // 16-byte pairs: aligned operand bases and row strides, even row lengths
    // (K for A and for B given [n][k], N for B given [k][n]) and, for A's
    // mirrored pairs, an even folded axis; every batch stride keeps alignment
    const bool vec = (reinterpret_cast<uintptr_t>(g.A) % 16 == 0) && (reinterpret_cast<uintptr_t>(g.B) % 16 == 0) &&
                     g.lda % 2 == 0 && g.ldb % 2 == 0 && g.sA % 2 == 0 && g.sB % 2 == 0 && g.K % 2 == 0 &&
                     (BT || g.N % 2 == 0) && (FOLD != 1 || g.Kfull % 2 == 0) && g.K >= 2 && (BT || g.N >= 2);
    return vec ? launch_f64_v<BT, FOLD, true>(g, epi, s) : launch_f64_v<BT, FOLD, false>(g, epi, s);
}

hipError_t launch_gemm_f64(const GemmArgs &g, int epi, hipStream_t s)
{
    if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.batch <= 0) return hipSuccess;
    if (g.fold < 0 || g.fold > 2) return hipErrorInvalidValue;
    // the combinations the plane chain uses (and the plain product)
    if (g.fold == 0) return g.b_trans ? launch_f64_t<1, 0>(g, epi, s) : launch_f64_t<0, 0>(g, epi, s);
    if (g.fold == 1) return g.b_trans ? launch_f64_t<1, 1>(g, epi, s) : launch_f64_t<0, 1>(g, epi, s);
    return g.b_trans ? launch_f64_t<1, 2>(g, epi, s) : launch_f64_t<0, 2>(g, epi, s);
}

}  // namespace bs
