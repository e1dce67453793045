// Plane-block solves: batched dense products for fast diagonalisation.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace bs {

enum { kEpiStore = 0, kEpiScale = 1, kEpiUpdate = 2, kEpiD64 = 3, kEpiUpdateAcc = 4, kEpiGather = 5 };

// C_b = A_b B_b, row-major, b in [0, batch); a zero batch stride shares an
// operand across the batch.  Epilogues:
//   kEpiStore:  C = A B
//   kEpiScale:  C = (A B) .* scale[b*sc_b + m*sc_m + n*sc_n]
//   kEpiUpdate: udst[u] = usrc[u] + omega (A B), u = u0 + b*u_b + m*u_m + n*u_n,
//               for columns n with (n + colour_shift) % 2 == ncolour (all if ncolour < 0)
//   kEpiGather: udst[u] = usrc[u] + omega (A B), u = ebase[m] + eoff[n] (rows
//               are cube blocks, columns the cells of a block; FP64 only,
//               b_trans = 1, fold = 0)
struct GemmArgs {
    const double *A;
    int64_t lda, sA;
    const double *B;
    int64_t ldb, sB;
    double *C;
    int64_t ldc, sC;
    int M, N, K, batch;
    const double *scale;
    int64_t sc_b, sc_m, sc_n;
    const double *usrc;
    double *udst;
    int64_t u0, u_b, u_m, u_n;
    double omega;
    int ncolour, colour_shift;
    // Options (zero-initialised = plain product):
    //   b_trans: B stored as [n][k] (element (k, n) at n*ldb + k);
    //   fold 1 / 2: the contraction runs over K entries of A's rows / B's
    //     columns folded about the middle of a length-Kfull axis:
    //     x'[k] = x[k] + fsign * x[Kfull-1-k] (x[k] alone where k = Kfull-1-k),
    //     the even/odd split of a product with a DST-I basis;
    //   row_s, row_o, col_s, col_o: the product's row m / column n stands for
    //     the logical row m*row_s + row_o / column n*col_s + col_o of C, of the
    //     scale grid and of the u mapping (1, 0, 1, 0 if row_s = 0).
    int b_trans, fold, Kfull, fsign;
    int row_s, row_o, col_s, col_o;
    const int64_t *ebase;
    const int32_t *eoff;
};

hipError_t launch_gemm_f64(const GemmArgs &g, int epi, hipStream_t s);

// The same product with float operands and FP32 accumulation (prec 1: FP32
// products); kEpiD64 stores (or adds, accumulate != 0) the result into the
// FP64 array D with C's indexing.  dlayout selects the register-to-row
// mapping of the 16x16 result block (0: 4*(lane/16)+r).  b_trans, fold,
// Kfull, fsign and row_s / row_o / col_s / col_o as in GemmArgs (the even /
// odd halves of a DST-I product), with these combinations: b_trans 0 and
// fold 0 or 2, b_trans 1 and fold 1.
struct GemmMixedArgs {
    const float *A;
    int64_t lda, sA;
    const float *B;
    int64_t ldb, sB;
    float *C;
    int64_t ldc, sC;
    int M, N, K, batch;
    const float *scale;
    int64_t sc_b, sc_m, sc_n;
    double *D;
    int accumulate;
    const double *usrc;
    double *udst;
    int64_t u0, u_b, u_m, u_n;
    double omega;
    int ncolour, colour_shift;
    int dlayout;
    int b_trans, fold, Kfull, fsign;
    int row_s, row_o, col_s, col_o;
};

hipError_t launch_gemm_mixed(const GemmMixedArgs &g, int prec, int epi, hipStream_t s);

// The same product with BF16 operands in memory (unsigned short bit patterns)
// and FP32 accumulation.  A is [m][k] (k contiguous, leading dimension lda);
// B is [n][k] with leading dimension ldb when b_trans != 0, else [k][n].
// Store / scale epilogues write BF16 C; kEpiD64 and kEpiUpdate as above, with
// the correction D held in FP32; kEpiUpdateAcc: udst[u] = usrc[u] +
// omega (D + C) in FP64 (the last defect step of a refined solve applied
// straight to u; D with C's indexing).
struct GemmBf16Args {
    const unsigned short *A;
    int64_t lda, sA;
    const unsigned short *B;
    int64_t ldb, sB;
    unsigned short *C;
    int64_t ldc, sC;
    int M, N, K, batch;
    const float *scale;
    int64_t sc_b, sc_m, sc_n;
    float *D;
    int accumulate;
    const double *usrc;
    double *udst;
    int64_t u0, u_b, u_m, u_n;
    double omega;
    int ncolour, colour_shift;
    int c_trans;   // store / scale epilogues: element (m, n) of C at b*sC + n*ldc + m (C^T)
};

hipError_t launch_gemm_bf16(const GemmBf16Args &g, int b_trans, int epi, hipStream_t s);
// Operand staging of the BF16 products: 1 direct to LDS where the shapes allow
// it, 0 always through registers, -1 (default) as 1.
void set_bf16_async(int mode);
hipError_t launch_plane_defect(const double *R, const double *D, float *E, int nx, int ny, int nz, int normal,
                               const double eps[3], hipStream_t s);
// The same defect from FP32 R and D (formed in FP64), rounded to BF16 (bit
// patterns).
hipError_t launch_plane_defect_bf16(const float *R, const float *D, unsigned short *E, int nx, int ny, int nz,
                                    int normal, const double eps[3], hipStream_t s);

}  // namespace bs
