"""The plane path's batched matrix-core products (FP64, FP32, BF16) against NumPy."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1208_1975_amd as bs
from gpu_util import need_gpu

pytestmark = pytest.mark.gpu


def gemm(A, lda, sA, B, ldb, sB, C, ldc, sC, M, N, K, batch, epi=0, scale=None, sc=(0, 0, 0)):
    L = bs.lib()
    f = L.bsi_gemm_f64
    i64, vp = ctypes.c_int64, ctypes.c_void_p
    f.argtypes = [vp, i64, i64, vp, i64, i64, vp, i64, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                  ctypes.c_int, vp, i64, i64, i64, vp]
    f.restype = ctypes.c_int
    st = torch.cuda.current_stream().cuda_stream
    rc = f(A.data_ptr(), lda, sA, B.data_ptr(), ldb, sB, C.data_ptr(), ldc, sC, M, N, K, batch, epi,
           scale.data_ptr() if scale is not None else None, sc[0], sc[1], sc[2], st)
    assert rc == 0
    torch.cuda.synchronize()


@pytest.mark.parametrize("M,N,K,batch", [(16, 16, 4, 1), (64, 64, 16, 1), (5, 7, 3, 2), (100, 130, 70, 3),
                                         (512, 64, 512, 2), (1, 1, 1, 1), (65, 17, 33, 4)])
def test_gemm_matches_numpy(M, N, K, batch):
    need_gpu()
    rng = np.random.default_rng(M * 1000 + N)
    A = rng.standard_normal((batch, M, K))
    B = rng.standard_normal((batch, K, N))
    ref = A @ B
    tA = torch.tensor(A, device="cuda")
    tB = torch.tensor(B, device="cuda")
    tC = torch.zeros((batch, M, N), dtype=torch.float64, device="cuda")
    gemm(tA, K, M * K, tB, N, K * N, tC, N, M * N, M, N, K, batch)
    got = tC.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_gemm_shared_operand_and_scale():
    need_gpu()
    rng = np.random.default_rng(7)
    M = N = K = 48
    batch = 3
    S = rng.standard_normal((K, N))
    A = rng.standard_normal((batch, M, K))
    sc = rng.standard_normal((M, N))
    ref = (A @ S) * sc
    tA, tS = torch.tensor(A, device="cuda"), torch.tensor(S, device="cuda")
    tsc = torch.tensor(sc, device="cuda")
    tC = torch.zeros((batch, M, N), dtype=torch.float64, device="cuda")
    gemm(tA, K, M * K, tS, N, 0, tC, N, M * N, M, N, K, batch, epi=1, scale=tsc, sc=(0, N, 1))
    assert np.max(np.abs(tC.cpu().numpy() - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_gemm_output_layout_probe():
    """A = row index pattern, B = identity: C must equal A (exposes any
    misplaced row or column of the matrix-core result layout)."""
    need_gpu()
    M = N = K = 64
    A = np.arange(M * K, dtype=np.float64).reshape(M, K)
    B = np.eye(K)
    tA, tB = torch.tensor(A, device="cuda"), torch.tensor(B, device="cuda")
    tC = torch.zeros((M, N), dtype=torch.float64, device="cuda")
    gemm(tA, K, 0, tB, N, 0, tC, N, 0, M, N, K, 1)
    got = tC.cpu().numpy()
    bad = np.argwhere(got != A)
    print("mismatches", len(bad), bad[:8].tolist(), [got[tuple(b)] for b in bad[:8]])
    assert len(bad) == 0


def gemm_mixed(A, lda, sA, B, ldb, sB, C, ldc, sC, M, N, K, batch, prec, dlayout):
    L = bs.lib()
    f = L.bsi_gemm_mixed
    i64, vp = ctypes.c_int64, ctypes.c_void_p
    f.argtypes = [vp, i64, i64, vp, i64, i64, vp, i64, i64] + [ctypes.c_int] * 6 + [vp]
    f.restype = ctypes.c_int
    rc = f(A.data_ptr(), lda, sA, B.data_ptr(), ldb, sB, C.data_ptr(), ldc, sC, M, N, K, batch, prec, dlayout,
           torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec,tol", [(1, 1e-5)])
@pytest.mark.parametrize("M,N,K,batch", [(64, 64, 32, 1), (100, 130, 70, 3), (512, 64, 512, 2), (5, 7, 3, 2)])
def test_mixed_gemm_matches_numpy(prec, tol, M, N, K, batch):
    """FP32 products with FP32 accumulation: relative to the FP64 product of
    the same float inputs, within FP32 rounding."""
    need_gpu()
    rng = np.random.default_rng(M + 7 * N + prec)
    A = rng.standard_normal((batch, M, K)).astype(np.float32)
    B = rng.standard_normal((batch, K, N)).astype(np.float32)
    ref = A.astype(np.float64) @ B.astype(np.float64)
    tA, tB = torch.tensor(A, device="cuda"), torch.tensor(B, device="cuda")
    tC = torch.zeros((batch, M, N), dtype=torch.float32, device="cuda")
    gemm_mixed(tA, K, M * K, tB, N, K * N, tC, N, M * N, M, N, K, batch, prec, 0)
    err = np.max(np.abs(tC.cpu().numpy() - ref)) / (np.sqrt(K) * np.max(np.abs(A)) * np.max(np.abs(B)))
    assert err < tol


@pytest.mark.parametrize("prec", [1])
def test_mixed_output_layout_probe(prec):
    """A = small integers (exact in BF16), B = identity: C must equal A."""
    need_gpu()
    M = N = K = 64
    A = (np.arange(M * K) % 97).astype(np.float32).reshape(M, K)
    B = np.eye(K, dtype=np.float32)
    tA, tB = torch.tensor(A, device="cuda"), torch.tensor(B, device="cuda")
    good = []
    for dl in (0, 1):
        tC = torch.zeros((M, N), dtype=torch.float32, device="cuda")
        gemm_mixed(tA, K, 0, tB, N, 0, tC, N, 0, M, N, K, 1, prec, dl)
        if np.array_equal(tC.cpu().numpy(), A):
            good.append(dl)
    print("prec %d: matching result layouts %s" % (prec, good))
    assert good == [0]


def gemm_bf16(A, lda, sA, B, ldb, sB, b_trans, C, ldc, sC, M, N, K, batch, epi=0, scale=None, sc=(0, 0, 0)):
    L = bs.lib()
    f = L.bsi_gemm_bf16
    i64, vp, ci = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
    f.argtypes = [vp, i64, i64, vp, i64, i64, ci, vp, i64, i64, ci, ci, ci, ci, ci, vp, i64, i64, i64, vp]
    f.restype = ctypes.c_int
    rc = f(A.data_ptr(), lda, sA, B.data_ptr(), ldb, sB, b_trans, C.data_ptr(), ldc, sC, M, N, K, batch, epi,
           scale.data_ptr() if scale is not None else None, sc[0], sc[1], sc[2], torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    torch.cuda.synchronize()


def _bf16_case(M, N, K, batch, seed):
    rng = np.random.default_rng(seed)
    tA = torch.tensor(rng.standard_normal((batch, M, K)), dtype=torch.bfloat16, device="cuda")
    tB = torch.tensor(rng.standard_normal((batch, K, N)), dtype=torch.bfloat16, device="cuda")
    A = tA.float().cpu().numpy().astype(np.float64)    # the exact BF16 inputs
    B = tB.float().cpu().numpy().astype(np.float64)
    return tA, tB, A, B


def _bf16_check(tC, ref, K, A, B):
    """FP32 accumulation of exact BF16 products, then one rounding to BF16:
    |C - ref| <= 2^-8 |ref| + K 2^-21 max|A| max|B| elementwise (rounding of
    the result plus a generous FP32 accumulation allowance)."""
    got = tC.float().cpu().numpy().astype(np.float64)
    bound = 2.0 ** -8 * np.abs(ref) + K * 2.0 ** -21 * np.max(np.abs(A)) * np.max(np.abs(B))
    bad = np.argwhere(np.abs(got - ref) > bound)
    assert len(bad) == 0, (bad[:5].tolist(), got[tuple(bad[0])], ref[tuple(bad[0])])


@pytest.mark.parametrize("M,N,K,batch", [(128, 128, 32, 1), (256, 128, 96, 2), (100, 130, 70, 3), (5, 7, 3, 2),
                                         (512, 512, 512, 1), (1, 1, 1, 1), (33, 200, 41, 2)])
@pytest.mark.parametrize("b_trans", [0, 1])
def test_bf16_gemm_matches_numpy(M, N, K, batch, b_trans):
    """BF16 operands, FP32 accumulation, BF16 result, for B given as [k][n] or
    as [n][k]; odd sizes exercise the unaligned (element-wise) loads."""
    need_gpu()
    tA, tB, A, B = _bf16_case(M, N, K, batch, M * 31 + N + K + b_trans)
    ref = A @ B
    tC = torch.zeros((batch, M, N), dtype=torch.bfloat16, device="cuda")
    if b_trans:
        tBt = tB.transpose(1, 2).contiguous()      # [n][k]
        gemm_bf16(tA, K, M * K, tBt, K, N * K, 1, tC, N, M * N, M, N, K, batch)
    else:
        gemm_bf16(tA, K, M * K, tB, N, K * N, 0, tC, N, M * N, M, N, K, batch)
    _bf16_check(tC, ref, K, A, B)


def test_bf16_gemm_shared_operand_and_scale():
    need_gpu()
    M = N = K = 96
    batch = 3
    tA, _, A, _ = _bf16_case(M, N, K, batch, 5)
    rng = np.random.default_rng(6)
    tS = torch.tensor(rng.standard_normal((K, N)), dtype=torch.bfloat16, device="cuda")
    S = tS.float().cpu().numpy().astype(np.float64)
    sc = rng.standard_normal((M, N)).astype(np.float32)
    tsc = torch.tensor(sc, device="cuda")
    ref = (A @ S) * sc.astype(np.float64)
    tC = torch.zeros((batch, M, N), dtype=torch.bfloat16, device="cuda")
    gemm_bf16(tA, K, M * K, tS, N, 0, 0, tC, N, M * N, M, N, K, batch, epi=1, scale=tsc, sc=(0, N, 1))
    _bf16_check(tC, ref, K, A, S * np.max(np.abs(sc)))


def test_bf16_gemm_output_layout_probe():
    """A = small integers (exact in BF16), B = identity: C must equal A."""
    need_gpu()
    M = N = K = 128
    A = (np.arange(M * K) % 97).astype(np.float32).reshape(M, K)
    tA = torch.tensor(A, dtype=torch.bfloat16, device="cuda")
    tB = torch.eye(K, dtype=torch.bfloat16, device="cuda")
    for bt in (0, 1):
        tC = torch.zeros((M, N), dtype=torch.bfloat16, device="cuda")
        gemm_bf16(tA, K, 0, tB, N, 0, bt, tC, N, 0, M, N, K, 1)
        assert np.array_equal(tC.float().cpu().numpy(), A), bt


def _set_bf16_async(mode):
    L = bs.lib()
    L.bsi_set_bf16_async.argtypes = [ctypes.c_int]
    L.bsi_set_bf16_async.restype = ctypes.c_int
    assert L.bsi_set_bf16_async(mode) == 0


@pytest.mark.parametrize("K", [64, 96, 128, 160, 192, 224, 512])
@pytest.mark.parametrize("M,N,batch", [(200, 136, 2), (128, 128, 1), (17, 300, 3)])
def test_bf16_direct_staging_matches_register_staging(M, N, K, batch):
    """B given [n][k] with K a multiple of 32: the products that stage their
    operand tiles straight into LDS (three stages, swizzled slots) give the
    bit pattern of the register-staged ones (same products in the same order),
    for every count of K steps (2 to 16: every tail of the three-stage loop)
    and for row counts that are not multiples of the 128-row tile."""
    need_gpu()
    tA, tB, A, B = _bf16_case(M, N, K, batch, M + 7 * N + K)
    tBt = tB.transpose(1, 2).contiguous()      # [n][k]
    out = {}
    try:
        for mode in (0, 1):
            _set_bf16_async(mode)
            tC = torch.zeros((batch, M, N), dtype=torch.bfloat16, device="cuda")
            gemm_bf16(tA, K, M * K, tBt, K, N * K, 1, tC, N, M * N, M, N, K, batch)
            out[mode] = tC
    finally:
        _set_bf16_async(-1)
    assert torch.equal(out[0], out[1])
    _bf16_check(out[1], A @ B, K, A, B)
