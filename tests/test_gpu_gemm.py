"""The plane path's batched FP64 matrix-core product against NumPy."""
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


@pytest.mark.parametrize("prec,tol", [(1, 1e-5), (2, 2e-2)])
@pytest.mark.parametrize("M,N,K,batch", [(64, 64, 32, 1), (100, 130, 70, 3), (512, 64, 512, 2), (5, 7, 3, 2)])
def test_mixed_gemm_matches_numpy(prec, tol, M, N, K, batch):
    """FP32 / BF16 products with FP32 accumulation: relative to the FP64 product
    of the same float inputs, within the precision's rounding (BF16: 8 bits)."""
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


@pytest.mark.parametrize("prec", [1, 2])
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
