"""The allocation-free residual entry point (bs_residual_noalloc), called
through the C ABI, against bs_residual on the same inputs: the same kernels
and reduction order, so r and the per-patch norms agree bit for bit; two calls
in a row, the second on a smaller patch set, so stale partial sums from the
first call cannot leak into the second; and a patch set with more residual
tiles than the static scratch holds is refused."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1208_1975_amd as bs
from gpu_util import need_gpu
from workloads import c4_patchset, small_patch

pytestmark = pytest.mark.gpu


def _noalloc(ps, u, f, r, n2):
    L = bs.lib()
    fn = L.bs_residual_noalloc
    fn.argtypes = [ctypes.c_void_p] * 6
    fn.restype = ctypes.c_int
    st = fn(ps.handle, bs._ptr(u), bs._ptr(f), bs._ptr(r), bs._ptr(n2),
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def _case(patches):
    ps = bs.PatchSet([p.dims for p in patches], [p.eps for p in patches], [p.h for p in patches])
    u = ps.pack_u([p.u0 for p in patches])
    f = ps.pack_f([p.f for p in patches])
    return ps, u, f


def test_noalloc_residual_matches_bs_residual_twice():
    need_gpu()
    big = [small_patch(96, 80, 70, seed=1, eps=(1.0, 2.0, 30.0)), small_patch(33, 17, 9, seed=2)]
    small = [small_patch(12, 10, 9, seed=3, eps=(3.0, 1.0, 1.0))]
    for patches in (big, small):
        ps, u, f = _case(patches)
        r_ref, n_ref = ps.empty_f(), torch.zeros(ps.npatch, dtype=torch.float64, device="cuda")
        ps.residual(u, f, r_ref, n_ref)
        r, n2 = torch.full_like(r_ref, np.nan), torch.full_like(n_ref, np.nan)
        assert _noalloc(ps, u, f, r, n2) == bs.BS_OK
        torch.cuda.synchronize()
        assert torch.equal(n2, n_ref)
        for q in range(ps.npatch):
            assert torch.equal(ps.view_f(r, q), ps.view_f(r_ref, q))
        # norms only
        n3 = torch.full_like(n_ref, np.nan)
        assert _noalloc(ps, u, f, None, n3) == bs.BS_OK
        torch.cuda.synchronize()
        assert torch.equal(n3, n_ref)
        ps.close()


def test_noalloc_refuses_oversized_and_bad_arguments():
    need_gpu()
    ps, u, f = _case([small_patch(8, 8, 8, seed=4)])
    assert _noalloc(ps, u, f, None, None) == bs.BS_ERR_INVALID
    ps.close()
    # 66000 one-cell patches: one residual tile each, more than the static
    # scratch holds (65536); the 3000-patch uneven set (about 18000 tiles) fits
    n = 66000
    ps = bs.PatchSet([(1, 1, 1)] * n, [(1.0, 1.0, 1.0)] * n, [1.0] * n)
    n2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    u = torch.zeros(ps.u_numel, dtype=torch.float64, device="cuda")
    f = torch.zeros(ps.f_numel, dtype=torch.float64, device="cuda")
    assert _noalloc(ps, u, f, None, n2) == bs.BS_ERR_UNSUPPORTED
    assert "static scratch" in bs.bs_last_error()
    ps.close()
    s = c4_patchset(npatch=3000)
    ps = bs.PatchSet([tuple(d) for d in s.dims], [tuple(e) for e in s.eps], list(s.h))
    u, f = ps.pack_u(s.u0), ps.pack_f(s.f)
    n_ref = torch.zeros(ps.npatch, dtype=torch.float64, device="cuda")
    ps.residual(u, f, None, n_ref)
    n2 = torch.full_like(n_ref, np.nan)
    assert _noalloc(ps, u, f, None, n2) == bs.BS_OK
    torch.cuda.synchronize()
    assert torch.equal(n2, n_ref)
    ps.close()
