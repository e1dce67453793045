"""GPU parity of the z-marching x-line kernel (x-lines of up to 64 cells; a
work item is a block of rows marched along z with each line's z-neighbours in
registers).

Jacobi is deterministic: every shape and item split matches the oracle's
Jacobi line sweeps to 1e-12.  Chaotic GS orders the lines of one item as
two-colour within each plane and lexicographically along z; when one item
covers a patch that order is a fixed sequence of line updates, which the
oracle reproduces line by line (oracle.line_update_some) to 1e-12.  On the
3000-patch set the chaotic residual after 5, 10, 15 and 20 sweeps stays within
the oracle's two-colour GS."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1208_1975_amd as bs
from conftest import relerr
from gpu_util import log, need_gpu
from workloads import c4_patchset, small_patch

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _setup():
    need_gpu()
    oracle.set_threads(0)
    yield


SHAPES = [(16, 20, 12), (24, 7, 9), (64, 33, 17), (5, 3, 40), (1, 4, 6), (48, 16, 16), (33, 64, 5), (63, 2, 3)]


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("waves,planes", [(4, 0), (2, 3), (1, 1)])
def test_xz_jacobi_matches_oracle(dims, waves, planes):
    p = small_patch(*dims, seed=91, eps=(2.0, 1.0, 5.0))
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    ps.set_xz_config("jacobi", waves, planes)
    assert ps.line_config(0, "jacobi")["form"] == 2
    for nsweeps in (1, 2, 3):
        u, f, w = ps.pack_u([p.u0]), ps.pack_f([p.f]), ps.empty_u()
        ps.line_relax(0, "jacobi", 0.8, nsweeps, u, f, w)
        torch.cuda.synchronize()
        ref = oracle.line_sweeps(p.u0, p.f, p.eps, p.h, 0, oracle.JACOBI, 0.8, nsweeps)
        assert relerr(ps.view_u(u, 0).cpu().numpy(), ref) < TOL, nsweeps
    ps.close()


def _xz_order_reference(p, nsweeps):
    """The chaotic z-marching order of one item covering the patch: plane by
    plane in increasing k, the colour-0 lines ((j + k) even) then colour 1."""
    u = p.u0.copy()
    nx, ny, nz = p.dims
    for _ in range(nsweeps):
        for k in range(nz):
            for c in (0, 1):
                lines = [(j, k) for j in range(ny) if (j + k) % 2 == c]
                if lines:
                    u = oracle.line_update_some(u, p.f, p.eps, p.h, 0, 1.0, lines)
    return u


@pytest.mark.parametrize("dims", [(16, 20, 12), (8, 64, 7), (3, 9, 11), (16, 1, 5)])
def test_xz_chaotic_single_item_is_plane_two_colour_z_lexicographic(dims):
    p = small_patch(*dims, seed=17, eps=(1.0, 4.0, 2.0))
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    nz = dims[2]
    ps.set_xz_config("chaotic", 4, nz)   # nx <= 16: 64 rows per item, one item per patch
    for nsweeps in (1, 2):
        u, f = ps.pack_u([p.u0]), ps.pack_f([p.f])
        ps.line_relax(0, "chaotic", 1.0, nsweeps, u, f)
        torch.cuda.synchronize()
        ref = _xz_order_reference(p, nsweeps)
        assert relerr(ps.view_u(u, 0).cpu().numpy(), ref) < TOL
    ps.close()


def test_xz_chaotic_c4_within_two_colour_gs():
    s = c4_patchset()
    ps = bs.PatchSet([tuple(d) for d in s.dims], [tuple(e) for e in s.eps], list(s.h))
    ps.set_xz_config("chaotic", 4, 0)
    u, f = ps.pack_u(s.u0), ps.pack_f(s.f)
    norms = []
    for blk in range(4):
        ps.line_relax(0, "chaotic", 1.0, 5, u, f)
        n1 = torch.zeros(ps.npatch, dtype=torch.float64, device="cuda")
        ps.residual(u, f, None, n1)
        norms.append(n1)
    torch.cuda.synchronize()
    rk = [n.sqrt().cpu().numpy() for n in norms]
    rng = np.random.default_rng(1)
    worst = [0.0] * 4
    for p in rng.choice(ps.npatch, 24, replace=False):
        ref = s.u0[p]
        for blk in range(4):
            ref = oracle.line_sweeps(ref, s.f[p], tuple(s.eps[p]), s.h[p], 0, oracle.COLORED_GS, 1.0, 5)
            rr = math.sqrt(oracle.residual(ref, s.f[p], tuple(s.eps[p]), s.h[p])[1])
            worst[blk] = max(worst[blk], rk[blk][p] / rr)
            assert rk[blk][p] / rr <= 1.15, (p, 5 * (blk + 1), rk[blk][p] / rr)
    log("xz chaotic / two-colour GS worst sampled ratio at 5/10/15/20: %s" % " ".join("%.4f" % w for w in worst))
    ps.close()


def test_xz_refuses_coloured_gs_and_long_lines():
    p = small_patch(65, 4, 4, seed=1)
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    with pytest.raises(bs.BSError):
        ps.set_xz_config("jacobi", 4, 0)     # x-lines longer than 64
    ps.close()
    p = small_patch(16, 4, 4, seed=1)
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    with pytest.raises(bs.BSError):
        ps.set_xz_config("colored", 4, 0)    # two-colour GS keeps the other forms
    ps.close()
