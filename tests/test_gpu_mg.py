"""GPU parity of the multigrid V-cycle with block smoothers against the
oracle's cycle (section 1: line and plane smoothers inside geometric
multigrid; section 5: multilevel use): the same transfers, coarse equations
and smoothing sweeps, so deterministic smoothers (Jacobi, two-colour GS) agree
to 1e-12 per cycle; the cycle's convergence factor stays small and
independent of the grid size, as the oracle's does."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1208_1975_amd as bs
from conftest import relerr
from gpu_util import log, need_gpu
from workloads import make_patch, small_patch

pytestmark = pytest.mark.gpu

TOL = 1e-12
OSCH = {"jacobi": oracle.JACOBI, "colored": oracle.COLORED_GS}


@pytest.fixture(scope="module", autouse=True)
def _setup():
    need_gpu()
    oracle.set_threads(0)
    yield


def _run(p, kind, arg, scheme, omega, nu1, nu2, ncoarse, levels, bc, cbc, ncycles):
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    if bc:
        ps.set_bc([bc])
    mg = bs.Multigrid(ps, kind, arg, scheme, omega, nu1, nu2, ncoarse, levels, cbc)
    u, f, w = ps.pack_u([p.u0]), ps.pack_f([p.f]), ps.empty_u()
    outs = []
    for _ in range(ncycles):
        mg.vcycle(u, f, w)
        torch.cuda.synchronize()
        outs.append(ps.view_u(u, 0).cpu().numpy().copy())
    lv = mg.levels
    mg.close()
    ps.close()
    return outs, lv


@pytest.mark.parametrize("kind,arg", [("line", 0), ("line", 2), ("plane", 0), ("plane", 2)])
@pytest.mark.parametrize("scheme", ["jacobi", "colored"])
@pytest.mark.parametrize("bc,cbc", [(0, 0), (0, 63), (63, 63), (12, 63)])
def test_vcycle_matches_oracle(kind, arg, scheme, bc, cbc):
    p = small_patch(16, 8, 12, seed=21, eps=(1.0, 3.0, 20.0))
    omega = 0.8 if scheme == "jacobi" else 1.0
    log("vcycle %s %d %s bc=%d cbc=%d" % (kind, arg, scheme, bc, cbc))
    # three cycles: eager, captured, replayed
    outs, lv = _run(p, kind, arg, scheme, omega, 2, 1, 6, 0, bc, cbc, 3)
    assert lv == oracle.mg_levels(p.dims) == 3
    ref = p.u0
    for c in range(3):
        ref = oracle.vcycle(ref, p.f, p.eps, p.h, kind, arg, OSCH[scheme], omega, 2, 1, 6, bc=bc, coarse_bc=cbc)
        got = outs[c]
        assert relerr(got[1:-1, 1:-1, 1:-1], ref[1:-1, 1:-1, 1:-1]) < TOL, c


def test_vcycle_two_levels_and_multi_patch():
    """levels = 2 and a set of two different patches (each coarsened on its own)."""
    p1 = small_patch(8, 12, 16, seed=3, eps=(1.0, 1.0, 30.0))
    p2 = small_patch(20, 6, 10, seed=4, eps=(5.0, 1.0, 2.0))
    ps = bs.PatchSet([p1.dims, p2.dims], [p1.eps, p2.eps], [p1.h, p2.h])
    mg = bs.Multigrid(ps, "line", 2, "colored", 1.0, 1, 1, 30, 2, 63)
    assert mg.levels == 2
    u, f = ps.pack_u([p1.u0, p2.u0]), ps.pack_f([p1.f, p2.f])
    for _ in range(2):
        mg.vcycle(u, f)
    torch.cuda.synchronize()
    for q, p in enumerate((p1, p2)):
        ref = p.u0
        for _ in range(2):
            ref = oracle.vcycle(ref, p.f, p.eps, p.h, "line", 2, oracle.COLORED_GS, 1.0, 1, 1, 30, levels=2,
                                coarse_bc=63)
        got = ps.view_u(u, q).cpu().numpy()
        assert relerr(got[1:-1, 1:-1, 1:-1], ref[1:-1, 1:-1, 1:-1]) < TOL
    mg.close()
    ps.close()


@pytest.mark.parametrize("kind,arg,eps", [("line", 2, (1.0, 1.0, 100.0)), ("plane", 0, (1.0, 100.0, 100.0)),
                                          ("line", 0, (1.0, 1.0, 1.0))])
def test_vcycle_factor_grid_independent(kind, arg, eps):
    """V(1,1) with two-colour GS block smoothing, extrapolated coarse faces: the
    residual reduction per cycle stays small from 16^3 to 128^3 (the oracle's
    cycle, which every cycle here matches to 1e-12, shows the same); with line
    smoothers it is also independent of n.  Plane smoothing of the strong
    planes under full coarsening drifts slowly upwards with n (0.002, 0.03,
    0.07, 0.12 from 16^3 to 128^3 for eps (1,100,100)), still far below 0.3."""
    facs = []
    for n in (16, 32, 64, 128):
        p = make_patch(n, n, n, eps, 1.0 / n, seed=4, f="zero", u0="uniform")
        ps = bs.PatchSet([p.dims], [p.eps], [p.h])
        ps.set_bc([63])
        mg = bs.Multigrid(ps, kind, arg, "colored", 1.0, 1, 1, 20, 0, 63)
        u, f = ps.pack_u([p.u0]), ps.pack_f([p.f])
        n2 = torch.zeros(1, dtype=torch.float64, device="cuda")
        rs = []
        for _ in range(7):
            ps.residual(u, f, None, n2)
            rs.append(math.sqrt(float(n2.item())))
            mg.vcycle(u, f)
        facs.append((rs[6] / rs[3]) ** (1 / 3))
        mg.close()
        ps.close()
    log("vcycle factors %s %s" % (kind, facs))
    assert max(facs) < 0.3, facs
    if kind == "line":
        assert max(facs) - min(facs) < 0.08, facs


def test_vcycle_errors():
    p = small_patch(8, 8, 8, seed=1)
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    for args in [("line", 3, "colored", 1.0), ("line", 0, "colored", 2.0), ("bad", 0, "colored", 1.0)]:
        with pytest.raises((bs.BSError, KeyError)):
            bs.Multigrid(ps, *args)
    mg = bs.Multigrid(ps, "line", 0, "jacobi", 0.8)
    u, f = ps.pack_u([p.u0]), ps.pack_f([p.f])
    with pytest.raises(bs.BSError):   # Jacobi smoothing needs the work buffer
        mg.vcycle(u, f)
    ps.set_eps([(2.0, 1.0, 1.0)])
    with pytest.raises(bs.BSError):   # the fine set changed under the cycle
        mg.vcycle(u, f, ps.empty_u())
    mg.close()
    ps.close()
