"""Batched patch sets (uneven AMR patches relaxed by the same launches),
graph capture and replay, the per-patch baseline and the autotuner."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1208_1975_amd as bs
from conftest import relerr
from gpu_util import log, need_gpu
from workloads import c4_patchset

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _setup():
    need_gpu()
    oracle.set_threads(0)
    yield


def small_set(n=40, seed=14):
    s = c4_patchset(npatch=n, seed=seed)
    ps = bs.PatchSet([tuple(d) for d in s.dims], [tuple(e) for e in s.eps], list(s.h))
    return s, ps


def test_graph_replays_match_eager():
    s, ps = small_set()
    f = ps.pack_f(s.f)
    for axis, scheme, om in ((0, "jacobi", 0.8), (2, "colored", 1.0), (1, "jacobi", 1.0)):
        ps.set_graphs(False)
        ue = ps.pack_u(s.u0)
        we = ps.empty_u()
        ps.line_relax(axis, scheme, om, 3, ue, f, we)
        torch.cuda.synchronize()
        ref = ue.clone()
        ps.set_graphs(True)
        ug = ps.pack_u(s.u0)
        wg = ps.empty_u()
        for rep in range(4):
            ug.copy_(ps.pack_u(s.u0))            # eager work between replays
            ps.residual(ug, f, None, torch.zeros(ps.npatch, dtype=torch.float64, device="cuda"))
            torch.cuda.synchronize()
            ps.line_relax(axis, scheme, om, 3, ug, f, wg)     # rep 0 captures, later reps replay
            torch.cuda.synchronize()
            log("graph axis %d %s replay %d" % (axis, scheme, rep))
            assert torch.equal(ug, ref)


def test_per_patch_launches_equal_batched():
    s, ps = small_set(n=25, seed=3)
    f = ps.pack_f(s.f)
    for axis, scheme, om in ((0, "jacobi", 0.8), (2, "colored", 1.0)):
        u1 = ps.pack_u(s.u0)
        u2 = ps.pack_u(s.u0)
        w = ps.empty_u()
        ps.line_relax(axis, scheme, om, 2, u1, f, w)
        ps.line_relax_per_patch(axis, scheme, om, 2, u2, f, w)
        torch.cuda.synchronize()
        assert torch.equal(u1, u2)


def test_autotuned_configuration_is_correct():
    s, ps = small_set(n=30, seed=5)
    f = ps.pack_f(s.f)
    u = ps.pack_u(s.u0)
    for axis in (0, 2):
        ps.autotune_line(axis, "jacobi", u, f)
        cfg = ps.line_config(axis, "jacobi")
        log("axis %d tuned config %s" % (axis, cfg))
        assert cfg["tuned"] == 1
        assert torch.equal(u, ps.pack_u(s.u0))      # tuning leaves the caller's u alone
        w = ps.empty_u()
        uu = ps.pack_u(s.u0)
        ps.line_relax(axis, "jacobi", 0.8, 3, uu, f, w)
        torch.cuda.synchronize()
        for p in range(ps.npatch):
            ref = oracle.line_sweeps(s.u0[p], s.f[p], tuple(s.eps[p]), s.h[p], axis, oracle.JACOBI, 0.8, 3)
            assert relerr(ps.view_u(uu, p).cpu().numpy(), ref) < TOL


def test_persistent_grid_matches_one_workgroup_per_tile():
    s, ps = small_set(n=20, seed=8)
    f = ps.pack_f(s.f)
    outs = []
    for grid in (0, 7, 300):
        ps.set_line_config(0, "jacobi", 1, tile=64, grid=grid)
        u = ps.pack_u(s.u0)
        w = ps.empty_u()
        ps.line_relax(0, "jacobi", 0.8, 2, u, f, w)
        torch.cuda.synchronize()
        outs.append(u)
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


@pytest.mark.parametrize("axis", [1, 2])
def test_persistent_grid_strided_lines(axis):
    """y/z lines: a persistent grid (each workgroup drains several tiles and
    fetches the next tile's first loads early) gives the bitwise result of one
    workgroup per tile for the deterministic schemes, which equals the oracle."""
    s, ps = small_set(n=20, seed=9)
    f = ps.pack_f(s.f)
    for scheme, om, osch in (("jacobi", 0.8, oracle.JACOBI), ("colored", 1.0, oracle.COLORED_GS)):
        outs = []
        for grid in (0, 5, 300):
            ps.set_line_config(axis, scheme, 16, tile=64, grid=grid)
            u = ps.pack_u(s.u0)
            w = ps.empty_u()
            ps.line_relax(axis, scheme, om, 2, u, f, w)
            torch.cuda.synchronize()
            outs.append(u)
        assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2]), (axis, scheme)
        for p in range(ps.npatch):
            ref = oracle.line_sweeps(s.u0[p], s.f[p], tuple(s.eps[p]), s.h[p], axis, osch, om, 2)
            assert relerr(ps.view_u(outs[2], p).cpu().numpy(), ref) < TOL, (axis, scheme, p)


@pytest.mark.timeout(900)
def test_c4_full_set_chaotic_x_lines():
    """3000 uneven patches, x-line chaotic GS, 20 sweeps (four graph launches of
    5 sweeps): at sweeps 5, 10, 15 and 20, every sampled patch's residual within
    1.15x the oracle's two-colour GS from the same start."""
    s = c4_patchset()
    log("C4: %d patches, %d cells" % (s.npatch, s.cells()))
    ps = bs.PatchSet([tuple(d) for d in s.dims], [tuple(e) for e in s.eps], list(s.h))
    u = ps.pack_u(s.u0)
    f = ps.pack_f(s.f)
    n0 = torch.zeros(ps.npatch, dtype=torch.float64, device="cuda")
    ps.residual(u, f, None, n0)
    norms = []
    for blk in range(4):
        ps.line_relax(0, "chaotic", 1.0, 5, u, f)
        n1 = torch.zeros(ps.npatch, dtype=torch.float64, device="cuda")
        ps.residual(u, f, None, n1)
        norms.append(n1)
    torch.cuda.synchronize()
    r0 = n0.sqrt().cpu().numpy()
    rk = [n.sqrt().cpu().numpy() for n in norms]
    rng = np.random.default_rng(0)
    worst = [0.0] * 4
    for p in rng.choice(ps.npatch, 24, replace=False):
        ref = s.u0[p]
        for blk in range(4):
            ref = oracle.line_sweeps(ref, s.f[p], tuple(s.eps[p]), s.h[p], 0, oracle.COLORED_GS, 1.0, 5)
            rr = math.sqrt(oracle.residual(ref, s.f[p], tuple(s.eps[p]), s.h[p])[1])
            ratio = rk[blk][p] / rr
            worst[blk] = max(worst[blk], ratio)
            assert ratio <= 1.15, (p, 5 * (blk + 1), ratio)
    log("C4 worst sampled chaotic/two-colour residual ratio at sweeps 5/10/15/20: %s"
        % " ".join("%.4f" % w for w in worst))
