"""Geometric cube blocks on the GPU (residual gather, FP64 matrix-core product
with the precomputed block inverses, update in the product's epilogue)
against the oracle's Cholesky block solves: max-norm relative error 1e-12.

Cases span several product tiles with ragged tails (more than 128 blocks of a
shape, blocks of more than 128 cells), ragged last blocks along every axis,
point, line and plane shaped blocks, odd cell counts (no paired loads),
patch sets whose patches share or do not share inverses, graph replay, eps
changes, and the block-size study's workload (64 patches of 64^3)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1208_1975_amd as bs
from conftest import relerr
from gpu_util import log, need_gpu
from workloads import c4_patchset, small_patch, uniform_patchset

pytestmark = pytest.mark.gpu
TOL = 1e-12
SCHEMES = (("jacobi", 0.8, oracle.JACOBI), ("colored", 1.0, oracle.COLORED_GS),
           ("chaotic", 1.0, oracle.COLORED_GS))


@pytest.fixture(scope="module", autouse=True)
def _setup():
    need_gpu()
    oracle.set_threads(0)
    yield


def run_single(p, block, scheme, omega, nsweeps, graphs=True):
    ps = bs.PatchSet([tuple(p.dims)], [p.eps], [p.h])
    ps.set_graphs(graphs)
    u = ps.pack_u([p.u0])
    f = ps.pack_f([p.f])
    w = ps.empty_u()
    ps.cube_prepare(block)
    ps.cube_relax(block, scheme, omega, nsweeps, u, f, w)
    torch.cuda.synchronize()
    return ps.view_u(u, 0).cpu().numpy().copy()


CASES = [((16, 16, 16), (4, 4, 4)), ((13, 10, 9), (2, 3, 4)), ((12, 11, 10), (8, 8, 8)), ((9, 7, 6), (1, 1, 1)),
         ((9, 7, 6), (9, 1, 1)), ((10, 9, 8), (10, 9, 1)), ((7, 9, 5), (3, 3, 3)), ((40, 36, 33), (4, 4, 4)),
         ((20, 6, 5), (64, 2, 2))]


@pytest.mark.parametrize("dims,block", CASES)
@pytest.mark.parametrize("scheme,omega,osch", SCHEMES)
def test_cubes_match_oracle(dims, block, scheme, omega, osch):
    p = small_patch(*dims, seed=sum(dims) + sum(block), eps=(1.0, 3.0, 7.0))
    for nsweeps in (1, 2):
        log("cubes %s block %s %s nsweeps=%d" % (dims, block, scheme, nsweeps))
        got = run_single(p, block, scheme, omega, nsweeps)
        ref = oracle.cube_sweeps(p.u0, p.f, p.eps, p.h, block, osch, omega, nsweeps)
        assert relerr(got, ref) < TOL, (dims, block, scheme, nsweeps)
        gm = ~np.pad(np.ones(p.f.shape, bool), 1, constant_values=False)
        assert np.array_equal(got[gm], p.u0[gm])


def test_big_blocks_several_product_tiles():
    """8^3 blocks on 64^3: 512 blocks x 512 cells, the product's 128 x 128
    tiles 4 x 4 with 32 steps along the block's cells."""
    p = small_patch(64, 64, 64, seed=9, eps=(1.0, 1.0, 100.0))
    log("cubes 64^3 block 8^3 jacobi")
    got = run_single(p, (8, 8, 8), "jacobi", 0.8, 1)
    ref = oracle.cube_sweeps(p.u0, p.f, p.eps, p.h, (8, 8, 8), oracle.JACOBI, 0.8, 1)
    assert relerr(got, ref) < TOL


def test_graph_replay_equals_eager():
    p = small_patch(24, 20, 18, seed=12)
    for scheme, omega, _ in SCHEMES:
        a = run_single(p, (4, 5, 3), scheme, omega, 3, graphs=True)
        b = run_single(p, (4, 5, 3), scheme, omega, 3, graphs=False)
        log("cubes graph vs eager %s" % scheme)
        assert np.array_equal(a, b), scheme
    # replay of one captured sequence several times, eager work between
    ps = bs.PatchSet([tuple(p.dims)], [p.eps], [p.h])
    u = ps.pack_u([p.u0])
    f = ps.pack_f([p.f])
    w = ps.empty_u()
    ps.cube_prepare((4, 4, 4))
    ref = p.u0
    for rep in range(3):
        ps.cube_relax((4, 4, 4), "jacobi", 0.8, 2, u, f, w)
        torch.cuda.synchronize()
        ref = oracle.cube_sweeps(ref, p.f, p.eps, p.h, (4, 4, 4), oracle.JACOBI, 0.8, 2)
        assert relerr(ps.view_u(u, 0).cpu().numpy(), ref) < TOL, rep


def test_patch_set_with_shared_and_distinct_inverses():
    """Uneven patches with their own eps, plus repeated patches that share
    inverses and tables; every patch equals the oracle on its own."""
    s = c4_patchset(npatch=10, seed=23, edges=(8, 12, 16, 20))
    dims = [tuple(d) for d in s.dims] + [tuple(s.dims[0])] * 3
    eps = [tuple(e) for e in s.eps] + [tuple(s.eps[0])] * 3
    hs = list(s.h) + [s.h[0]] * 3
    u0s = list(s.u0) + [s.u0[0] * (1 + 0.5 * k) for k in range(3)]
    fs = list(s.f) + [s.f[0] * (1 - 0.25 * k) for k in range(3)]
    ps = bs.PatchSet(dims, eps, hs)
    f = ps.pack_f(fs)
    for block in ((4, 4, 4), (3, 5, 2)):
        ps.cube_prepare(block)
        for scheme, omega, osch in SCHEMES:
            u = ps.pack_u(u0s)
            w = ps.empty_u()
            ps.cube_relax(block, scheme, omega, 2, u, f, w)
            torch.cuda.synchronize()
            log("cubes patch set block %s %s" % (block, scheme))
            for p in range(ps.npatch):
                ref = oracle.cube_sweeps(u0s[p], fs[p], eps[p], hs[p], block, osch, omega, 2)
                assert relerr(ps.view_u(u, p).cpu().numpy(), ref) < TOL, (block, scheme, p)


def test_set_eps_rebuilds_inverses():
    p = small_patch(12, 10, 9, seed=4)
    ps = bs.PatchSet([tuple(p.dims)], [p.eps], [p.h])
    ps.cube_prepare((4, 4, 4))
    new_eps = (2.0, 0.5, 30.0)
    ps.set_eps([new_eps])
    u = ps.pack_u([p.u0])
    f = ps.pack_f([p.f])
    ps.cube_relax((4, 4, 4), "colored", 1.0, 2, u, f)
    torch.cuda.synchronize()
    ref = oracle.cube_sweeps(p.u0, p.f, new_eps, p.h, (4, 4, 4), oracle.COLORED_GS, 1.0, 2)
    assert relerr(ps.view_u(u, 0).cpu().numpy(), ref) < TOL


def test_errors():
    p = small_patch(12, 10, 9, seed=4)
    ps = bs.PatchSet([tuple(p.dims)], [p.eps], [p.h])
    u = ps.pack_u([p.u0])
    f = ps.pack_f([p.f])
    with pytest.raises(bs.BSError, match="not prepared"):
        ps.cube_relax((4, 4, 4), "colored", 1.0, 1, u, f)
    ps.cube_prepare((4, 4, 4))
    with pytest.raises(bs.BSError, match="FP64"):
        ps.cube_relax((4, 4, 4), "colored", 1.0, 1, u, f, prec="fp32")
    with pytest.raises(bs.BSError, match="work"):
        ps.cube_relax((4, 4, 4), "jacobi", 0.8, 1, u, f)
    with pytest.raises(bs.BSError, match="512"):
        ps.cube_prepare((12, 10, 5))
    with pytest.raises(bs.BSError, match=">= 1"):
        ps.cube_prepare((0, 4, 4))
    ps.cube_prepare((12, 10, 4))   # 480 cells: allowed
    ps.cube_relax((12, 10, 4), "chaotic", 1.0, 0, u, f)   # zero sweeps: nothing enqueued


@pytest.mark.parametrize("block", [(8, 8, 8), (4, 4, 4)])
def test_block_size_study_workload(block):
    """64 patches of 64^3 (all sharing one inverse per shape), as timed by the
    benchmark: one Jacobi and one chaotic sweep; two patches checked whole
    against the oracle."""
    s = uniform_patchset()
    ps = bs.PatchSet([tuple(d) for d in s.dims], [tuple(e) for e in s.eps], list(s.h))
    f = ps.pack_f(s.f)
    ps.cube_prepare(block)
    for scheme, omega, osch in (("jacobi", 0.8, oracle.JACOBI), ("chaotic", 1.0, oracle.COLORED_GS)):
        u = ps.pack_u(s.u0)
        w = ps.empty_u()
        ps.cube_relax(block, scheme, omega, 1, u, f, w)
        torch.cuda.synchronize()
        for p in (0, 63):
            log("cubes 64 x 64^3 block %s %s patch %d" % (block, scheme, p))
            ref = oracle.cube_sweeps(s.u0[p], s.f[p], tuple(s.eps[p]), s.h[p], block, osch, omega, 1)
            assert relerr(ps.view_u(u, p).cpu().numpy(), ref) < TOL, (block, scheme, p)


def test_block_size_study_on_the_gpu():
    """The block-size study's workload (one 64^3 patch, eps = 1, f = 0, random
    initial guess): three sweeps improve monotonically with the block size for
    both schemes; two sizes equal the oracle; point blocks converge at the
    closed-form rates: damped Jacobi 1 - 1.6 sin^2(pi/130), two-colour GS
    cos^2(pi/65)."""
    import math
    from workloads import make_patch
    n = 64
    p = make_patch(n, n, n, (1.0, 1.0, 1.0), 1.0 / n, seed=8, f="zero", u0="uniform", ghosts="zero")
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    u0, f, w = ps.pack_u([p.u0]), ps.pack_f([p.f]), ps.empty_u()
    n2 = torch.zeros(1, dtype=torch.float64, device="cuda")

    def rnorm(u):
        ps.residual(u, f, None, n2)
        torch.cuda.synchronize()
        return math.sqrt(float(n2.item()))

    r0 = rnorm(u0)
    sizes = [(1, 1, 1), (2, 2, 2), (4, 2, 2), (4, 4, 2), (4, 4, 4), (8, 4, 4), (8, 8, 4), (8, 8, 8)]
    for scheme, omega, osch in (("jacobi", 0.8, oracle.JACOBI), ("chaotic", 1.0, oracle.COLORED_GS)):
        rel = []
        for b in sizes:
            ps.cube_prepare(b)
            u = u0.clone()
            ps.cube_relax(b, scheme, omega, 3, u, f, w)
            rel.append(rnorm(u) / r0)
            if b in ((4, 2, 2), (8, 8, 8)) and scheme == "jacobi":
                log("study parity %s %s" % (b, scheme))
                ref = oracle.cube_sweeps(p.u0, p.f, p.eps, p.h, b, osch, omega, 3)
                assert relerr(ps.view_u(u, 0).cpu().numpy(), ref) < TOL, b
        log("study %s %s" % (scheme, ["%.4f" % v for v in rel]))
        assert all(a > b for a, b in zip(rel, rel[1:])), (scheme, rel)
    u = u0.clone()
    ps.cube_relax((1, 1, 1), "jacobi", 0.8, 4000, u, f, w)
    ra = rnorm(u)
    ps.cube_relax((1, 1, 1), "jacobi", 0.8, 4000, u, f, w)
    factor = (rnorm(u) / ra) ** (1.0 / 4000)
    rho = 1.0 - 1.6 * math.sin(math.pi / (2 * (n + 1))) ** 2
    log("point Jacobi factor %.8f closed form %.8f" % (factor, rho))
    assert abs(factor - rho) < 1e-4
    # two-colour point GS (omega 1): rho_J^2 with rho_J = cos(pi/(n+1))
    u = u0.clone()
    ps.cube_relax((1, 1, 1), "chaotic", 1.0, 2000, u, f)
    ra = rnorm(u)
    ps.cube_relax((1, 1, 1), "chaotic", 1.0, 2000, u, f)
    factor = (rnorm(u) / ra) ** (1.0 / 2000)
    rho = math.cos(math.pi / (n + 1)) ** 2
    log("point two-colour GS factor %.8f closed form %.8f" % (factor, rho))
    assert abs(factor - rho) < 1e-4


def test_many_classes_one_launch_per_operand_size():
    """40 uneven patches, each its own class (own dims and eps): blocks of up to
    64 cells of all of them run in one fused launch per operand size; with
    8 x 8 x 2 blocks the same sweep also runs the two-kernel form for the
    128-cell blocks.  Every patch equals the oracle."""
    s = c4_patchset(npatch=40, seed=29, edges=(6, 9, 12, 16, 20))
    dims = [tuple(d) for d in s.dims]
    eps = [tuple(e) for e in s.eps]
    ps = bs.PatchSet(dims, eps, list(s.h))
    f = ps.pack_f(s.f)
    for block in ((4, 4, 4), (2, 3, 2), (8, 8, 2)):
        ps.cube_prepare(block)
        for scheme, omega, osch in SCHEMES:
            u = ps.pack_u(s.u0)
            w = ps.empty_u()
            ps.cube_relax(block, scheme, omega, 3, u, f, w)
            torch.cuda.synchronize()
            log("cubes 40 classes block %s %s" % (block, scheme))
            for p in range(ps.npatch):
                ref = oracle.cube_sweeps(s.u0[p], s.f[p], eps[p], s.h[p], block, osch, omega, 3)
                assert relerr(ps.view_u(u, p).cpu().numpy(), ref) < TOL, (block, scheme, p)


def test_set_eps_after_a_captured_sequence():
    """A captured two-sweep sequence, then an eps change (new inverses and
    tables), then the same call: the replay must use the new inverses."""
    p = small_patch(16, 12, 10, seed=14)
    ps = bs.PatchSet([tuple(p.dims)], [p.eps], [p.h])
    u = ps.pack_u([p.u0])
    f = ps.pack_f([p.f])
    w = ps.empty_u()
    for block in ((4, 4, 4), (8, 4, 4)):
        ps.cube_prepare(block)
    for block in ((4, 4, 4), (8, 4, 4)):
        ps.cube_relax(block, "jacobi", 0.8, 2, u, f, w)      # captured
    new_eps = (5.0, 0.25, 2.0)
    ps.set_eps([new_eps])
    for block in ((4, 4, 4), (8, 4, 4)):
        ps.pack_u([p.u0], out=u)
        ps.cube_relax(block, "jacobi", 0.8, 2, u, f, w)
        torch.cuda.synchronize()
        ref = oracle.cube_sweeps(p.u0, p.f, new_eps, p.h, block, oracle.JACOBI, 0.8, 2)
        log("cubes eps change after capture %s" % (block,))
        assert relerr(ps.view_u(u, 0).cpu().numpy(), ref) < TOL, block


@pytest.mark.parametrize("block", [(8, 4, 4), (8, 8, 4), (7, 6, 5)])
def test_fused_large_blocks_equal_two_kernel_form_on_many_workgroups(block):
    """Blocks of 65-256 cells run fused (residuals of 32 blocks in LDS, the
    product, the update in one kernel).  On 32 patches of 64^3 thousands of
    workgroups run at different times, so an in-place pass that wrote cells
    of a block another workgroup still reads would show here (small patches
    run every workgroup at once and hide it): the fused sweeps must equal the
    residual-matrix + product form to rounding, in place and into a second
    vector."""
    import ctypes
    L = bs.lib()
    L.bsi_set_cube_fused_max.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.bsi_set_cube_fused_max.restype = ctypes.c_int
    s = uniform_patchset(npatch=32)
    ps = bs.PatchSet([tuple(d) for d in s.dims], [tuple(e) for e in s.eps], list(s.h))
    u0, f, w = ps.pack_u(s.u0), ps.pack_f(s.f), ps.empty_u()
    try:
        for scheme, omega in (("jacobi", 0.8), ("chaotic", 1.0)):
            res = {}
            for fmax in (64, 256):
                assert L.bsi_set_cube_fused_max(ps.handle, fmax) == 0
                ps.cube_prepare(block)
                u = u0.clone()
                ps.cube_relax(block, scheme, omega, 2, u, f, w)
                torch.cuda.synchronize()
                res[fmax] = u
            d = float((res[64] - res[256]).abs().max() / res[64].abs().max())
            log("cube %s %s: fused vs two kernels %.3e" % (block, scheme, d))
            assert d < 1e-13, (block, scheme, d)
    finally:
        L.bsi_set_cube_fused_max(ps.handle, 256)
        ps.close()
