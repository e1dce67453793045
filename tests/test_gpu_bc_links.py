"""GPU parity of extrapolated-Dirichlet faces and of the ghost exchange
between face-adjacent patches, against the oracle.

Extrapolated faces (section 1.1: boundary conditions are extrapolated into
the ghost layer): the residual and every line sweep (Jacobi, two-colour GS,
and chaotic GS, which such patch sets dispatch colour-major) match the oracle,
which folds ghost = -interior into the operator, to 1e-12 on the interior;
the library leaves the negated adjacent interior values in the ghosts of those
faces and every other ghost bit-unchanged.

Ghost exchange (section 2: ghosts are updated Jacobi-fashion after every
smoothing step): line, plane and cube sweeps of a patch set with links match
the oracle's patch-set sweeps (one sweep per patch from its own ghosts, then
the exchange) to 1e-12 on every array, ghosts included; one exchange call
copies exactly."""
import numpy as np
import pytest
import torch

import oracle
import paper_1208_1975_amd as bs
from conftest import relerr
from gpu_util import log, need_gpu
from workloads import small_patch, split_patch

pytestmark = pytest.mark.gpu

TOL = 1e-12
OSCH = {"jacobi": oracle.JACOBI, "colored": oracle.COLORED_GS, "chaotic": oracle.COLORED_GS}


@pytest.fixture(scope="module", autouse=True)
def _setup():
    need_gpu()
    oracle.set_threads(0)
    yield


def _ghost_faces(nx, ny, nz):
    """(axis, side) -> index expression of that face's ghost cells (face only)."""
    I, J, K = slice(1, nx + 1), slice(1, ny + 1), slice(1, nz + 1)
    return {
        (0, 0): ((K, J, 0), (K, J, 1)), (0, 1): ((K, J, nx + 1), (K, J, nx)),
        (1, 0): ((K, 0, I), (K, 1, I)), (1, 1): ((K, ny + 1, I), (K, ny, I)),
        (2, 0): ((0, J, I), (1, J, I)), (2, 1): ((nz + 1, J, I), (nz, J, I)),
    }


def _check_ghosts(got, u0, bc):
    nz, ny, nx = (s - 2 for s in got.shape)
    for (axis, side), (g, adj) in _ghost_faces(nx, ny, nz).items():
        if (bc >> (2 * axis + side)) & 1:
            assert np.array_equal(got[g], -got[adj]), "extrapolated ghosts of face (%d, %d)" % (axis, side)
        else:
            assert np.array_equal(got[g], u0[g]), "ghosts of face (%d, %d) changed" % (axis, side)


def _single(p, bc):
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    ps.set_bc([bc])
    return ps, ps.pack_u([p.u0]), ps.pack_f([p.f]), ps.empty_u()


@pytest.mark.parametrize("dims", [(5, 4, 3), (1, 3, 2), (33, 17, 9), (64, 8, 70), (2, 1, 1)])
@pytest.mark.parametrize("bc", [63, 1 | 8 | 32, 2 | 4 | 16, 12, 48])
def test_residual_bc(dims, bc):
    p = small_patch(*dims, seed=5, eps=(1.0, 3.0, 7.0))
    log("residual bc=%d %s" % (bc, dims))
    ps, u, f, _ = _single(p, bc)
    r = ps.empty_f()
    n2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    ps.residual(u, f, r, n2)
    torch.cuda.synchronize()
    rr, nn2 = oracle.residual(p.u0, p.f, p.eps, p.h, bc=bc)
    assert relerr(ps.view_f(r, 0).cpu().numpy(), rr) < TOL
    assert float(n2.item()) == pytest.approx(nn2, rel=TOL)
    ps.close()


LINE_SHAPES = [(5, 4, 3), (7, 6, 5), (1, 1, 1), (2, 3, 1), (1, 5, 2), (33, 17, 9), (64, 8, 70), (130, 3, 67),
               (20, 65, 3)]


@pytest.mark.parametrize("dims", LINE_SHAPES)
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("bc", [63, 3, 12, 48, 1 | 8 | 16])
def test_line_bc_parity(dims, axis, bc):
    p = small_patch(*dims, seed=41 + axis, eps=(1.0, 3.0, 7.0))
    for scheme in ("jacobi", "colored", "chaotic"):
        omega = 0.8 if scheme == "jacobi" else 1.0
        for nsweeps in (1, 2, 3):
            log("line bc=%d %s axis %d %s %d" % (bc, dims, axis, scheme, nsweeps))
            ps, u, f, w = _single(p, bc)
            ps.line_relax(axis, scheme, omega, nsweeps, u, f, w)
            torch.cuda.synchronize()
            got = ps.view_u(u, 0).cpu().numpy()
            ref = oracle.line_sweeps(p.u0, p.f, p.eps, p.h, axis, OSCH[scheme], omega, nsweeps, bc=bc)
            err = relerr(got[1:-1, 1:-1, 1:-1], ref[1:-1, 1:-1, 1:-1])
            assert err < TOL, (scheme, nsweeps, err)
            _check_ghosts(got, p.u0, bc)
            ps.close()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_line_bc_large_and_fp32(axis):
    """A patch big enough for chunked lines and the one-launch chaotic order on
    line-axis-only faces; FP32 line solves stay within the FP32 bound."""
    dims = (96, 80, 72)
    bc_line = 3 << (2 * axis)
    p = small_patch(*dims, seed=7, eps=(1.0, 2.0, 30.0))
    for bc in (bc_line, 63):
        ps, u, f, w = _single(p, bc)
        log("line bc=%d large axis %d" % (bc, axis))
        ps.line_relax(axis, "jacobi", 0.8, 4, u, f, w)
        ref = oracle.line_sweeps(p.u0, p.f, p.eps, p.h, axis, oracle.JACOBI, 0.8, 4, bc=bc)
        torch.cuda.synchronize()
        assert relerr(ps.view_u(u, 0).cpu().numpy()[1:-1, 1:-1, 1:-1], ref[1:-1, 1:-1, 1:-1]) < TOL
        u2 = ps.pack_u([p.u0])
        ps.line_relax(axis, "jacobi", 0.8, 4, u2, f, w, prec="fp32")
        torch.cuda.synchronize()
        assert relerr(ps.view_u(u2, 0).cpu().numpy()[1:-1, 1:-1, 1:-1], ref[1:-1, 1:-1, 1:-1]) < 4 * 1e-6
        ps.close()


@pytest.mark.parametrize("axis", [1, 2])
def test_jacobi_direct_and_update_forms(axis):
    """Jacobi on y/z lines in the direct form M^{-1}(omega b + (1 - omega) M u)
    (the FP64 default) and in the update form u + omega M^{-1} r: both match
    the oracle to 1e-12 for every chunk count, lines of 129..256 cells (four
    chunks by default) included, with Dirichlet, extrapolated line-end and
    all-extrapolated faces, omega below, at and above 1."""
    dims = (40, 150, 24) if axis == 1 else (37, 21, 201)
    p = small_patch(*dims, seed=13 + axis, eps=(1.0, 3.0, 40.0))
    ps0, _, _, _ = _single(p, 0)
    assert ps0.line_config(axis, "jacobi")["chunks"] == 4
    ps0.close()
    for bc in (0, 3 << (2 * axis), 63):
        for omega in (0.8, 1.0, 1.3):
            ref = oracle.line_sweeps(p.u0, p.f, p.eps, p.h, axis, oracle.JACOBI, omega, 3, bc=bc)
            for direct in (True, False):
                for chunks in (0, 4, 8, 16):
                    log("jacobi forms axis %d bc=%d omega %.1f direct=%s chunks=%d" % (axis, bc, omega, direct, chunks))
                    ps, u, f, w = _single(p, bc)
                    ps.set_line_direct(direct)
                    if chunks:
                        ps.set_line_config(axis, "jacobi", chunks, 64)
                    ps.line_relax(axis, "jacobi", omega, 3, u, f, w)
                    torch.cuda.synchronize()
                    got = ps.view_u(u, 0).cpu().numpy()
                    err = relerr(got[1:-1, 1:-1, 1:-1], ref[1:-1, 1:-1, 1:-1])
                    assert err < TOL, (bc, omega, direct, chunks, err)
                    _check_ghosts(got, p.u0, bc)
                    ps.close()


def test_line_bc_fixed_point():
    """The exact discrete solution with extrapolated faces is a fixed point."""
    p = small_patch(24, 20, 18, seed=9, eps=(1.0, 1.0, 50.0))
    bc = 63
    r, _ = oracle.residual(p.u0, np.zeros_like(p.f), p.eps, p.h, bc=bc)
    f = np.ascontiguousarray(-r / (p.h * p.h))
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    ps.set_bc([bc])
    for axis in (0, 1, 2):
        for scheme in ("jacobi", "colored", "chaotic"):
            u = ps.pack_u([p.u0])
            ps.line_relax(axis, scheme, 0.8 if scheme == "jacobi" else 1.0, 3, u, ps.pack_f([f]), ps.empty_u())
            torch.cuda.synchronize()
            got = ps.view_u(u, 0).cpu().numpy()
            assert relerr(got[1:-1, 1:-1, 1:-1], p.u0[1:-1, 1:-1, 1:-1]) < 1e-13
    ps.close()


def test_line_bc_graph_replays_equal_eager():
    p = small_patch(40, 36, 33, seed=11, eps=(1.0, 4.0, 9.0))
    ps, u, f, w = _single(p, 63)
    ps.set_graphs(False)
    ps.line_relax(2, "colored", 1.0, 3, u, f, w)
    torch.cuda.synchronize()
    ref = ps.view_u(u, 0).cpu().numpy().copy()
    ps.set_graphs(True)
    for _ in range(3):
        u2 = ps.pack_u([p.u0])
        ps.line_relax(2, "colored", 1.0, 3, u2, f, w)
        torch.cuda.synchronize()
        assert np.array_equal(ps.view_u(u2, 0).cpu().numpy(), ref)
    ps.close()


# --- ghost exchange between face-adjacent patches ------------------------------

def _linked(ls):
    ps = bs.PatchSet(ls.dims, ls.eps, ls.h)
    ps.set_links(ls.links)
    return ps, ps.pack_u(ls.u0), ps.pack_f(ls.f), ps.empty_u()


def _split(seed=3, dims=(24, 20, 18), cuts=([11], [9], [8]), eps=(1.0, 3.0, 7.0)):
    p = small_patch(*dims, seed=seed, eps=eps)
    return p, split_patch(p, cuts)


def test_exchange_call_copies_exactly():
    _, ls = _split()
    ps, u, _, _ = _linked(ls)
    ps.exchange_ghosts(u)
    torch.cuda.synchronize()
    ref = oracle.exchange_ghosts(ls.u0, ls.links)
    for q in range(ls.npatch):
        assert np.array_equal(ps.view_u(u, q).cpu().numpy(), ref[q])
    ps.close()


@pytest.mark.parametrize("kind,arg", [("line", 0), ("line", 1), ("line", 2), ("plane", 0), ("plane", 2),
                                      ("cube", (4, 4, 4)), ("cube", (3, 5, 2))])
@pytest.mark.parametrize("scheme", ["jacobi", "colored"])
def test_patchset_sweeps_with_exchange(kind, arg, scheme):
    _, ls = _split()
    # per-patch eps and uneven ghosts: the exchange, not the symmetry, must make it agree
    rng = np.random.default_rng(17)
    ls.eps = [tuple(float(v) for v in 10 ** rng.uniform(0, 1, 3)) for _ in range(ls.npatch)]
    omega = 0.8 if scheme == "jacobi" else 1.0
    for nsweeps in (1, 2, 3):
        log("exchange %s %s %s %d" % (kind, arg, scheme, nsweeps))
        ps, u, f, w = _linked(ls)
        if kind == "line":
            ps.line_relax(arg, scheme, omega, nsweeps, u, f, w)
        elif kind == "plane":
            ps.plane_relax(arg, scheme, omega, nsweeps, u, f, w)
        else:
            ps.cube_prepare(arg)
            ps.cube_relax(arg, scheme, omega, nsweeps, u, f, w)
        torch.cuda.synchronize()
        ref = oracle.patchset_sweeps(ls.u0, ls.f, ls.eps, ls.h, ls.links, kind, arg, OSCH[scheme], omega, nsweeps)
        for q in range(ls.npatch):
            got = ps.view_u(u, q).cpu().numpy()
            assert relerr(got, ref[q]) < TOL, (q, relerr(got, ref[q]))
        ps.close()


def test_jacobi_split_along_free_axes_equals_whole_patch():
    """z-line Jacobi with the patch cut along x and y (never along a line): the
    patch set with exchange reproduces the whole patch's sweeps on the GPU."""
    p, ls = _split(dims=(40, 30, 50), cuts=([13, 27], [16], []))
    ps, u, f, w = _linked(ls)
    ps.line_relax(2, "jacobi", 0.8, 5, u, f, w)
    whole = bs.PatchSet([p.dims], [p.eps], [p.h])
    uw = whole.pack_u([p.u0])
    whole.line_relax(2, "jacobi", 0.8, 5, uw, whole.pack_f([p.f]), whole.empty_u())
    torch.cuda.synchronize()
    W = whole.view_u(uw, 0).cpu().numpy()
    for q, (x0, y0, z0) in enumerate(ls.offsets):
        nx, ny, nz = ls.dims[q]
        got = ps.view_u(u, q).cpu().numpy()[1:-1, 1:-1, 1:-1]
        assert relerr(got, W[z0 + 1:z0 + nz + 1, y0 + 1:y0 + ny + 1, x0 + 1:x0 + nx + 1]) < TOL
    ps.close()
    whole.close()


def test_links_and_bc_together():
    """Extrapolated outer faces with exchanged inner faces: z-line two-colour GS
    against the oracle's patch-set sweeps (each patch with its own face mask)."""
    p, ls = _split(dims=(20, 16, 24), cuts=([10], [], [12]))
    ps = bs.PatchSet(ls.dims, ls.eps, ls.h)
    masks = []
    for q, (x0, y0, z0) in enumerate(ls.offsets):
        nx, ny, nz = ls.dims[q]
        m = 4 | 8   # both y faces are outer faces
        m |= 1 if x0 == 0 else 2
        m |= 16 if z0 == 0 else 32
        masks.append(m)
    ps.set_bc(masks)
    ps.set_links(ls.links)
    u, f = ps.pack_u(ls.u0), ps.pack_f(ls.f)
    ps.line_relax(2, "colored", 1.0, 3, u, f)
    torch.cuda.synchronize()
    out = [np.array(a, copy=True) for a in ls.u0]
    for _ in range(3):
        out = [oracle.line_sweeps(out[q], ls.f[q], ls.eps[q], ls.h[q], 2, oracle.COLORED_GS, 1.0, 1, bc=masks[q])
               for q in range(ls.npatch)]
        out = oracle.exchange_ghosts(out, ls.links)
    for q in range(ls.npatch):
        got = ps.view_u(u, q).cpu().numpy()
        assert relerr(got[1:-1, 1:-1, 1:-1], out[q][1:-1, 1:-1, 1:-1]) < TOL
    ps.close()


def test_bc_and_links_errors():
    _, ls = _split()
    ps = bs.PatchSet(ls.dims, ls.eps, ls.h)
    bad = [[(0, 3, 1)], [(0, 0, 0)], [(0, 0, ls.npatch)], [(0, 1, 1)],   # axis, self, range, extents differ
           [ls.links[0], ls.links[0]]]                                 # a face linked twice
    for links in bad:
        with pytest.raises(bs.BSError) as ei:
            ps.set_links(links)
        assert ei.value.status == bs.BS_ERR_INVALID
    with pytest.raises(bs.BSError):
        ps.set_bc([64] + [0] * (ls.npatch - 1))
    ps.set_links(ls.links)
    a, axis, b = ls.links[0]
    with pytest.raises(bs.BSError):   # a linked face cannot be extrapolated
        ps.set_bc([(2 << (2 * axis)) if q == a else 0 for q in range(ls.npatch)])
    ps.set_bc([0] * ls.npatch)
    ps.set_links([])
    ps.set_bc([63] * ls.npatch)
    u, f, w = ps.pack_u(ls.u0), ps.pack_f(ls.f), ps.empty_u()
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(bs.BSError) as ei:
        bs.bs_relax_backward(ps.handle, 2, 0.8, 2, 1, u, f, u, None, None, None, ws)
    assert ei.value.status == bs.BS_ERR_UNSUPPORTED
    ps.close()


PLANE_SHAPES = [(5, 4, 3), (1, 3, 2), (2, 1, 1), (33, 17, 9), (20, 31, 18), (64, 8, 70)]


@pytest.mark.parametrize("dims", PLANE_SHAPES)
@pytest.mark.parametrize("normal", [0, 1, 2])
@pytest.mark.parametrize("bc", [63, 3, 12, 48, 1 | 8 | 32, 2 | 4 | 16])
def test_plane_bc_parity(dims, normal, bc):
    """Plane blocks with extrapolated faces: DST-II bases (both faces of an
    in-plane axis), one-sided sine bases (one face), shifted eigenvalue grids
    for the planes next to an extrapolated face normal to them."""
    p = small_patch(*dims, seed=51 + normal, eps=(1.0, 3.0, 7.0))
    for scheme in ("jacobi", "colored"):
        omega = 0.8 if scheme == "jacobi" else 1.0
        for nsweeps in (1, 2):
            log("plane bc=%d %s normal %d %s %d" % (bc, dims, normal, scheme, nsweeps))
            ps, u, f, w = _single(p, bc)
            ps.plane_relax(normal, scheme, omega, nsweeps, u, f, w)
            torch.cuda.synchronize()
            got = ps.view_u(u, 0).cpu().numpy()
            ref = oracle.plane_sweeps(p.u0, p.f, p.eps, p.h, normal, OSCH[scheme], omega, nsweeps, bc=bc)
            err = relerr(got[1:-1, 1:-1, 1:-1], ref[1:-1, 1:-1, 1:-1])
            assert err < TOL, (scheme, nsweeps, err)
            ps.close()


def test_plane_bc_fixed_point_and_mixed_refused():
    p = small_patch(24, 20, 18, seed=9, eps=(1.0, 50.0, 50.0))
    r, _ = oracle.residual(p.u0, np.zeros_like(p.f), p.eps, p.h, bc=63)
    f = np.ascontiguousarray(-r / (p.h * p.h))
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    ps.set_bc([63])
    for normal in (0, 1, 2):
        u = ps.pack_u([p.u0])
        ps.plane_relax(normal, "colored", 1.0, 2, u, ps.pack_f([f]), ps.empty_u())
        torch.cuda.synchronize()
        got = ps.view_u(u, 0).cpu().numpy()
        assert relerr(got[1:-1, 1:-1, 1:-1], p.u0[1:-1, 1:-1, 1:-1]) < 1e-13
    with pytest.raises(bs.BSError) as ei:
        ps.plane_relax(2, "jacobi", 1.0, 1, ps.pack_u([p.u0]), ps.pack_f([f]), ps.empty_u(), prec="fp32")
    assert ei.value.status == bs.BS_ERR_UNSUPPORTED
    ps.close()


CUBE_CASES = [((9, 7, 6), (4, 4, 4)), ((8, 8, 8), (2, 2, 2)), ((10, 6, 7), (3, 5, 2)), ((12, 12, 10), (8, 8, 4)),
              ((5, 9, 11), (8, 8, 8)), ((16, 4, 9), (4, 2, 2))]


@pytest.mark.parametrize("dims,block", CUBE_CASES)
@pytest.mark.parametrize("bc", [63, 3, 1 | 8 | 32, 2 | 4 | 16, 48])
def test_cube_bc_parity(dims, block, bc):
    """Cube blocks with extrapolated faces: the blocks touching such a face get
    the inverse of their raised block matrix (one-sided or DST-II factors
    along the touching axes); fused (<= 64 cells) and two-kernel forms."""
    p = small_patch(*dims, seed=61, eps=(1.0, 3.0, 7.0))
    for scheme in ("jacobi", "colored", "chaotic"):
        omega = 0.8 if scheme == "jacobi" else 1.0
        for nsweeps in (1, 2):
            log("cube bc=%d %s %s %s %d" % (bc, dims, block, scheme, nsweeps))
            ps, u, f, w = _single(p, bc)
            ps.cube_prepare(block)
            ps.cube_relax(block, scheme, omega, nsweeps, u, f, w)
            torch.cuda.synchronize()
            got = ps.view_u(u, 0).cpu().numpy()
            ref = oracle.cube_sweeps(p.u0, p.f, p.eps, p.h, block, OSCH[scheme], omega, nsweeps, bc=bc)
            err = relerr(got[1:-1, 1:-1, 1:-1], ref[1:-1, 1:-1, 1:-1])
            assert err < TOL, (scheme, nsweeps, err)
            _check_ghosts(got, p.u0, bc)
            ps.close()
