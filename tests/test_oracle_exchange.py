"""Pins for the oracle's ghost exchange between adjacent patches (section 2:
ghosts between patches are updated Jacobi-fashion after each full smoothing
step).  The exchange itself is checked against the unsplit array it cuts; the
smoothing of a split patch against the unsplit patch: block Jacobi whose
blocks stay whole under the split is the same iteration (bitwise), and the
exact discrete solution of the whole box is a fixed point of every scheme."""
import numpy as np
import pytest

import oracle
from conftest import relerr
from workloads import ghost_mask, small_patch, split_patch

EPS = (1.0, 3.0, 7.0)


@pytest.fixture(scope="module", autouse=True)
def _threads():
    oracle.set_threads(4)
    yield


def _face_mask(nx, ny, nz):
    """Interior cells and face ghosts (edge and corner ghosts are never read)."""
    m = np.zeros((nz + 2, ny + 2, nx + 2), bool)
    m[1:-1, 1:-1, :] = True
    m[1:-1, :, 1:-1] = True
    m[:, 1:-1, 1:-1] = True
    return m


def _assemble(s, whole_shape):
    """Interiors of the sub-patches placed back into one array."""
    nz, ny, nx = whole_shape
    out = np.zeros((nz, ny, nx))
    for u, (x0, y0, z0), (mx, my, mz) in zip(s.u0, s.offsets, s.dims):
        out[z0:z0 + mz, y0:y0 + my, x0:x0 + mx] = u[1:-1, 1:-1, 1:-1]
    return out


def test_exchange_restores_neighbour_values():
    p = small_patch(11, 9, 8, seed=5, eps=EPS)
    s = split_patch(p, ([4, 7], [5], [3]))
    assert len(s.links) == (2 * 2 * 2) + (3 * 1 * 2) + (3 * 2 * 1)
    # scramble every ghost layer, then exchange: face ghosts between patches
    # must come back to the whole array's values; outer ghosts stay scrambled
    rng = np.random.default_rng(1)
    junk = []
    for u, d in zip(s.u0, s.dims):
        v = u.copy()
        gm = ghost_mask(*d)
        v[gm] = rng.uniform(5, 6, int(gm.sum()))
        junk.append(v)
    ex = oracle.exchange_ghosts(junk, s.links)
    for q, (u, v, (x0, y0, z0), (mx, my, mz)) in enumerate(zip(ex, junk, s.offsets, s.dims)):
        ref = p.u0[z0:z0 + mz + 2, y0:y0 + my + 2, x0:x0 + mx + 2]
        fm = _face_mask(mx, my, mz)
        inner = np.zeros_like(fm)
        # face ghost positions shared with another patch
        for axis, lo, hi in ((0, x0 == 0, x0 + mx == 11), (1, y0 == 0, y0 + my == 9), (2, z0 == 0, z0 + mz == 8)):
            sl_lo = [slice(1, -1)] * 3
            sl_hi = [slice(1, -1)] * 3
            sl_lo[2 - axis] = slice(0, 1)
            sl_hi[2 - axis] = slice(-1, None)
            if not lo:
                inner[tuple(sl_lo)] = True
            if not hi:
                inner[tuple(sl_hi)] = True
        assert np.array_equal(u[inner], ref[inner]), q
        outer = fm & ghost_mask(mx, my, mz) & ~inner
        assert np.array_equal(u[outer], v[outer]), q       # boundary ghosts untouched
        assert np.array_equal(u[1:-1, 1:-1, 1:-1], v[1:-1, 1:-1, 1:-1])


def test_exchange_rejects_mismatched_faces():
    a = np.zeros((5, 6, 7))
    b = np.zeros((5, 5, 7))
    with pytest.raises(ValueError):
        oracle.exchange_ghosts([a, b], [(0, 0, 1)])   # y extents 4 vs 3
    with pytest.raises(ValueError):
        oracle.exchange_ghosts([a, a], [(0, 3, 1)])


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_split_line_jacobi_equals_whole(axis):
    """Lines along `axis` stay whole when the patch is cut across the two other
    axes, so Jacobi line sweeps of the sub-patches with an exchange after
    every sweep are the whole patch's sweeps, bitwise."""
    p = small_patch(13, 10, 9, seed=7 + axis, eps=EPS)
    cuts = [[5, 9], [4], [3, 6]]
    cuts[axis] = []
    s = split_patch(p, tuple(cuts))
    got = oracle.patchset_sweeps(s.u0, s.f, s.eps, s.h, s.links, "line", axis, oracle.JACOBI, 0.8, 4)
    ref = oracle.line_sweeps(p.u0, p.f, p.eps, p.h, axis, oracle.JACOBI, 0.8, 4)
    s.u0 = got
    assert np.array_equal(_assemble(s, p.f.shape), ref[1:-1, 1:-1, 1:-1])


@pytest.mark.parametrize("normal", [0, 1, 2])
def test_split_plane_jacobi_equals_whole(normal):
    p = small_patch(9, 8, 10, seed=17 + normal, eps=EPS)
    cuts = [[], [], []]
    cuts[normal] = [3, 5]
    s = split_patch(p, tuple(cuts))
    got = oracle.patchset_sweeps(s.u0, s.f, s.eps, s.h, s.links, "plane", normal, oracle.JACOBI, 0.8, 3)
    ref = oracle.plane_sweeps(p.u0, p.f, p.eps, p.h, normal, oracle.JACOBI, 0.8, 3)
    s.u0 = got
    assert np.array_equal(_assemble(s, p.f.shape), ref[1:-1, 1:-1, 1:-1])


def test_split_cube_jacobi_equals_whole():
    p = small_patch(12, 8, 10, seed=27, eps=EPS)
    s = split_patch(p, ([4, 8], [4], [4]))   # cuts on 4^3 block boundaries
    got = oracle.patchset_sweeps(s.u0, s.f, s.eps, s.h, s.links, "cube", (4, 4, 4), oracle.JACOBI, 0.8, 3)
    ref = oracle.cube_sweeps(p.u0, p.f, p.eps, p.h, (4, 4, 4), oracle.JACOBI, 0.8, 3)
    s.u0 = got
    assert relerr(_assemble(s, p.f.shape), ref[1:-1, 1:-1, 1:-1]) < 1e-14


@pytest.mark.parametrize("scheme", [oracle.JACOBI, oracle.LEX_GS, oracle.COLORED_GS])
def test_whole_solution_is_fixed_point_of_split_sweeps(scheme):
    """Cutting lines too (x-lines cut at x = 5): the exact solution of the whole
    box is still a fixed point of every scheme with exchange."""
    p = small_patch(11, 9, 8, seed=37, eps=EPS)
    r, _ = oracle.residual(p.u0, np.zeros_like(p.f), p.eps, p.h)
    p.f = -r / (p.h * p.h)
    s = split_patch(p, ([5], [4], [3]))
    for kind, arg in (("line", 0), ("line", 2), ("plane", 1)):
        got = oracle.patchset_sweeps(s.u0, s.f, s.eps, s.h, s.links, kind, arg, scheme, 1.0, 2)
        t = split_patch(p, ([5], [4], [3]))
        t.u0 = got
        assert relerr(_assemble(t, p.f.shape), p.u0[1:-1, 1:-1, 1:-1]) < 1e-13, (kind, arg)


def test_split_lines_converge_to_whole_solution():
    """With x-lines cut, Jacobi with exchange is a different (weaker) smoother,
    yet it converges to the same solution as the whole patch."""
    p = small_patch(10, 6, 5, seed=47, eps=(1.0, 1.0, 1.0))
    s = split_patch(p, ([4], [], []))
    got = oracle.patchset_sweeps(s.u0, s.f, s.eps, s.h, s.links, "line", 0, oracle.JACOBI, 1.0, 400)
    ref = oracle.line_sweeps(p.u0, p.f, p.eps, p.h, 0, oracle.JACOBI, 1.0, 400)
    s.u0 = got
    assert relerr(_assemble(s, p.f.shape), ref[1:-1, 1:-1, 1:-1]) < 1e-8
