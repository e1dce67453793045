"""Pins for the oracle's geometric cube blocks (blocks of bx x by x bz cells
tiling the patch from its origin, shorter at the upper ends; each block solved
exactly): dense brute force of the splitting, the special cases that are
point, line and plane blocks, and the whole patch as one block.

Runs on the CPU only (no GPU, no HIP library)."""
import numpy as np
import pytest

import brute
import oracle
from conftest import relerr
from workloads import small_patch

EPS = (1.0, 3.0, 7.0)
CODE = {"jacobi": oracle.JACOBI, "lex": oracle.LEX_GS, "colored": oracle.COLORED_GS}


@pytest.fixture(scope="module", autouse=True)
def _threads():
    oracle.set_threads(4)
    yield


@pytest.mark.parametrize("dims,block", [((5, 4, 3), (2, 2, 2)), ((6, 5, 4), (2, 3, 2)), ((7, 4, 5), (3, 1, 2)),
                                        ((4, 4, 4), (4, 4, 1)), ((5, 6, 3), (5, 2, 3)), ((12, 10, 9), (8, 8, 8))])
@pytest.mark.parametrize("scheme,omega", [("jacobi", 0.8), ("jacobi", 1.0), ("lex", 1.0), ("colored", 1.0),
                                          ("colored", 0.7)])
def test_cubes_vs_dense(dims, block, scheme, omega):
    """The splitting of eq. sm:blockm with geometric blocks, as dense matrices
    (block diagonal for Jacobi, block lower triangular in the visiting order for
    GS); ragged last blocks in every axis."""
    if dims == (12, 10, 9) and scheme != "jacobi":
        pytest.skip("one scheme suffices at the largest brute-force size")
    p = small_patch(*dims, seed=31 + sum(block), eps=EPS)
    got = oracle.cube_sweeps(p.u0, p.f, p.eps, p.h, block, CODE[scheme], omega, 2)
    ref = brute.sweeps(p.u0, p.f, p.eps, p.h, "cube", block, scheme, omega, 2)
    assert relerr(got, ref) < 1e-13
    gm = ~np.pad(np.ones(p.f.shape, bool), 1, constant_values=False)
    assert np.array_equal(got[gm], p.u0[gm])


def test_point_blocks_are_point_jacobi():
    """1 x 1 x 1 blocks: u + omega r / d with r the 7-point residual, written
    out here with array slices."""
    p = small_patch(9, 7, 6, seed=4, eps=EPS)
    got = oracle.cube_sweeps(p.u0, p.f, p.eps, p.h, (1, 1, 1), oracle.JACOBI, 0.8, 1)
    u = p.u0
    ex, ey, ez = p.eps
    c = u[1:-1, 1:-1, 1:-1]
    au = (ex * (2 * c - u[1:-1, 1:-1, :-2] - u[1:-1, 1:-1, 2:]) + ey * (2 * c - u[1:-1, :-2, 1:-1] - u[1:-1, 2:, 1:-1])
          + ez * (2 * c - u[:-2, 1:-1, 1:-1] - u[2:, 1:-1, 1:-1]))
    r = p.h ** 2 * p.f - au
    ref = u.copy()
    ref[1:-1, 1:-1, 1:-1] = c + 0.8 * r / (2 * (ex + ey + ez))
    assert relerr(got, ref) < 1e-14


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("scheme,omega", [("jacobi", 0.8), ("lex", 1.0), ("colored", 1.0)])
def test_line_shaped_blocks_are_line_blocks(axis, scheme, omega):
    """A block spanning one whole axis and one cell of the others is a line:
    the Cholesky solve must give the Thomas-solved line sweeps, in the same
    visiting order and colouring."""
    p = small_patch(7, 6, 5, seed=8 + axis, eps=EPS)
    block = [1, 1, 1]
    block[axis] = p.f.shape[2 - axis]
    got = oracle.cube_sweeps(p.u0, p.f, p.eps, p.h, tuple(block), CODE[scheme], omega, 3)
    ref = oracle.line_sweeps(p.u0, p.f, p.eps, p.h, axis, CODE[scheme], omega, 3)
    assert relerr(got, ref) < 1e-13


@pytest.mark.parametrize("normal", [0, 1, 2])
@pytest.mark.parametrize("scheme,omega", [("jacobi", 0.8), ("lex", 1.0), ("colored", 1.0)])
def test_plane_shaped_blocks_are_plane_blocks(normal, scheme, omega):
    """A block spanning two whole axes and one cell of the third is a plane: the
    dense solve must give the partial-diagonalisation plane sweeps."""
    p = small_patch(7, 6, 5, seed=18 + normal, eps=EPS)
    block = list(p.f.shape[::-1])
    block[normal] = 1
    got = oracle.cube_sweeps(p.u0, p.f, p.eps, p.h, tuple(block), CODE[scheme], omega, 3)
    ref = oracle.plane_sweeps(p.u0, p.f, p.eps, p.h, normal, CODE[scheme], omega, 3)
    assert relerr(got, ref) < 1e-13


@pytest.mark.parametrize("dims", [(8, 8, 8), (6, 5, 7)])
def test_whole_patch_block_solves_the_system(dims):
    """One block covering the patch, omega = 1: a single sweep solves A u = h^2 f
    with the ghosts as Dirichlet data, so the residual vanishes to rounding."""
    p = small_patch(*dims, seed=2, eps=EPS)
    got = oracle.cube_sweeps(p.u0, p.f, p.eps, p.h, dims, oracle.JACOBI, 1.0, 1)
    r, _ = oracle.residual(got, p.f, p.eps, p.h)
    r0, _ = oracle.residual(p.u0, p.f, p.eps, p.h)
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(r0))


def test_blocks_larger_than_the_patch_are_clipped():
    p = small_patch(3, 4, 2, seed=6, eps=EPS)
    a = oracle.cube_sweeps(p.u0, p.f, p.eps, p.h, (8, 8, 8), oracle.JACOBI, 0.8, 2)
    b = oracle.cube_sweeps(p.u0, p.f, p.eps, p.h, (3, 4, 2), oracle.JACOBI, 0.8, 2)
    assert np.array_equal(a, b)


STUDY_SIZES = [(2, 2, 2), (4, 2, 2), (4, 4, 2), (4, 4, 4), (8, 4, 4), (8, 8, 4), (8, 8, 8)]


@pytest.mark.parametrize("scheme,omega", [("jacobi", 0.8), ("colored", 1.0)])
def test_block_size_study_improves_monotonically(scheme, omega):
    """The block-size study (section 3): random initial guess, f = 0, three
    sweeps; the relative residual improves monotonically with the block sizes
    the paper lists (here on a 16^3 patch; point blocks first)."""
    from workloads import make_patch
    p = make_patch(16, 16, 16, (1.0, 1.0, 1.0), 1.0 / 16, seed=7, f="zero", u0="uniform", ghosts="zero")
    r0 = np.sqrt(oracle.residual(p.u0, p.f, p.eps, p.h)[1])
    rel = []
    for b in [(1, 1, 1)] + STUDY_SIZES:
        u = oracle.cube_sweeps(p.u0, p.f, p.eps, p.h, b, CODE[scheme], omega, 3)
        rel.append(np.sqrt(oracle.residual(u, p.f, p.eps, p.h)[1]) / r0)
    assert all(a > b for a, b in zip(rel, rel[1:])), rel
    assert rel[-1] < 0.5 * rel[0]
