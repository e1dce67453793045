"""Pins for the oracle's multigrid with block smoothers (section 1: line and
plane smoothers as components of robust geometric multigrid; section 5):
transfers against independent NumPy forms and exactness properties, the
two-grid cycle against a dense brute force, and the V-cycle's convergence
factor, which must stay small and independent of the grid size."""
import math

import numpy as np
import pytest

import brute
import oracle
from conftest import relerr
from workloads import make_patch, small_patch


@pytest.fixture(scope="module", autouse=True)
def _threads():
    oracle.set_threads(4)
    yield


def test_restriction_is_the_mean_of_children():
    rng = np.random.default_rng(0)
    r = rng.uniform(-1, 1, (6, 4, 8))
    got = oracle.restrict(r, 3.0)
    ref = 3.0 * r.reshape(3, 2, 2, 2, 4, 2).mean(axis=(1, 3, 5))
    assert relerr(got, ref) < 1e-15
    assert oracle.restrict(np.full((4, 4, 4), 2.5)).tolist() == np.full((2, 2, 2), 2.5).tolist()
    with pytest.raises(ValueError):
        oracle.restrict(np.zeros((3, 4, 4)))


def _p1(n, extrap=False):
    """1D cell-centred linear interpolation, fine n = 2m from coarse m with zero
    ghosts, or with extrapolated ghosts (-(the end value)) when extrap."""
    m = n // 2
    P = np.zeros((n, m))
    for i in range(n):
        I = i // 2
        P[i, I] += 0.75
        nb = I + (1 if i % 2 else -1)
        if 0 <= nb < m:
            P[i, nb] += 0.25
        elif extrap:
            P[i, I] -= 0.25
    return P


def test_prolongation_against_kronecker_form():
    """Trilinear prolongation equals the Kronecker product of 1D linear
    interpolations (zero coarse ghosts)."""
    rng = np.random.default_rng(1)
    nx, ny, nz = 8, 6, 4
    uc = np.zeros((nz // 2 + 2, ny // 2 + 2, nx // 2 + 2))
    ec = rng.uniform(-1, 1, (nz // 2, ny // 2, nx // 2))
    uc[1:-1, 1:-1, 1:-1] = ec
    base = np.pad(rng.uniform(-1, 1, (nz, ny, nx)), 1)
    got = oracle.prolong_add(uc, base)
    P = np.kron(_p1(nz), np.kron(_p1(ny), _p1(nx)))
    ref = base[1:-1, 1:-1, 1:-1].reshape(-1) + P @ ec.reshape(-1)
    assert relerr(got[1:-1, 1:-1, 1:-1].reshape(-1), ref) < 1e-15
    assert np.array_equal(got[0], base[0])          # ghosts untouched


def test_prolongation_reproduces_trilinear_functions():
    """Tensor-product linear interpolation is exact on span{1,x} x {1,y} x {1,z}
    (coarse ghosts holding the function's values at the ghost centres)."""
    nx, ny, nz = 8, 10, 6
    fun = lambda x, y, z: 0.3 + 1.1 * x - 0.7 * y + 0.5 * z + 0.9 * x * y - 1.3 * y * z + 0.4 * x * y * z
    cz, cy, cx = (np.arange(-1, n // 2 + 1) * 2.0 + 0.5 for n in (nz, ny, nx))   # coarse centres incl. ghosts
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    uc = fun(X, Y, Z)
    fz, fy, fx = (np.arange(-1, n + 1) + 0.0 for n in (nz, ny, nx))
    Z, Y, X = np.meshgrid(fz, fy, fx, indexing="ij")
    ref = fun(X, Y, Z)
    got = oracle.prolong_add(uc, np.zeros((nz + 2, ny + 2, nx + 2)))
    assert relerr(got[1:-1, 1:-1, 1:-1], ref[1:-1, 1:-1, 1:-1]) < 1e-14


@pytest.mark.parametrize("kind,arg,scheme", [("line", 2, oracle.LEX_GS), ("plane", 0, oracle.JACOBI),
                                             ("line", 0, oracle.COLORED_GS)])
@pytest.mark.parametrize("bc,cbc", [(0, 0), (0, 63), (63, 63)])
def test_two_grid_against_dense(kind, arg, scheme, bc, cbc):
    """Two levels with the coarse problem solved to convergence: against a
    dense two-grid cycle built from the definitions (independent R, P, coarse
    matrix with cell width 2h and the smoother's sweeps from the brute force),
    for zero or extrapolated fine faces and zero or extrapolated coarse faces."""
    nx, ny, nz = 6, 4, 8
    eps = (1.0, 3.0, 7.0)
    p = small_patch(nx, ny, nz, seed=3, eps=eps)
    h = p.h
    name = {oracle.JACOBI: "jacobi", oracle.LEX_GS: "lex", oracle.COLORED_GS: "colored"}[scheme]
    om = 0.8 if scheme == oracle.JACOBI else 1.0
    got = oracle.vcycle(p.u0, p.f, eps, h, kind, arg, scheme, om, 2, 1, 400, levels=2, bc=bc, coarse_bc=cbc)
    # dense form
    u1 = brute.sweeps(p.u0, p.f, eps, h, kind, arg, name, om, 2, bc=bc)
    A = brute.assemble(nx, ny, nz, eps, bc)
    b = h * h * p.f.reshape(-1) + brute.ghost_rhs(p.u0, eps, bc)
    d = b - A @ u1[1:-1, 1:-1, 1:-1].reshape(-1)
    R = np.kron(np.kron(np.eye(nz // 2).repeat(2, 1), np.eye(ny // 2).repeat(2, 1)), np.eye(nx // 2).repeat(2, 1)) / 8
    Ac = brute.assemble(nx // 2, ny // 2, nz // 2, eps, cbc)
    ec = np.linalg.solve(Ac, (2 * h) ** 2 * (R @ d) / h ** 2)
    ex = cbc == 63
    P = np.kron(_p1(nz, ex), np.kron(_p1(ny, ex), _p1(nx, ex)))
    u2 = u1.copy()
    u2[1:-1, 1:-1, 1:-1] += (P @ ec).reshape(nz, ny, nx)
    ref = brute.sweeps(u2, p.f, eps, h, kind, arg, name, om, 1, bc=bc)
    assert relerr(got, ref) < 1e-12


def test_exact_solution_is_fixed_point_of_vcycle():
    p = small_patch(16, 8, 16, seed=9, eps=(1.0, 1.0, 50.0))
    r, _ = oracle.residual(p.u0, np.zeros_like(p.f), p.eps, p.h)
    f = -r / (p.h * p.h)
    got = oracle.vcycle(p.u0, f, p.eps, p.h, "line", 2, oracle.COLORED_GS, 1.0, 1, 1, 10)
    assert relerr(got, p.u0) < 1e-13


@pytest.mark.parametrize("kind,arg,eps", [("line", 2, (1.0, 1.0, 100.0)), ("plane", 0, (1.0, 100.0, 100.0)),
                                          ("line", 0, (1.0, 1.0, 1.0))])
@pytest.mark.parametrize("bc", [0, oracle.BC_ALL])
def test_vcycle_factor_small_and_grid_independent(kind, arg, eps, bc):
    """V(1,1) with two-colour GS block smoothing and full coarsening: a line
    smoother along the strong axis, or a plane smoother in the strong plane,
    keeps the cycle's residual reduction small and independent of n (8, 16,
    32), for zero ghosts or extrapolated faces on the fine level.  The coarse
    error equations take the extrapolated (zero-at-the-face) condition on every
    face, which puts the boundary at the same place on every level; with zero
    ghosts there instead (zero one coarse cell width beyond each face, a
    boundary that moves out with each level) the cycle loses its
    grid-independence (0.22 -> 0.48 -> 0.81 from 8^3 to 32^3 for x-lines)."""
    facs = []
    for n in (8, 16, 32):
        p = make_patch(n, n, n, eps, 1.0 / n, seed=4, f="zero", u0="uniform")
        u = p.u0
        r0 = math.sqrt(oracle.residual(u, p.f, eps, p.h, bc=bc)[1])
        rs = [r0]
        for _ in range(6):
            u = oracle.vcycle(u, p.f, eps, p.h, kind, arg, oracle.COLORED_GS, 1.0, 1, 1, 20, bc=bc,
                              coarse_bc=oracle.BC_ALL)
            rs.append(math.sqrt(oracle.residual(u, p.f, eps, p.h, bc=bc)[1]))
        facs.append((rs[6] / rs[3]) ** (1 / 3))
    assert max(facs) < 0.3, facs
    assert max(facs) - min(facs) < 0.08, facs
