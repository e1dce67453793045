"""Pins for the oracle's extrapolated-Dirichlet boundary reading (section 1.1:
boundary conditions are extrapolated into the ghost layer): on a face whose
bit is set, the ghost is -(the adjacent interior value), i.e. zero on the
face, and the ghost term folds into the operator and into every block.
Pinned by dense brute force, by the DST-II / mixed sine eigenmodes that these
boundaries have in closed form, and by the exact solution as a fixed point."""
import math

import numpy as np
import pytest

import brute
import oracle
from conftest import relerr
from workloads import small_patch

EPS = (1.0, 3.0, 7.0)
MASKS = [oracle.BC_ALL, 0b010110, 0b000001, 0b101000]
CODE = {"jacobi": oracle.JACOBI, "lex": oracle.LEX_GS, "colored": oracle.COLORED_GS}


@pytest.fixture(scope="module", autouse=True)
def _threads():
    oracle.set_threads(4)
    yield


@pytest.mark.parametrize("bc", MASKS)
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("scheme,omega", [("jacobi", 0.8), ("lex", 1.0), ("colored", 1.0)])
def test_lines_vs_dense(bc, axis, scheme, omega):
    p = small_patch(5, 4, 6, seed=11 + axis, eps=EPS)
    got = oracle.line_sweeps(p.u0, p.f, p.eps, p.h, axis, CODE[scheme], omega, 3, bc=bc)
    ref = brute.sweeps(p.u0, p.f, p.eps, p.h, "line", axis, scheme, omega, 3, bc=bc)
    assert relerr(got, ref) < 1e-14
    gm = ~np.pad(np.ones(p.f.shape, bool), 1, constant_values=False)
    assert np.array_equal(got[gm], p.u0[gm])     # ghosts are never written


@pytest.mark.parametrize("bc", MASKS)
@pytest.mark.parametrize("normal", [0, 1, 2])
@pytest.mark.parametrize("scheme,omega", [("jacobi", 0.8), ("lex", 1.0), ("colored", 1.0)])
def test_planes_vs_dense(bc, normal, scheme, omega):
    p = small_patch(6, 5, 4, seed=21 + normal, eps=EPS)
    got = oracle.plane_sweeps(p.u0, p.f, p.eps, p.h, normal, CODE[scheme], omega, 3, bc=bc)
    ref = brute.sweeps(p.u0, p.f, p.eps, p.h, "plane", normal, scheme, omega, 3, bc=bc)
    assert relerr(got, ref) < 1e-13


@pytest.mark.parametrize("bc", MASKS)
@pytest.mark.parametrize("scheme,omega", [("jacobi", 0.8), ("colored", 1.0)])
def test_cubes_vs_dense(bc, scheme, omega):
    p = small_patch(7, 5, 6, seed=31, eps=EPS)
    got = oracle.cube_sweeps(p.u0, p.f, p.eps, p.h, (3, 2, 4), CODE[scheme], omega, 2, bc=bc)
    ref = brute.sweeps(p.u0, p.f, p.eps, p.h, "cube", (3, 2, 4), scheme, omega, 2, bc=bc)
    assert relerr(got, ref) < 1e-13


def _mode(dims, thetas, kinds):
    """Product of sines: kind 'I' sin(theta (i+1)), 'II' sin(theta (i+1/2)),
    'lo' sin(theta (i+1/2)), 'hi' sin(theta (n-i-1/2)); padded, zero ghosts."""
    vs = []
    for n, th, kd in zip(dims, thetas, kinds):
        i = np.arange(n)
        if kd == "I":
            vs.append(np.sin(th * (i + 1)))
        elif kd == "hi":
            vs.append(np.sin(th * (n - i - 0.5)))
        else:
            vs.append(np.sin(th * (i + 0.5)))
    u = np.zeros((dims[2] + 2, dims[1] + 2, dims[0] + 2))
    u[1:-1, 1:-1, 1:-1] = vs[2][:, None, None] * vs[1][None, :, None] * vs[0][None, None, :]
    return u


def _theta(n, kd, p):
    return {"I": p * math.pi / (n + 1), "II": p * math.pi / n, "lo": p * math.pi / (n + 0.5),
            "hi": p * math.pi / (n + 0.5)}[kd]


@pytest.mark.parametrize("kinds,bc", [(("II", "II", "II"), 63), (("lo", "hi", "II"), 0b111001),
                                      (("I", "II", "lo"), 0b011100)])
def test_residual_of_eigenmodes(kinds, bc):
    """A sine mode of the boundary reading is an eigenvector of the operator:
    with f = 0 the residual is -sum_a 4 eps_a sin^2(theta_a / 2) times the mode."""
    dims = (7, 6, 5)
    th = [_theta(n, kd, p) for n, kd, p in zip(dims, kinds, (2, 5, 3))]
    u = _mode(dims, th, kinds)
    lam = sum(4 * e * math.sin(t / 2) ** 2 for e, t in zip(EPS, th))
    r, _ = oracle.residual(u, np.zeros((5, 6, 7)), EPS, 0.1, bc=bc)
    assert relerr(r, -lam * u[1:-1, 1:-1, 1:-1]) < 1e-13


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_line_jacobi_damping_of_dst2_modes(axis):
    """Extrapolated faces along the line axis only (zero ghosts elsewhere): the
    mode with a DST-II profile along the line and DST-I profiles across it is
    damped by g = 1 - omega + omega nu / mu, mu = 4 eps_a sin^2(theta_a/2) +
    2 eps_b + 2 eps_c, nu = 2 eps_b cos(theta_b) + 2 eps_c cos(theta_c)."""
    dims = (8, 7, 6)
    kinds = ["I", "I", "I"]
    kinds[axis] = "II"
    th = [_theta(n, kd, p) for n, kd, p in zip(dims, kinds, (3, 2, 4))]
    bc = 3 << (2 * axis)
    u = _mode(dims, th, kinds)
    others = [b for b in (0, 1, 2) if b != axis]
    mu = 4 * EPS[axis] * math.sin(th[axis] / 2) ** 2 + sum(2 * EPS[b] for b in others)
    nu = sum(2 * EPS[b] * math.cos(th[b]) for b in others)
    om = 0.8
    g = 1 - om + om * nu / mu
    got = oracle.line_sweeps(u, np.zeros((6, 7, 8)), EPS, 0.1, axis, oracle.JACOBI, om, 1, bc=bc)
    assert relerr(got, g * u) < 1e-13


@pytest.mark.parametrize("normal", [0, 1, 2])
@pytest.mark.parametrize("inplane", [("II", "II"), ("lo", "hi")])
def test_plane_jacobi_damping_of_dst2_modes(normal, inplane):
    """Extrapolated faces along the two in-plane axes: g = 1 - omega + omega
    nu / mu, mu = sum over in-plane axes of 4 eps sin^2(theta/2) + 2 eps_c,
    nu = 2 eps_c cos(theta_c)."""
    dims = (6, 7, 8)
    a, b = [x for x in (0, 1, 2) if x != normal]
    kinds = ["I", "I", "I"]
    kinds[a], kinds[b] = inplane
    bcbits = {"II": 3, "lo": 1, "hi": 2}
    bc = (bcbits[inplane[0]] << (2 * a)) | (bcbits[inplane[1]] << (2 * b))
    th = [_theta(n, kd, p) for n, kd, p in zip(dims, kinds, (2, 3, 5))]
    u = _mode(dims, th, kinds)
    mu = sum(4 * EPS[x] * math.sin(th[x] / 2) ** 2 for x in (a, b)) + 2 * EPS[normal]
    nu = 2 * EPS[normal] * math.cos(th[normal])
    om = 0.8
    g = 1 - om + om * nu / mu
    got = oracle.plane_sweeps(u, np.zeros((8, 7, 6)), EPS, 0.1, normal, oracle.JACOBI, om, 1, bc=bc)
    assert relerr(got, g * u) < 1e-13


@pytest.mark.parametrize("bc", MASKS)
def test_exact_solution_is_fixed_point(bc):
    p = small_patch(9, 8, 7, seed=41, eps=(2.0, 1.0, 5.0))
    r, _ = oracle.residual(p.u0, np.zeros_like(p.f), p.eps, p.h, bc=bc)
    f = -r / (p.h * p.h)
    for kind, fn, arg in (("line", oracle.line_sweeps, 1), ("plane", oracle.plane_sweeps, 2),
                          ("cube", oracle.cube_sweeps, (4, 4, 4))):
        for sch in (oracle.JACOBI, oracle.LEX_GS, oracle.COLORED_GS):
            got = fn(p.u0, f, p.eps, p.h, arg, sch, 0.9, 2, bc=bc)
            assert relerr(got, p.u0) < 1e-13, (kind, sch)


def test_masked_ghosts_are_never_read():
    """Values stored in the ghosts of extrapolated faces change nothing."""
    p = small_patch(6, 5, 4, seed=51, eps=EPS)
    q = p.u0.copy()
    q[:, :, 0] = 1e6                    # low x face (bit 0)
    q[-1, :, :] = -1e6                  # high z face (bit 5)
    bc = 0b100001
    for fn, arg in ((oracle.line_sweeps, 0), (oracle.plane_sweeps, 1), (oracle.cube_sweeps, (2, 2, 2))):
        a = fn(p.u0, p.f, p.eps, p.h, arg, oracle.COLORED_GS, 1.0, 2, bc=bc)
        b = fn(q, p.f, p.eps, p.h, arg, oracle.COLORED_GS, 1.0, 2, bc=bc)
        assert np.array_equal(a[1:-1, 1:-1, 1:-1], b[1:-1, 1:-1, 1:-1])
