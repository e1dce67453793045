"""Pins for the oracle's reverse mode of line and plane block sweeps under
damped block Jacobi and two-colour block GS (the adjoints of the
differentiable smoother beyond Jacobi line sweeps).

The sweep map is affine in (u0, f, ghosts): x_K = T^K x_0 + sum_j T^j M^{-1}
(h^2 f + B g) with T = I - M^{-1} A, M the scheme's splitting (eq.
blockiteration2; two-colour GS with omega is the SOR splitting D/omega + L in
colour order).  The dense brute force builds T, M, A and B from their
definitions (tests/brute.py, no oracle code), so the gradients in u0, f and the
face ghosts are checked against the transposed dense Jacobians, and the eps
gradient against central differences of the dense sweeps."""
import numpy as np
import pytest

import brute
import oracle
from conftest import relerr
from workloads import small_patch


@pytest.fixture(scope="module", autouse=True)
def _threads():
    oracle.set_threads(2)
    yield


def _faces(nx, ny, nz):
    """Padded-array indices of every face ghost cell (edges and corners excluded)."""
    out = []
    for k in range(nz + 2):
        for j in range(ny + 2):
            for i in range(nx + 2):
                outside = (i in (0, nx + 1)) + (j in (0, ny + 1)) + (k in (0, nz + 1))
                if outside == 1:
                    out.append((k, j, i))
    return out


def _dense_grads(p, kind, axis, scheme, omega, K, gK):
    nx, ny, nz = p.dims
    A = brute.assemble(nx, ny, nz, p.eps)
    bid, order, colour = brute.block_ids(nx, ny, nz, kind, axis)
    M = brute.splitting(A, bid, order, colour, scheme, omega)
    m = A.shape[0]
    T = np.eye(m) - np.linalg.solve(M, A)
    Minv = np.linalg.inv(M)
    TK = np.linalg.matrix_power(T, K)
    S = sum(np.linalg.matrix_power(T, j) for j in range(K)) @ Minv
    g = gK[1:-1, 1:-1, 1:-1].reshape(-1)
    gu = TK.T @ g
    gf = (p.h * p.h) * (S.T @ g)
    # ghost gradients: column of B for each face ghost cell
    sg = S.T @ g
    gg = {}
    for (k, j, i) in _faces(nx, ny, nz):
        e = np.zeros((nz + 2, ny + 2, nx + 2))
        e[k, j, i] = 1.0
        gg[(k, j, i)] = float(brute.ghost_rhs(e, p.eps) @ sg)
    return gu.reshape(nz, ny, nx), gf.reshape(nz, ny, nx), gg


def _fd_eps(p, kind, axis, scheme, omega, K, gK, hrel=1e-6):
    out = []
    for b in range(3):
        vals = []
        for sgn in (1, -1):
            e = list(p.eps)
            e[b] *= 1 + sgn * hrel
            uK = brute.sweeps(p.u0, p.f, tuple(e), p.h, kind, axis, scheme, omega, K)
            vals.append(float(np.sum(gK[1:-1, 1:-1, 1:-1] * uK[1:-1, 1:-1, 1:-1])))
        out.append((vals[0] - vals[1]) / (2 * hrel * p.eps[b]))
    return np.array(out)


CASES = [("line", 0), ("line", 1), ("line", 2), ("plane", 0), ("plane", 1), ("plane", 2)]
OS = {"jacobi": oracle.JACOBI, "colored": oracle.COLORED_GS}


@pytest.mark.parametrize("kind,axis", CASES)
@pytest.mark.parametrize("scheme,omega", [("jacobi", 0.8), ("colored", 1.0), ("colored", 1.3)])
@pytest.mark.parametrize("dims", [(3, 4, 2), (4, 3, 5)])
def test_block_adjoint_against_dense(kind, axis, scheme, omega, dims):
    p = small_patch(*dims, seed=13, eps=(1.0, 3.0, 7.0))
    K = 3
    rng = np.random.default_rng(5)
    gK = rng.uniform(-1, 1, p.u0.shape)
    g_u0, g_f, g_eps = oracle.block_adjoint(p.u0, p.f, p.eps, p.h, kind, axis, OS[scheme], omega, K, gK)
    gu, gf, gg = _dense_grads(p, kind, axis, scheme, omega, K, gK)
    assert relerr(g_u0[1:-1, 1:-1, 1:-1], gu) < 1e-12
    assert relerr(g_f, gf) < 1e-12
    got_g = np.array([g_u0[c] for c in gg])
    assert relerr(got_g, np.array(list(gg.values()))) < 1e-12
    fd = _fd_eps(p, kind, axis, scheme, omega, K, gK)
    assert np.max(np.abs(g_eps - fd)) / np.max(np.abs(fd)) < 1e-6


def test_jacobi_lines_equal_the_line_adjoint():
    p = small_patch(7, 6, 5, seed=2, eps=(1.0, 2.0, 9.0))
    gK = np.random.default_rng(1).uniform(-1, 1, p.u0.shape)
    for axis in (0, 1, 2):
        a = oracle.block_adjoint(p.u0, p.f, p.eps, p.h, "line", axis, oracle.JACOBI, 0.8, 4, gK)
        b = oracle.line_jacobi_adjoint(p.u0, p.f, p.eps, p.h, axis, 0.8, 4, gK)
        for x, y in zip(a, b):
            assert relerr(x, y) < 1e-13


def test_colored_adjoint_reverses_colour_order():
    """One two-colour sweep is colour 0 then colour 1; its adjoint must undo them
    in reverse order: running the half-steps the other way round (the brute
    force with colours swapped) gives different gradients, and the oracle
    matches only the right order."""
    p = small_patch(4, 4, 3, seed=8, eps=(1.0, 1.0, 5.0))
    gK = np.random.default_rng(2).uniform(-1, 1, p.u0.shape)
    g_u0, _, _ = oracle.block_adjoint(p.u0, p.f, p.eps, p.h, "line", 2, oracle.COLORED_GS, 1.0, 1, gK)
    gu, _, _ = _dense_grads(p, "line", 2, "colored", 1.0, 1, gK)
    assert relerr(g_u0[1:-1, 1:-1, 1:-1], gu) < 1e-12
    nx, ny, nz = p.dims
    A = brute.assemble(nx, ny, nz, p.eps)
    bid, order, colour = brute.block_ids(nx, ny, nz, "line", 2)
    Mswap = brute.splitting(A, bid, order, 1 - colour, "colored", 1.0)
    Tswap = np.eye(A.shape[0]) - np.linalg.solve(Mswap, A)
    wrong = Tswap.T @ gK[1:-1, 1:-1, 1:-1].reshape(-1)
    assert relerr(g_u0[1:-1, 1:-1, 1:-1].reshape(-1), wrong) > 1e-3
