"""Pins for the oracle: each test checks it against something other than
itself -- dense brute force, closed forms, eigenvalues, invariants.

Runs on the CPU only (no GPU, no HIP library)."""
import math

import numpy as np
import pytest
import scipy.linalg

import brute
import oracle
from conftest import relerr
from workloads import small_patch

GRIDS = [(5, 4, 3), (7, 6, 5)]
EPS = (1.0, 3.0, 7.0)


@pytest.fixture(scope="module", autouse=True)
def _threads():
    oracle.set_threads(4)
    yield


# --- dense brute force (every block kind, scheme and axis) -----------------------------------

@pytest.mark.parametrize("dims", GRIDS)
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("scheme,omega", [("jacobi", 0.8), ("jacobi", 1.0), ("lex", 1.0), ("lex", 1.3),
                                          ("colored", 1.0), ("colored", 0.7)])
def test_lines_vs_dense(dims, axis, scheme, omega):
    p = small_patch(*dims, seed=11 + axis, eps=EPS)
    code = {"jacobi": oracle.JACOBI, "lex": oracle.LEX_GS, "colored": oracle.COLORED_GS}[scheme]
    got = oracle.line_sweeps(p.u0, p.f, p.eps, p.h, axis, code, omega, 3)
    ref = brute.sweeps(p.u0, p.f, p.eps, p.h, "line", axis, scheme, omega, 3)
    assert relerr(got, ref) < 1e-14
    # ghosts are never modified
    gm = ~np.pad(np.ones(p.f.shape, bool), 1, constant_values=False)
    assert np.array_equal(got[gm], p.u0[gm])


@pytest.mark.parametrize("dims", GRIDS)
@pytest.mark.parametrize("normal", [0, 1, 2])
@pytest.mark.parametrize("scheme,omega", [("jacobi", 0.8), ("jacobi", 1.0), ("lex", 1.0), ("colored", 1.0)])
def test_planes_vs_dense(dims, normal, scheme, omega):
    p = small_patch(*dims, seed=21 + normal, eps=EPS)
    code = {"jacobi": oracle.JACOBI, "lex": oracle.LEX_GS, "colored": oracle.COLORED_GS}[scheme]
    got = oracle.plane_sweeps(p.u0, p.f, p.eps, p.h, normal, code, omega, 3)
    ref = brute.sweeps(p.u0, p.f, p.eps, p.h, "plane", normal, scheme, omega, 3)
    assert relerr(got, ref) < 1e-14


def test_dense_brute_force_of_single_cells_is_point_gauss_seidel():
    """Sanity of the brute force itself: with 1x1x1 'lines' (a 1-cell axis) the
    block iteration is the point iteration of eq. sm:blockm with s = m."""
    p = small_patch(1, 4, 3, seed=5, eps=EPS)
    got = oracle.line_sweeps(p.u0, p.f, p.eps, p.h, 0, oracle.LEX_GS, 1.0, 2)
    # point lexicographic Gauss-Seidel written out directly
    u = p.u0.copy()
    ex, ey, ez = p.eps
    d = 2 * (ex + ey + ez)
    for _ in range(2):
        for k in range(1, 4):
            for j in range(1, 5):
                i = 1
                s = (ex * (u[k, j, i - 1] + u[k, j, i + 1]) + ey * (u[k, j - 1, i] + u[k, j + 1, i])
                     + ez * (u[k - 1, j, i] + u[k + 1, j, i]))
                u[k, j, i] = (p.h ** 2 * p.f[k - 1, j - 1, i - 1] + s) / d
    assert relerr(got, u) < 1e-14


# --- residual: closed forms --------------------------------------------------------------------

@pytest.mark.parametrize("axis", [0, 1, 2])
def test_residual_of_quadratic_is_constant(axis):
    """For U = i_a^2 (index units, ghosts included) the second difference is
    exactly -2, so with f = 0: r = 2 eps_a at every interior cell."""
    nx, ny, nz = 6, 5, 4
    idx = np.meshgrid(np.arange(-1, nz + 1), np.arange(-1, ny + 1), np.arange(-1, nx + 1), indexing="ij")
    coord = {0: idx[2], 1: idx[1], 2: idx[0]}[axis]
    u = (coord.astype(np.float64)) ** 2
    f = np.zeros((nz, ny, nx))
    r, s = oracle.residual(np.ascontiguousarray(u), f, EPS, 0.25)
    assert np.all(r == 2.0 * EPS[axis])
    assert s == pytest.approx(nx * ny * nz * (2.0 * EPS[axis]) ** 2, rel=1e-15)


def test_residual_of_zero_is_h2f():
    p = small_patch(5, 6, 7, seed=3, ghosts="zero", u0="zero")
    r, _ = oracle.residual(p.u0, p.f, p.eps, p.h)
    assert np.array_equal(r, p.h * p.h * p.f)


def sine_mode(nx, ny, nz, pm):
    """phi = prod_a sin(theta_a (i_a+1)), theta_a = p_a pi / (n_a+1), zero ghosts."""
    th = [pm[0] * math.pi / (nx + 1), pm[1] * math.pi / (ny + 1), pm[2] * math.pi / (nz + 1)]
    sx = np.sin(th[0] * np.arange(1, nx + 1))
    sy = np.sin(th[1] * np.arange(1, ny + 1))
    sz = np.sin(th[2] * np.arange(1, nz + 1))
    u = np.zeros((nz + 2, ny + 2, nx + 2))
    u[1:-1, 1:-1, 1:-1] = sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    return u, th


def test_residual_of_sine_mode_is_eigenvalue():
    nx, ny, nz = 9, 7, 6
    u, th = sine_mode(nx, ny, nz, (2, 3, 1))
    lam = sum(4 * e * math.sin(t / 2) ** 2 for e, t in zip(EPS, th))
    r, _ = oracle.residual(u, np.zeros((nz, ny, nx)), EPS, 0.1)
    assert relerr(r, -lam * u[1:-1, 1:-1, 1:-1]) < 1e-13


# --- Fourier damping of single modes (Jacobi lines and planes) -------------------------------

@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("pm", [(1, 1, 1), (2, 3, 1), (5, 2, 4)])
@pytest.mark.parametrize("omega", [0.8, 1.0])
def test_line_jacobi_damping(axis, pm, omega):
    nx, ny, nz = 9, 7, 6
    u, th = sine_mode(nx, ny, nz, pm)
    others = [b for b in (0, 1, 2) if b != axis]
    mu = 4 * EPS[axis] * math.sin(th[axis] / 2) ** 2 + sum(2 * EPS[b] for b in others)
    nu = sum(2 * EPS[b] * math.cos(th[b]) for b in others)
    g = 1 - omega + omega * nu / mu
    got = oracle.line_sweeps(u, np.zeros((nz, ny, nx)), EPS, 0.1, axis, oracle.JACOBI, omega, 1)
    assert relerr(got, g * u) < 1e-13


@pytest.mark.parametrize("normal", [0, 1, 2])
@pytest.mark.parametrize("pm", [(1, 1, 1), (2, 3, 1), (5, 2, 4)])
def test_plane_jacobi_damping(normal, pm):
    nx, ny, nz = 9, 7, 6
    omega = 0.9
    u, th = sine_mode(nx, ny, nz, pm)
    a, b = [c for c in (0, 1, 2) if c != normal]
    mu = 4 * EPS[a] * math.sin(th[a] / 2) ** 2 + 4 * EPS[b] * math.sin(th[b] / 2) ** 2 + 2 * EPS[normal]
    nu = 2 * EPS[normal] * math.cos(th[normal])
    g = 1 - omega + omega * nu / mu
    got = oracle.plane_sweeps(u, np.zeros((nz, ny, nx)), EPS, 0.1, normal, oracle.JACOBI, omega, 1)
    assert relerr(got, g * u) < 1e-13


# --- fixed point of the exact discrete solution ------------------------------------------------

def exact_rhs(u, eps, h):
    """F with A u = h^2 F for a given padded u: built from the dense matrix
    (brute force), not from the oracle's stencil."""
    nz, ny, nx = (s - 2 for s in u.shape)
    A = brute.assemble(nx, ny, nz, eps)
    x = u[1:-1, 1:-1, 1:-1].reshape(-1)
    b = A @ x - brute.ghost_rhs(u, eps)
    return (b / (h * h)).reshape(nz, ny, nx)


@pytest.mark.parametrize("kind", ["line", "plane"])
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("scheme", [oracle.JACOBI, oracle.LEX_GS, oracle.COLORED_GS])
def test_exact_solution_is_fixed_point(kind, axis, scheme):
    p = small_patch(6, 5, 4, seed=7, eps=EPS)
    f = exact_rhs(p.u0, p.eps, p.h)
    if kind == "line":
        got = oracle.line_sweeps(p.u0, f, p.eps, p.h, axis, scheme, 1.0, 1)
    else:
        got = oracle.plane_sweeps(p.u0, f, p.eps, p.h, axis, scheme, 1.0, 1)
    assert relerr(got, p.u0) < 1e-13


# --- spectral radii and asymptotic rates --------------------------------------------------------

def rho_jacobi_lines(dims, eps, axis):
    """Closed form: max over modes of nu/mu at omega = 1 (lowest modes)."""
    th = [math.pi / (n + 1) for n in dims]
    others = [b for b in (0, 1, 2) if b != axis]
    mu = 4 * eps[axis] * math.sin(th[axis] / 2) ** 2 + sum(2 * eps[b] for b in others)
    nu = sum(2 * eps[b] * math.cos(th[b]) for b in others)
    return nu / mu


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_spectral_radii(axis):
    dims = (6, 5, 4)
    rj = rho_jacobi_lines(dims, EPS, axis)
    G, _, _ = brute.iteration_matrix(*dims, EPS, "line", axis, "jacobi", 1.0)
    assert max(abs(np.linalg.eigvals(G))) == pytest.approx(rj, rel=1e-10)
    # block 2-cyclic, consistently ordered: lexicographic and red-black GS both give rho_J^2
    for scheme in ("lex", "colored"):
        G, _, _ = brute.iteration_matrix(*dims, EPS, "line", axis, scheme, 1.0)
        assert max(abs(np.linalg.eigvals(G))) == pytest.approx(rj ** 2, rel=1e-8)


def test_measured_rates_approach_closed_form():
    """Windowed factor (||r_{i+k}||/||r_i||)^(1/k) (section 3) -> rho."""
    dims, axis = (8, 8, 8), 2
    eps = (1.0, 1.0, 4.0)
    p = small_patch(*dims, seed=9, eps=eps, ghosts="zero")
    f = np.zeros_like(p.f)
    rj = rho_jacobi_lines(dims, eps, axis)
    for scheme, target in ((oracle.JACOBI, rj), (oracle.LEX_GS, rj ** 2), (oracle.COLORED_GS, rj ** 2)):
        u = p.u0
        u = oracle.line_sweeps(u, f, eps, p.h, axis, scheme, 1.0, 150)
        _, s0 = oracle.residual(u, f, eps, p.h)
        u = oracle.line_sweeps(u, f, eps, p.h, axis, scheme, 1.0, 20)
        _, s1 = oracle.residual(u, f, eps, p.h)
        fac = (math.sqrt(s1) / math.sqrt(s0)) ** (1 / 20)
        assert fac == pytest.approx(target, rel=1e-3)


# --- energy is non-increasing (2M/omega - A is SPD for these splittings) -----------------------

@pytest.mark.parametrize("kind", ["line", "plane"])
@pytest.mark.parametrize("scheme,omega", [(oracle.JACOBI, 0.8), (oracle.JACOBI, 1.0), (oracle.LEX_GS, 1.0),
                                          (oracle.COLORED_GS, 1.0)])
def test_energy_monotone(kind, scheme, omega):
    p = small_patch(6, 5, 4, seed=13, eps=EPS)
    A = brute.assemble(6, 5, 4, EPS)
    b = p.h ** 2 * p.f.reshape(-1) + brute.ghost_rhs(p.u0, EPS)

    def energy(u):
        x = u[1:-1, 1:-1, 1:-1].reshape(-1)
        return 0.5 * x @ A @ x - b @ x

    u = p.u0
    e_prev = energy(u)
    for _ in range(8):
        if kind == "line":
            u = oracle.line_sweeps(u, p.f, EPS, p.h, 2, scheme, omega, 1)
        else:
            u = oracle.plane_sweeps(u, p.f, EPS, p.h, 2, scheme, omega, 1)
        e = energy(u)
        assert e <= e_prev + 1e-14 * abs(e_prev)
        e_prev = e


# --- line solver against LAPACK ------------------------------------------------------------------

@pytest.mark.parametrize("n,off,diag", [(1, -1.0, 4.0), (2, -3.0, 10.0), (17, -100.0, 204.0),
                                        (256, -100.0, 204.0), (64, -1.0, 4.0001)])
def test_thomas_vs_banded(n, off, diag):
    rng = np.random.default_rng(n)
    rhs = rng.uniform(-1, 1, n)
    ab = np.zeros((3, n))
    ab[0, 1:] = off
    ab[1, :] = diag
    ab[2, :-1] = off
    ref = scipy.linalg.solve_banded((1, 1), ab, rhs)
    got = oracle.tridiag_solve(off, diag, rhs)
    assert relerr(got, ref) < 1e-13


# --- lexicographic GS: serial loop == anti-diagonal form, bit for bit ---------------------------

@pytest.mark.parametrize("axis", [0, 1, 2])
def test_lex_antidiagonal_bitwise(axis):
    p = small_patch(9, 7, 5, seed=17, eps=EPS)
    a = oracle.line_sweeps(p.u0, p.f, p.eps, p.h, axis, oracle.LEX_GS, 1.0, 3, lex_form=0)
    b = oracle.line_sweeps(p.u0, p.f, p.eps, p.h, axis, oracle.LEX_GS, 1.0, 3, lex_form=1)
    assert np.array_equal(a, b)


# --- adjoint of K Jacobi line sweeps --------------------------------------------------------------

def _loss(u0, f, eps, h, axis, omega, K, tgt):
    uK = oracle.line_sweeps(u0, f, eps, h, axis, oracle.JACOBI, omega, K)
    d = uK[1:-1, 1:-1, 1:-1] - tgt
    return float(np.sum(d * d)), uK


def _adjoint_case(axis, seed=23):
    p = small_patch(5, 4, 6, seed=seed, eps=(1.3, 0.7, 2.1))
    rng = np.random.default_rng(seed + 100)
    tgt = rng.uniform(-1, 1, p.f.shape)
    return p, tgt


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_adjoint_vs_finite_differences(axis):
    p, tgt = _adjoint_case(axis)
    omega, K = 0.8, 4
    L0, uK = _loss(p.u0, p.f, p.eps, p.h, axis, omega, K, tgt)
    gK = np.zeros_like(p.u0)
    gK[1:-1, 1:-1, 1:-1] = 2 * (uK[1:-1, 1:-1, 1:-1] - tgt)
    g_u0, g_f, g_eps = oracle.line_jacobi_adjoint(p.u0, p.f, p.eps, p.h, axis, omega, K, gK)
    hstep = 1e-6
    for b in range(3):
        ep = list(p.eps); em = list(p.eps)
        ep[b] += hstep; em[b] -= hstep
        fd = (_loss(p.u0, p.f, ep, p.h, axis, omega, K, tgt)[0]
              - _loss(p.u0, p.f, em, p.h, axis, omega, K, tgt)[0]) / (2 * hstep)
        assert g_eps[b] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    rng = np.random.default_rng(5)
    # directional derivatives in f, interior u0 and face ghosts
    df = rng.standard_normal(p.f.shape); df /= np.linalg.norm(df)
    fd = (_loss(p.u0, p.f + hstep * df, p.eps, p.h, axis, omega, K, tgt)[0]
          - _loss(p.u0, p.f - hstep * df, p.eps, p.h, axis, omega, K, tgt)[0]) / (2 * hstep)
    assert np.sum(g_f * df) == pytest.approx(fd, rel=1e-6, abs=1e-9)
    du = np.zeros_like(p.u0)
    du[1:-1, 1:-1, 1:-1] = rng.standard_normal(p.f.shape)
    gmask = ~np.pad(np.ones(p.f.shape, bool), 1, constant_values=False)
    du[gmask] = rng.standard_normal(int(gmask.sum()))
    du /= np.linalg.norm(du)
    fd = (_loss(p.u0 + hstep * du, p.f, p.eps, p.h, axis, omega, K, tgt)[0]
          - _loss(p.u0 - hstep * du, p.f, p.eps, p.h, axis, omega, K, tgt)[0]) / (2 * hstep)
    assert np.sum(g_u0 * du) == pytest.approx(fd, rel=1e-6, abs=1e-9)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_adjoint_vs_forward_tangent(axis):
    p, tgt = _adjoint_case(axis, seed=29)
    omega, K = 0.8, 5
    _, uK = _loss(p.u0, p.f, p.eps, p.h, axis, omega, K, tgt)
    gK = np.zeros_like(p.u0)
    gK[1:-1, 1:-1, 1:-1] = 2 * (uK[1:-1, 1:-1, 1:-1] - tgt)
    _, _, g_eps = oracle.line_jacobi_adjoint(p.u0, p.f, p.eps, p.h, axis, omega, K, gK)
    t_eps = oracle.line_jacobi_eps_tangent(p.u0, p.f, p.eps, p.h, axis, omega, K, gK)
    assert relerr(g_eps, t_eps) < 1e-10


@pytest.mark.parametrize("axis", [0, 2])
def test_euler_identity(axis):
    """Scaling eps and f together (ghosts fixed) leaves every iterate unchanged,
    so <eps, dL/deps> + <f, dL/df> = 0."""
    p, tgt = _adjoint_case(axis, seed=31)
    omega, K = 0.8, 4
    _, uK = _loss(p.u0, p.f, p.eps, p.h, axis, omega, K, tgt)
    gK = np.zeros_like(p.u0)
    gK[1:-1, 1:-1, 1:-1] = 2 * (uK[1:-1, 1:-1, 1:-1] - tgt)
    _, g_f, g_eps = oracle.line_jacobi_adjoint(p.u0, p.f, p.eps, p.h, axis, omega, K, gK)
    t1 = float(np.dot(p.eps, g_eps))
    t2 = float(np.sum(p.f * g_f))
    assert abs(t1 + t2) < 1e-10 * max(abs(t1), abs(t2))


def test_adjoint_dot_product():
    """u0 -> u_K is affine; its linear part J (f = 0, zero ghosts) satisfies
    <J v, w> = <v, J^T w> with J^T w from the adjoint (gK = w)."""
    nx, ny, nz, axis, omega, K = 5, 4, 6, 1, 0.8, 3
    rng = np.random.default_rng(3)
    v = np.zeros((nz + 2, ny + 2, nx + 2)); v[1:-1, 1:-1, 1:-1] = rng.standard_normal((nz, ny, nx))
    w = np.zeros_like(v); w[1:-1, 1:-1, 1:-1] = rng.standard_normal((nz, ny, nx))
    f0 = np.zeros((nz, ny, nx))
    Jv = oracle.line_sweeps(v, f0, EPS, 0.2, axis, oracle.JACOBI, omega, K)
    JTw, _, _ = oracle.line_jacobi_adjoint(v, f0, EPS, 0.2, axis, omega, K, w)
    lhs = float(np.sum(Jv[1:-1, 1:-1, 1:-1] * w[1:-1, 1:-1, 1:-1]))
    rhs = float(np.sum(v[1:-1, 1:-1, 1:-1] * JTw[1:-1, 1:-1, 1:-1]))
    assert lhs == pytest.approx(rhs, rel=1e-12)


# --- the partial-update helpers (checkers of single planes / lines of a large sweep) ----------

@pytest.mark.parametrize("normal", [0, 1, 2])
def test_plane_update_some_all_planes_is_one_jacobi_sweep(normal):
    """Updating every plane from the same u is one plane-Jacobi sweep (bitwise,
    both use the same per-plane arithmetic); a subset changes only its planes,
    each exactly as in the full sweep, and is pinned to the dense brute force."""
    p = small_patch(9, 7, 6, seed=33 + normal, eps=EPS)
    nc = p.dims[normal]
    full = oracle.plane_sweeps(p.u0, p.f, p.eps, p.h, normal, oracle.JACOBI, 0.8, 1)
    every = oracle.plane_update_some(p.u0, p.f, p.eps, p.h, normal, 0.8, list(range(nc)))
    assert np.array_equal(every, full)
    some = [1, nc - 1]
    part = oracle.plane_update_some(p.u0, p.f, p.eps, p.h, normal, 0.8, some)
    idx = lambda s: tuple(slice(s + 1, s + 2) if ax == normal else slice(None) for ax in (2, 1, 0))
    for s in range(nc):
        sl = idx(s)
        if s in some:
            assert np.array_equal(part[sl], full[sl]), s
        else:
            assert np.array_equal(part[sl], p.u0[sl]), s
    dense = brute.sweeps(p.u0, p.f, p.eps, p.h, "plane", normal, "jacobi", 0.8, 1)
    assert relerr(every, dense) < 1e-14


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_line_update_some_reproduces_every_scheme(axis):
    """Line updates of listed lines from a given u: all lines at once is a
    Jacobi sweep; colour 0 then colour 1 is the two-colour GS sweep; one line at
    a time in lexicographic order is lexicographic GS (each bitwise against the
    oracle's sweeps, and Jacobi against the dense brute force)."""
    p = small_patch(6, 5, 7, seed=41 + axis, eps=EPS)
    n = p.dims
    free = [a for a in (0, 1, 2) if a != axis]
    npq = (n[free[0]], n[free[1]])
    lines = [(a, b) for b in range(npq[1]) for a in range(npq[0])]   # lower free axis fastest
    jac = oracle.line_update_some(p.u0, p.f, p.eps, p.h, axis, 0.8, lines)
    assert np.array_equal(jac, oracle.line_sweeps(p.u0, p.f, p.eps, p.h, axis, oracle.JACOBI, 0.8, 1))
    assert relerr(jac, brute.sweeps(p.u0, p.f, p.eps, p.h, "line", axis, "jacobi", 0.8, 1)) < 1e-14
    u = p.u0.copy()
    for c in (0, 1):
        u = oracle.line_update_some(u, p.f, p.eps, p.h, axis, 1.0, [l for l in lines if (l[0] + l[1]) % 2 == c])
    assert np.array_equal(u, oracle.line_sweeps(p.u0, p.f, p.eps, p.h, axis, oracle.COLORED_GS, 1.0, 1))
    u = p.u0.copy()
    for l in lines:
        u = oracle.line_update_some(u, p.f, p.eps, p.h, axis, 1.0, [l])
    assert np.array_equal(u, oracle.line_sweeps(p.u0, p.f, p.eps, p.h, axis, oracle.LEX_GS, 1.0, 1))
    with pytest.raises(ValueError):
        oracle.line_update_some(p.u0, p.f, p.eps, p.h, axis, 1.0, [(npq[0], 0)])
