"""The oracle: plain FP64 CPU block relaxation, written from the paper.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The product
path (``paper_1208_1975_amd``) never imports it, and the two share no code.

The arithmetic lives in ``bso.c`` (plain C, ``-O2 -ffp-contract=off``,
OpenMP only over independent blocks).  This module builds it with ``gcc`` and
wraps it with ctypes; it adds no arithmetic of its own.

Layout (section 2.1, index spaces): ``u`` is padded with one ghost layer,
shape ``(nz+2, ny+2, nx+2)``; ``f`` is unpadded, shape ``(nz, ny, nx)``;
x is the fastest axis.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bso.c")
_LIB = os.path.join(_HERE, "libbso.so")

JACOBI, LEX_GS, COLORED_GS = 0, 1, 2

_lib = None


def build(force: bool = True) -> str:
    """Compile bso.c into libbso.so next to it (plain gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    D, I, P = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
    lib.bso_residual.argtypes = [I, I, I, P, D, P, P, P]
    lib.bso_residual.restype = D
    lib.bso_residual_bc.argtypes = [I, I, I, P, D, P, P, P, I]
    lib.bso_residual_bc.restype = D
    lib.bso_line_sweeps_bc.argtypes = [I, I, I, P, D, I, I, D, I, I, P, P, I]
    lib.bso_line_sweeps_bc.restype = I
    lib.bso_plane_sweeps_bc.argtypes = [I, I, I, P, D, I, I, D, I, P, P, I]
    lib.bso_plane_sweeps_bc.restype = I
    lib.bso_cube_sweeps_bc.argtypes = [I, I, I, P, D, I, I, I, I, D, I, P, P, I]
    lib.bso_cube_sweeps_bc.restype = I
    lib.bso_tridiag_solve.argtypes = [I, D, D, P, P]
    lib.bso_tridiag_solve.restype = None
    lib.bso_line_sweeps.argtypes = [I, I, I, P, D, I, I, D, I, I, P, P]
    lib.bso_line_sweeps.restype = I
    lib.bso_plane_sweeps.argtypes = [I, I, I, P, D, I, I, D, I, P, P]
    lib.bso_plane_sweeps.restype = I
    lib.bso_plane_update_some.argtypes = [I, I, I, P, D, I, D, I, P, P, P, P]
    lib.bso_plane_update_some.restype = I
    lib.bso_line_update_some.argtypes = [I, I, I, P, D, I, D, I, P, P, P, P]
    lib.bso_line_update_some.restype = I
    lib.bso_line_jacobi_adjoint.argtypes = [I, I, I, P, D, I, D, I, P, P, P, P, P, P]
    lib.bso_line_jacobi_adjoint.restype = I
    lib.bso_line_jacobi_eps_tangent.argtypes = [I, I, I, P, D, I, D, I, P, P, P, P]
    lib.bso_line_jacobi_eps_tangent.restype = I
    lib.bso_block_adjoint.argtypes = [I, I, I, P, D, I, I, I, D, I, P, P, P, P, P, P]
    lib.bso_block_adjoint.restype = I
    lib.bso_cube_sweeps.argtypes = [I, I, I, P, D, I, I, I, I, D, I, P, P]
    lib.bso_cube_sweeps.restype = I
    lib.bso_exchange_ghosts.argtypes = [I, P, P, I, P]
    lib.bso_exchange_ghosts.restype = I
    lib.bso_restrict.argtypes = [I, I, I, P, D, P]
    lib.bso_restrict.restype = I
    lib.bso_prolong_add_bc.argtypes = [I, I, I, P, P, I]
    lib.bso_prolong_add_bc.restype = I
    lib.bso_set_threads.argtypes = [I]
    lib.bso_set_threads.restype = None
    lib.bso_get_threads.argtypes = []
    lib.bso_get_threads.restype = I
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _dims_of(u):
    nz, ny, nx = (s - 2 for s in u.shape)
    return nx, ny, nz


def _check(u, f=None):
    assert u.dtype == np.float64 and u.flags.c_contiguous and u.ndim == 3
    nx, ny, nz = _dims_of(u)
    if f is not None:
        assert f.dtype == np.float64 and f.flags.c_contiguous and f.shape == (nz, ny, nx)
    return nx, ny, nz


def _eps(eps):
    return np.ascontiguousarray(np.asarray(eps, dtype=np.float64).reshape(3))


def set_threads(n: int) -> None:
    _load().bso_set_threads(int(n))


def get_threads() -> int:
    return int(_load().bso_get_threads())


# Boundary reading: bc is a 6-bit mask of faces with extrapolated Dirichlet
# conditions (bit 2a: low face of axis a, bit 2a+1: high face), where the
# ghost takes -(the adjacent interior value) and folds into the operator
# (section 1.1: boundary conditions extrapolated into the ghost layer); other
# faces read their ghosts as data.  bc = 0 everywhere by default.
BC_ALL = 63


def residual(u, f, eps, h, want_r=True, bc=0):
    """(r, sum r^2): r = h^2 f - A_eps u over interior cells (eq. stencil3d7)."""
    lib = _load()
    nx, ny, nz = _check(u, f)
    e = _eps(eps)
    r = np.empty((nz, ny, nx)) if want_r else None
    s = lib.bso_residual_bc(nx, ny, nz, _p(e), float(h), _p(u), _p(f), _p(r), int(bc))
    return r, s


def tridiag_solve(off, diag, rhs):
    """Textbook Thomas solve of tridiag(off, diag, off) x = rhs."""
    lib = _load()
    rhs = np.ascontiguousarray(rhs, dtype=np.float64)
    x = np.empty_like(rhs)
    lib.bso_tridiag_solve(rhs.size, float(off), float(diag), _p(rhs), _p(x))
    return x


def line_sweeps(u, f, eps, h, axis, scheme, omega, nsweeps, lex_form=0, bc=0):
    """Return u after nsweeps line-block sweeps (u is not modified)."""
    lib = _load()
    nx, ny, nz = _check(u, f)
    out = u.copy()
    rc = lib.bso_line_sweeps_bc(nx, ny, nz, _p(_eps(eps)), float(h), int(axis), int(scheme),
                                float(omega), int(nsweeps), int(lex_form), _p(out), _p(f), int(bc))
    if rc:
        raise ValueError("bso_line_sweeps failed (%d)" % rc)
    return out


def plane_sweeps(u, f, eps, h, normal, scheme, omega, nsweeps, bc=0):
    """Return u after nsweeps plane-block sweeps (u is not modified)."""
    lib = _load()
    nx, ny, nz = _check(u, f)
    out = u.copy()
    rc = lib.bso_plane_sweeps_bc(nx, ny, nz, _p(_eps(eps)), float(h), int(normal), int(scheme),
                                 float(omega), int(nsweeps), _p(out), _p(f), int(bc))
    if rc:
        raise ValueError("bso_plane_sweeps failed (%d)" % rc)
    return out


def cube_sweeps(u, f, eps, h, block, scheme, omega, nsweeps, bc=0):
    """Return u after nsweeps sweeps over geometric blocks of block = (bx, by, bz)
    cells (shorter last blocks where an edge does not divide the patch; each
    block solved exactly).  u is not modified."""
    lib = _load()
    nx, ny, nz = _check(u, f)
    bx, by, bz = (int(b) for b in block)
    out = u.copy()
    rc = lib.bso_cube_sweeps_bc(nx, ny, nz, _p(_eps(eps)), float(h), bx, by, bz, int(scheme),
                                float(omega), int(nsweeps), _p(out), _p(f), int(bc))
    if rc:
        raise ValueError("bso_cube_sweeps failed (%d)" % rc)
    return out


def plane_update_some(usrc, f, eps, h, normal, omega, planes, udst=None):
    """One Jacobi update of the listed planes from usrc; other cells copied from usrc."""
    lib = _load()
    nx, ny, nz = _check(usrc, f)
    out = usrc.copy() if udst is None else udst
    pl = np.ascontiguousarray(np.asarray(planes, dtype=np.int32))
    rc = lib.bso_plane_update_some(nx, ny, nz, _p(_eps(eps)), float(h), int(normal), float(omega),
                                   pl.size, _p(pl), _p(usrc), _p(out), _p(f))
    if rc:
        raise ValueError("bso_plane_update_some failed")
    return out


def line_update_some(usrc, f, eps, h, axis, omega, lines, udst=None):
    """One update of the listed lines (p, q) from usrc; other cells copied from usrc."""
    lib = _load()
    nx, ny, nz = _check(usrc, f)
    out = usrc.copy() if udst is None else udst
    pq = np.ascontiguousarray(np.asarray(lines, dtype=np.int32).reshape(-1, 2))
    rc = lib.bso_line_update_some(nx, ny, nz, _p(_eps(eps)), float(h), int(axis), float(omega),
                                  pq.shape[0], _p(pq), _p(usrc), _p(out), _p(f))
    if rc:
        raise ValueError("bso_line_update_some failed")
    return out


def line_jacobi_adjoint(u0, f, eps, h, axis, omega, K, gK):
    """Reverse-mode gradients of K damped Jacobi line sweeps for dL/du_K = gK.

    Returns (g_u0 padded incl. face-ghost gradients, g_f unpadded, g_eps[3])."""
    lib = _load()
    nx, ny, nz = _check(u0, f)
    gK = np.ascontiguousarray(gK, dtype=np.float64)
    assert gK.shape == u0.shape
    g_u0 = np.zeros_like(u0)
    g_f = np.zeros_like(f)
    g_eps = np.zeros(3)
    rc = lib.bso_line_jacobi_adjoint(nx, ny, nz, _p(_eps(eps)), float(h), int(axis), float(omega),
                                     int(K), _p(u0), _p(f), _p(gK), _p(g_u0), _p(g_f), _p(g_eps))
    if rc:
        raise ValueError("bso_line_jacobi_adjoint failed")
    return g_u0, g_f, g_eps


def block_adjoint(u0, f, eps, h, kind, axis, scheme, omega, K, gK):
    """Reverse-mode gradients of K sweeps of line ('line', along axis) or plane
    ('plane', normal axis) blocks under JACOBI or COLORED_GS, every state
    stored.  Returns (g_u0 padded incl. face-ghost gradients, g_f, g_eps[3])."""
    lib = _load()
    nx, ny, nz = _check(u0, f)
    gK = np.ascontiguousarray(gK, dtype=np.float64)
    assert gK.shape == u0.shape
    k = {"line": 0, "plane": 1}[kind]
    g_u0 = np.zeros_like(u0)
    g_f = np.zeros_like(f)
    g_eps = np.zeros(3)
    rc = lib.bso_block_adjoint(nx, ny, nz, _p(_eps(eps)), float(h), k, int(axis), int(scheme), float(omega),
                               int(K), _p(u0), _p(f), _p(gK), _p(g_u0), _p(g_f), _p(g_eps))
    if rc:
        raise ValueError("bso_block_adjoint failed")
    return g_u0, g_f, g_eps


def line_jacobi_eps_tangent(u0, f, eps, h, axis, omega, K, gK):
    """Forward-mode dL/deps (3 values) for dL/du_K = gK."""
    lib = _load()
    nx, ny, nz = _check(u0, f)
    gK = np.ascontiguousarray(gK, dtype=np.float64)
    out = np.zeros(3)
    rc = lib.bso_line_jacobi_eps_tangent(nx, ny, nz, _p(_eps(eps)), float(h), int(axis),
                                         float(omega), int(K), _p(u0), _p(f), _p(gK), _p(out))
    if rc:
        raise ValueError("bso_line_jacobi_eps_tangent failed")
    return out


def exchange_ghosts(us, links):
    """Ghost exchange between adjacent patches: copies of the padded arrays
    us[p] in which, for every link (a, axis, b) (patch b on a's high side
    along axis, equal extents along the other axes), a's high ghost layer
    holds b's first interior layer and b's low ghost layer a's last one."""
    lib = _load()
    out = [np.array(u, dtype=np.float64, order="C", copy=True) for u in us]
    dims = np.ascontiguousarray([_dims_of(u) for u in out], dtype=np.int32).reshape(-1)
    ptrs = (ctypes.c_void_p * len(out))(*[u.ctypes.data for u in out])
    lk = np.ascontiguousarray(np.asarray(links, dtype=np.int32).reshape(-1, 3))
    rc = lib.bso_exchange_ghosts(len(out), _p(dims), ptrs, lk.shape[0], _p(lk))
    if rc:
        raise ValueError("bso_exchange_ghosts: bad link (%d)" % rc)
    return out


def patchset_sweeps(us, fs, eps, h, links, kind, arg, scheme, omega, nsweeps):
    """nsweeps smoothing steps of a patch set with adjacency: in every step
    each patch takes one sweep of `kind` ('line' along axis arg, 'plane' with
    normal arg, 'cube' with block arg) of `scheme` from its own ghosts, then
    the ghosts are exchanged (section 2).  eps and h are per patch."""
    fn = {"line": line_sweeps, "plane": plane_sweeps, "cube": cube_sweeps}[kind]
    out = [np.array(u, copy=True) for u in us]
    for _ in range(nsweeps):
        out = [fn(out[p], fs[p], eps[p], h[p], arg, scheme, omega, 1) for p in range(len(out))]
        out = exchange_ghosts(out, links)
    return out


# --- multigrid with the block smoothers (section 1: line and plane smoothers are
# components of robust geometric multigrid; section 5: multilevel use) ---------

def restrict(r, scale=1.0):
    """Cell-centred restriction: mean of each 2x2x2 group of fine values (f
    layout, even dims), times scale."""
    lib = _load()
    r = np.ascontiguousarray(r, dtype=np.float64)
    nz, ny, nx = r.shape
    out = np.empty((nz // 2, ny // 2, nx // 2))
    if lib.bso_restrict(nx, ny, nz, _p(r), float(scale), _p(out)):
        raise ValueError("restrict: fine dims must be even and >= 2")
    return out


def prolong_add(uc, uf, bc=0):
    """uf (padded, fine) + trilinear interpolation of the coarse padded uc
    (coarse ghosts are read at the edges, or extrapolated across the faces in
    bc); returns a new array."""
    lib = _load()
    out = np.array(uf, dtype=np.float64, copy=True)
    nx, ny, nz = _dims_of(out)
    uc = np.ascontiguousarray(uc, dtype=np.float64)
    assert uc.shape == (nz // 2 + 2, ny // 2 + 2, nx // 2 + 2)
    if lib.bso_prolong_add_bc(nx, ny, nz, _p(uc), _p(out), int(bc)):
        raise ValueError("prolong_add: fine dims must be even and >= 2")
    return out


def mg_levels(dims, max_levels=32):
    """Levels of the factor-2 hierarchy: halve while every edge is even and >= 2."""
    n = 1
    d = list(dims)
    while n < max_levels and all(v % 2 == 0 and v >= 2 for v in d):
        d = [v // 2 for v in d]
        n += 1
    return n


def vcycle(u, f, eps, h, kind, arg, scheme, omega, nu1, nu2, ncoarse, levels=None, bc=0, coarse_bc=None):
    """One V(nu1, nu2) cycle for A u = h^2 f on one patch: nu1 smoothing sweeps
    of `kind` ('line' along axis arg, 'plane' with normal arg) and `scheme`;
    the defect d = h^2 f - A u restricted to f_c = R(d / h^2) on the grid of
    cell width 2h (so that the coarse equation is A e_c = (2h)^2 f_c with zero
    ghosts and the same eps); the cycle applied to e_c = 0 there; u += P e_c;
    nu2 sweeps.  On the coarsest level: ncoarse sweeps.  bc is this level's
    boundary reading; the coarse levels take coarse_bc (default: bc), whose
    ghosts carry the error's homogeneous condition.  Returns the new u."""
    fn = {"line": line_sweeps, "plane": plane_sweeps}[kind]
    nx, ny, nz = _dims_of(u)
    if coarse_bc is None:
        coarse_bc = bc
    if levels is None:
        levels = mg_levels((nx, ny, nz))
    if levels <= 1:
        return fn(u, f, eps, h, arg, scheme, omega, ncoarse, bc=bc)
    u = fn(u, f, eps, h, arg, scheme, omega, nu1, bc=bc)
    d, _ = residual(u, f, eps, h, bc=bc)
    fc = restrict(d, 1.0 / (h * h))
    ec = vcycle(np.zeros((nz // 2 + 2, ny // 2 + 2, nx // 2 + 2)), fc, eps, 2.0 * h, kind, arg, scheme, omega,
                nu1, nu2, ncoarse, levels - 1, bc=coarse_bc, coarse_bc=coarse_bc)
    u = prolong_add(ec, u, bc=coarse_bc)
    return fn(u, f, eps, h, arg, scheme, omega, nu2, bc=bc)
