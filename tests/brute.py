"""Dense brute force for tiny grids: assemble the interior matrix A and the
block splitting M as dense matrices and run sweeps with numpy.linalg.solve.

This pins the oracle to the paper's definitions without sharing any of its
code: the splitting A = M - N and the residual-correction form
u <- u + M^{-1} r (eq. blockiteration1 / blockiteration2), with M block
diagonal (Jacobi, scaled by 1/omega for damping) or block lower triangular in
the visiting order (block Gauss-Seidel / SOR, eq. sm:blockm).
"""
from __future__ import annotations

import numpy as np


def interior_index(nx, ny, nz):
    idx = np.arange(nx * ny * nz).reshape(nz, ny, nx)
    return idx


def assemble(nx, ny, nz, eps, bc=0):
    """Dense A_int (m x m) for interior cells, C order [k][j][i].  bc: faces
    with an extrapolated ghost (-(the boundary cell's value); bit 2a low, bit
    2a+1 high face of axis a), whose stencil term lands on the diagonal."""
    m = nx * ny * nz
    A = np.zeros((m, m))
    idx = interior_index(nx, ny, nz)
    ex, ey, ez = eps
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = idx[k, j, i]
                A[c, c] = 2 * (ex + ey + ez)
                for (ax, di, dj, dk, e) in ((0, 1, 0, 0, ex), (0, -1, 0, 0, ex), (1, 0, 1, 0, ey), (1, 0, -1, 0, ey),
                                            (2, 0, 0, 1, ez), (2, 0, 0, -1, ez)):
                    ii, jj, kk = i + di, j + dj, k + dk
                    if 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz:
                        A[c, idx[kk, jj, ii]] = -e
                    else:
                        side = 0 if (di + dj + dk) < 0 else 1
                        if bc >> (2 * ax + side) & 1:
                            A[c, c] += e      # ghost = -u_c: -e * (-u_c)
    return A


def ghost_rhs(upad, eps, bc=0):
    """B g: the ghost terms of the stencil moved to the right-hand side (faces
    in bc carry none: their ghost is part of the operator)."""
    nz, ny, nx = (s - 2 for s in upad.shape)
    ex, ey, ez = eps
    g = np.zeros((nz, ny, nx))
    if not bc & 1:
        g[:, :, 0] += ex * upad[1:-1, 1:-1, 0]
    if not bc & 2:
        g[:, :, -1] += ex * upad[1:-1, 1:-1, -1]
    if not bc & 4:
        g[:, 0, :] += ey * upad[1:-1, 0, 1:-1]
    if not bc & 8:
        g[:, -1, :] += ey * upad[1:-1, -1, 1:-1]
    if not bc & 16:
        g[0, :, :] += ez * upad[0, 1:-1, 1:-1]
    if not bc & 32:
        g[-1, :, :] += ez * upad[-1, 1:-1, 1:-1]
    return g.reshape(-1)


def block_ids(nx, ny, nz, kind, axis):
    """(block id per cell, visiting order key per block id, colour per block id).

    Lines along `axis` are named by their free indices (p, q), p the lower
    remaining axis; lexicographic order is p fastest.  Planes with normal
    `axis` are named by their index s.  Cube blocks: `axis` is the block
    shape (bx, by, bz)."""
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    coords = {0: i, 1: j, 2: k}
    dims = {0: nx, 1: ny, 2: nz}
    if kind == "cube":
        # geometric blocks of axis = (bx, by, bz) cells from the origin, shorter
        # at the upper ends; lexicographic order bi fastest; colour bi+bj+bk
        bx, by, bz = axis
        mi, mj = -(-nx // bx), -(-ny // by)
        mk = -(-nz // bz)
        bid = ((k // bz) * mj * mi + (j // by) * mi + i // bx).reshape(-1)
        ids = np.arange(mi * mj * mk)
        order = ids
        colour = (ids % mi + (ids // mi) % mj + ids // (mi * mj)) % 2
        return bid, order, colour
    if kind == "line":
        others = [a for a in (0, 1, 2) if a != axis]
        p, q = coords[others[0]], coords[others[1]]
        bid = (q * dims[others[0]] + p).reshape(-1)
        nb = dims[others[0]] * dims[others[1]]
        pp = np.arange(nb) % dims[others[0]]
        qq = np.arange(nb) // dims[others[0]]
        order = np.arange(nb)
        colour = (pp + qq) % 2
    else:
        s = coords[axis]
        bid = s.reshape(-1)
        nb = dims[axis]
        order = np.arange(nb)
        colour = np.arange(nb) % 2
    return bid, order, colour


def splitting(A, bid, order, colour, scheme, omega):
    """M for the scheme: 'jacobi' -> D/omega, 'lex' -> D/omega + L(order),
    'colored' -> D/omega + L(colour 0 before colour 1)."""
    same = bid[:, None] == bid[None, :]
    D = np.where(same, A, 0.0)
    if scheme == "jacobi":
        return D / omega
    if scheme == "lex":
        key = order[bid]
    elif scheme == "colored":
        key = colour[bid]
    else:
        raise ValueError(scheme)
    L = np.where(key[:, None] > key[None, :], A, 0.0)
    return D / omega + L


def sweeps(upad, f, eps, h, kind, axis, scheme, omega, nsweeps, bc=0):
    nz, ny, nx = f.shape
    A = assemble(nx, ny, nz, eps, bc)
    bid, order, colour = block_ids(nx, ny, nz, kind, axis)
    M = splitting(A, bid, order, colour, scheme, omega)
    b = h * h * f.reshape(-1) + ghost_rhs(upad, eps, bc)
    x = upad[1:-1, 1:-1, 1:-1].reshape(-1).copy()
    for _ in range(nsweeps):
        r = b - A @ x
        x = x + np.linalg.solve(M, r)
    out = upad.copy()
    out[1:-1, 1:-1, 1:-1] = x.reshape(nz, ny, nx)
    return out


def iteration_matrix(nx, ny, nz, eps, kind, axis, scheme, omega):
    A = assemble(nx, ny, nz, eps)
    bid, order, colour = block_ids(nx, ny, nz, kind, axis)
    M = splitting(A, bid, order, colour, scheme, omega)
    return np.eye(A.shape[0]) - np.linalg.solve(M, A), A, M
