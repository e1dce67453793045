"""Seeded synthetic inputs for block relaxation, shared by the tests, the
benchmark and the smoke check.

This module holds NO arithmetic of the smoother: it only draws random numbers
and places them in the storage layout (u padded with one ghost layer, f
unpadded, x fastest; section 2.1, index spaces).  Everything is NumPy
``Generator(PCG64(seed))`` and the draw order is fixed:

  single patch:  f (interior, C order [k][j][i]), then u0 interior, then the
                 ghost shell (every ghost position of the padded array, in C
                 order), each only when that field is random;
  patch set:     dims = choice({16,24,32,48,64}, (P,3)) (columns nx,ny,nz),
                 eps = 10**uniform(0, 2, (P,3)), then per patch f, u, ghosts.

The paper's workloads are synthetic (random initial guess, section 3); no
dataset exists or is needed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

EDGE_CHOICES = (16, 24, 32, 48, 64)


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def ghost_mask(nx: int, ny: int, nz: int) -> np.ndarray:
    m = np.ones((nz + 2, ny + 2, nx + 2), dtype=bool)
    m[1:-1, 1:-1, 1:-1] = False
    return m


@dataclass
class Patch:
    """One patch: padded u0 (nz+2, ny+2, nx+2), unpadded f (nz, ny, nx)."""
    u0: np.ndarray
    f: np.ndarray
    eps: tuple
    h: float
    extra: dict = field(default_factory=dict)

    @property
    def dims(self):
        nz, ny, nx = self.f.shape
        return nx, ny, nz


def make_patch(nx, ny, nz, eps, h, seed, f="uniform", u0="uniform", ghosts="zero") -> Patch:
    """Draw one patch.  Each of f/u0/ghosts is 'uniform' (U[-1,1]) or 'zero'."""
    rng = rng_for(seed)
    ff = rng.uniform(-1.0, 1.0, size=(nz, ny, nx)) if f == "uniform" else np.zeros((nz, ny, nx))
    u = np.zeros((nz + 2, ny + 2, nx + 2))
    if u0 == "uniform":
        u[1:-1, 1:-1, 1:-1] = rng.uniform(-1.0, 1.0, size=(nz, ny, nx))
    if ghosts == "uniform":
        gm = ghost_mask(nx, ny, nz)
        u[gm] = rng.uniform(-1.0, 1.0, size=int(gm.sum()))
    return Patch(u0=u, f=np.ascontiguousarray(ff), eps=tuple(float(e) for e in eps), h=float(h))


# --- the five workloads -------------------------------------------------------

def c1_patch() -> Patch:
    """32^3, eps (1,1,1), h 1/32, zero ghosts, f ~ U[-1,1], u0 = 0 (seed 1)."""
    return make_patch(32, 32, 32, (1.0, 1.0, 1.0), 1.0 / 32, seed=1, f="uniform", u0="zero")


def c2_patch(n: int = 256) -> Patch:
    """256^3, eps (1,1,100), h 1/256, zero ghosts, f, u0 ~ U[-1,1] (seed 2)."""
    return make_patch(n, n, n, (1.0, 1.0, 100.0), 1.0 / n, seed=2, f="uniform", u0="uniform")


def c3_patch(n: int = 512) -> Patch:
    """512^3, eps (1,100,100), h 1/512, zero ghosts, f, u0 ~ U[-1,1] (seed 3)."""
    return make_patch(n, n, n, (1.0, 100.0, 100.0), 1.0 / n, seed=3, f="uniform", u0="uniform")


def c5_patch(n: int = 128):
    """128^3, eps init (1,1,10), h 1/128, zero ghosts, f ~ U[-1,1], u0 = 0 (seed 5),
    and a smooth target: sum of 8 products of sines with integer frequencies in
    {1..4} and amplitudes U[-1,1], sampled at cell centres (i+1/2)h."""
    rng = rng_for(5)
    f = rng.uniform(-1.0, 1.0, size=(n, n, n))
    u0 = np.zeros((n + 2, n + 2, n + 2))
    freqs = rng.integers(1, 5, size=(8, 3))
    amps = rng.uniform(-1.0, 1.0, size=8)
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    tgt = np.zeros((n, n, n))
    for m in range(8):
        p, q, s = (int(v) for v in freqs[m])
        tgt += amps[m] * (np.sin(np.pi * s * x)[:, None, None] * np.sin(np.pi * q * x)[None, :, None]
                          * np.sin(np.pi * p * x)[None, None, :])
    return Patch(u0=u0, f=f, eps=(1.0, 1.0, 10.0), h=h, extra={"target": tgt})


@dataclass
class PatchSet:
    dims: np.ndarray     # (P,3) int32: nx, ny, nz
    eps: np.ndarray      # (P,3) float64
    h: np.ndarray        # (P,) float64
    u0: list             # P padded arrays
    f: list              # P unpadded arrays

    @property
    def npatch(self):
        return int(self.dims.shape[0])

    def cells(self) -> int:
        return int(np.prod(self.dims.astype(np.int64), axis=1).sum())


def c4_patchset(npatch: int = 3000, seed: int = 4, edges=EDGE_CHOICES) -> PatchSet:
    """Uneven patches: edges from `edges` per axis, eps = 10^U[0,2] per axis,
    h = 1/max(n), u, f and ghosts ~ U[-1,1]."""
    rng = rng_for(seed)
    dims = rng.choice(np.asarray(edges, dtype=np.int64), size=(npatch, 3)).astype(np.int32)
    eps = 10.0 ** rng.uniform(0.0, 2.0, size=(npatch, 3))
    h = 1.0 / dims.max(axis=1).astype(np.float64)
    us, fs = [], []
    for p in range(npatch):
        nx, ny, nz = (int(v) for v in dims[p])
        f = rng.uniform(-1.0, 1.0, size=(nz, ny, nx))
        u = np.empty((nz + 2, ny + 2, nx + 2))
        u[1:-1, 1:-1, 1:-1] = rng.uniform(-1.0, 1.0, size=(nz, ny, nx))
        gm = ghost_mask(nx, ny, nz)
        u[gm] = rng.uniform(-1.0, 1.0, size=int(gm.sum()))
        us.append(u)
        fs.append(f)
    return PatchSet(dims=dims, eps=eps, h=h, u0=us, f=fs)


def uniform_patchset(npatch: int = 64, n: int = 64, seed: int = 6, eps=(1.0, 1.0, 1.0)) -> PatchSet:
    """npatch equal patches of n^3 cells (the block-size study's 64 patches of
    64^3): eps as given, h = 1/n, then per patch f, u, ghosts ~ U[-1,1]."""
    rng = rng_for(seed)
    dims = np.full((npatch, 3), n, dtype=np.int32)
    epsa = np.tile(np.asarray(eps, dtype=np.float64), (npatch, 1))
    h = np.full(npatch, 1.0 / n)
    gm = ghost_mask(n, n, n)
    us, fs = [], []
    for _ in range(npatch):
        f = rng.uniform(-1.0, 1.0, size=(n, n, n))
        u = np.empty((n + 2, n + 2, n + 2))
        u[1:-1, 1:-1, 1:-1] = rng.uniform(-1.0, 1.0, size=(n, n, n))
        u[gm] = rng.uniform(-1.0, 1.0, size=int(gm.sum()))
        us.append(u)
        fs.append(f)
    return PatchSet(dims=dims, eps=epsa, h=h, u0=us, f=fs)


def small_patch(nx, ny, nz, seed, eps=None, ghosts="uniform", u0="uniform", f="uniform") -> Patch:
    """A small random test patch; eps defaults to distinct per-axis weights."""
    if eps is None:
        eps = (1.0, 3.0, 7.0)
    return make_patch(nx, ny, nz, eps, 1.0 / max(nx, ny, nz), seed, f=f, u0=u0, ghosts=ghosts)


# --- patch sets with adjacency (ghost exchange between patches) ----------------

@dataclass
class LinkedSet:
    """Patches that tile a box face to face.  links: (a, axis, b) with b on a's
    high side along axis; offsets: (x0, y0, z0) of each patch in the box."""
    dims: list
    eps: list
    h: list
    u0: list
    f: list
    links: list
    offsets: list

    @property
    def npatch(self):
        return len(self.dims)

    def cells(self) -> int:
        return int(sum(nx * ny * nz for nx, ny, nz in self.dims))


def split_patch(patch: Patch, cuts) -> LinkedSet:
    """Cut one patch into a grid of sub-patches at the cell positions
    cuts = (xcuts, ycuts, zcuts) (interior boundaries along each axis).  Each
    sub-patch's u holds the global array's values on its interior and face
    ghosts (so the ghosts are already consistent), f its slice of f."""
    nx, ny, nz = patch.dims
    edges = [[0] + sorted(c) + [n] for c, n in zip(cuts, (nx, ny, nz))]
    counts = [len(e) - 1 for e in edges]
    index = {}
    dims, us, fs, offs = [], [], [], []
    for c in range(counts[2]):
        for b in range(counts[1]):
            for a in range(counts[0]):
                x0, x1 = edges[0][a], edges[0][a + 1]
                y0, y1 = edges[1][b], edges[1][b + 1]
                z0, z1 = edges[2][c], edges[2][c + 1]
                index[(a, b, c)] = len(dims)
                dims.append((x1 - x0, y1 - y0, z1 - z0))
                us.append(np.ascontiguousarray(patch.u0[z0:z1 + 2, y0:y1 + 2, x0:x1 + 2]))
                fs.append(np.ascontiguousarray(patch.f[z0:z1, y0:y1, x0:x1]))
                offs.append((x0, y0, z0))
    links = []
    for (a, b, c), p in index.items():
        for axis, nb in ((0, (a + 1, b, c)), (1, (a, b + 1, c)), (2, (a, b, c + 1))):
            if nb in index:
                links.append((p, axis, index[nb]))
    n = len(dims)
    return LinkedSet(dims=dims, eps=[patch.eps] * n, h=[patch.h] * n, u0=us, f=fs, links=links, offsets=offs)


def c4_adjacent_patchset(grid=(14, 14, 15), seed=4, edges=EDGE_CHOICES) -> LinkedSet:
    """An adjacent version of the uneven AMR set: a grid of patches that tile a
    box face to face (14 x 14 x 15 = 2940 patches by default), the edge of
    every slab of patches drawn from `edges` (so faces always match), eps =
    10^U[0,2] per axis and patch, h = 1/64, u, f and the box's outer ghosts ~
    U[-1,1]; the ghosts between patches start from the neighbours' values."""
    rng = rng_for(seed)
    ex = [int(v) for v in rng.choice(np.asarray(edges), size=grid[0])]
    ey = [int(v) for v in rng.choice(np.asarray(edges), size=grid[1])]
    ez = [int(v) for v in rng.choice(np.asarray(edges), size=grid[2])]
    X, Y, Z = sum(ex), sum(ey), sum(ez)
    npatch = grid[0] * grid[1] * grid[2]
    eps = 10.0 ** rng.uniform(0.0, 2.0, size=(npatch, 3))
    f = rng.uniform(-1.0, 1.0, size=(Z, Y, X))
    u = np.empty((Z + 2, Y + 2, X + 2))
    u[1:-1, 1:-1, 1:-1] = rng.uniform(-1.0, 1.0, size=(Z, Y, X))
    gm = ghost_mask(X, Y, Z)
    u[gm] = rng.uniform(-1.0, 1.0, size=int(gm.sum()))
    whole = Patch(u0=u, f=f, eps=(1.0, 1.0, 1.0), h=1.0 / 64)
    cuts = [list(np.cumsum(e)[:-1]) for e in (ex, ey, ez)]
    s = split_patch(whole, cuts)
    s.eps = [tuple(float(v) for v in e) for e in eps]
    return s
