"""GPU parity of the chaotic GS kernel for y- and z-lines with omega = 1 that
holds two adjacent x-cells per lane (one of each colour) and solves the
colour-0 lines, then the colour-1 lines, in each tile of 128 x-cells by one
row.

With a persistent grid of one workgroup the tiles run one after another in
the dispatch order (rows in increasing order here), so the sweep is a fixed
sequence of line updates: per row, its colour-0 lines from the current
values, then its colour-1 lines.  The oracle reproduces that sequence line by
line (oracle.line_update_some) to 1e-12.  On the 256^3 workload the default
launch stays within the oracle's two-colour GS residual (the chaotic tests of
test_gpu_lines.py run this kernel too)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1208_1975_amd as bs
from conftest import relerr
from gpu_util import log, need_gpu
from workloads import small_patch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    need_gpu()
    oracle.set_threads(0)
    yield


def _dispatch_rows(no):
    """Row order of the one-patch chaotic dispatch with one-tile chunks: the
    rows split into 8 contiguous blocks (one per XCD), interleaved block by
    block -- what a single persistent workgroup walks through."""
    blocks = [list(range(no * x // 8, no * (x + 1) // 8)) for x in range(8)]
    order = []
    for j in range(max(len(b) for b in blocks)):
        for b in blocks:
            if j < len(b):
                order.append(b[j])
    return order


def _row_order_reference(p, axis, nsweeps):
    nx, ny, nz = p.dims
    no = nz if axis == 1 else ny
    u = p.u0.copy()
    for _ in range(nsweeps):
        for o in _dispatch_rows(no):
            for c in (0, 1):
                lines = [(i, o) for i in range(nx) if (i + o) % 2 == c]
                u = oracle.line_update_some(u, p.f, p.eps, p.h, axis, 1.0, lines)
    return u


@pytest.mark.parametrize("dims,axis,chunks", [((100, 8, 37), 2, 4), ((120, 16, 20), 2, 2), ((64, 9, 21), 1, 2),
                                              ((127, 33, 8), 2, 1), ((7, 40, 12), 1, 4), ((98, 12, 16), 2, 1),
                                              ((40, 8, 100), 2, 4), ((30, 150, 9), 1, 8)])   # 32-cell chunks
def test_pair_sequential_tiles_match_line_by_line_order(dims, axis, chunks):
    p = small_patch(*dims, seed=23, eps=(1.0, 2.0, 30.0))
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    nx = dims[0]
    no = dims[2] if axis == 1 else dims[1]
    assert nx <= 128 and ((nx + 63) // 64) * no >= 8   # one 128-cell tile per row, one-launch chaotic path
    ps.set_line_config(axis, "chaotic", chunks, 64, 1)   # one persistent workgroup: tiles in order
    ps.set_chaotic_chunk(1)
    cfg = ps.line_config(axis, "chaotic")
    assert cfg["grid"] == 1
    for nsweeps in (1, 2):
        log("pair %s axis %d chunks %d sweeps %d" % (dims, axis, chunks, nsweeps))
        u, f = ps.pack_u([p.u0]), ps.pack_f([p.f])
        ps.line_relax(axis, "chaotic", 1.0, nsweeps, u, f)
        torch.cuda.synchronize()
        ref = _row_order_reference(p, axis, nsweeps)
        assert relerr(ps.view_u(u, 0).cpu().numpy(), ref) < 1e-12
    ps.close()


def test_pair_and_single_line_forms_agree_in_rate():
    """256^3 anisotropic workload: the two chaotic forms reach residuals within
    a few percent of each other after 20 sweeps."""
    from workloads import c2_patch
    p = c2_patch(256)
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    f = ps.pack_f([p.f])
    n2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    res = {}
    for pair in (True, False):
        ps.set_pair(pair)
        u = ps.pack_u([p.u0])
        ps.line_relax(2, "chaotic", 1.0, 20, u, f)
        ps.residual(u, f, None, n2)
        res[pair] = float(n2.sqrt().item())
        del u
    log("chaotic residual after 20 sweeps: pair %.6e, single %.6e" % (res[True], res[False]))
    assert 0.9 < res[True] / res[False] < 1.1
    ps.close()
