"""Register x-lines (form 1): x-lines of up to 64 cells spread over the lanes
of a 16-lane row, four cells per lane, with the Thomas recurrences carried
across lanes by a log-step scan.  Parity against the oracle at 1e-12 for every
line length 1..64 (ragged lane counts, several lines per lane row, several
tiles), for every workgroup size, against the chunked kernel (form 0), and for
the in-tile two-colour (chaotic) form with more than one wavefront."""
import numpy as np
import pytest
import torch

import oracle
import paper_1208_1975_amd as bs
from conftest import relerr
from gpu_util import Single, log, need_gpu
from workloads import c4_patchset, small_patch

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _setup():
    need_gpu()
    oracle.set_threads(0)
    yield


def test_default_form_for_short_x_lines():
    """x-lines of up to 64 cells: Jacobi marches one-wavefront items along
    z, the Gauss-Seidel schemes take the register form; longer lines the
    chunked kernel."""
    p = small_patch(48, 5, 6, seed=3)
    s = Single(p)
    cfg = s.ps.line_config(0, "jacobi")
    assert cfg["form"] == 2 and cfg["chunks"] == 1 and cfg["chunk_len"] == 4, cfg
    for scheme in ("colored", "chaotic"):
        cfg = s.ps.line_config(0, scheme)
        assert cfg["form"] == 1 and cfg["chunk_len"] == 4, (scheme, cfg)
    q = small_patch(65, 3, 3, seed=3)
    assert Single(q).ps.line_config(0, "jacobi")["form"] == 0   # longer lines: chunked kernel


@pytest.mark.parametrize("nx", list(range(1, 65)))
def test_every_line_length(nx):
    """9 x 17 = 153 lines (three 64-line tiles, the last one ragged)."""
    p = small_patch(nx, 9, 17, seed=200 + nx, eps=(1.0 + 0.01 * nx, 3.0, 7.0))
    waves = (1, 2, 4)[nx % 3]
    for scheme, om, osch in (("jacobi", 0.8, oracle.JACOBI), ("colored", 1.0, oracle.COLORED_GS)):
        log("register x-lines nx=%d %s waves=%d" % (nx, scheme, waves))
        s = Single(p)
        s.ps.set_xline_config(scheme, waves=waves)
        s.line(0, scheme, om, 2)
        ref = oracle.line_sweeps(p.u0, p.f, p.eps, p.h, 0, osch, om, 2)
        got = s.u_np()
        assert relerr(got, ref) < TOL, (nx, scheme)
        gm = ~np.pad(np.ones(p.f.shape, bool), 1, constant_values=False)
        assert np.array_equal(got[gm], p.u0[gm])   # ghosts bit-unchanged


@pytest.mark.parametrize("waves", [1, 2, 4])
@pytest.mark.parametrize("dims", [(20, 6, 8), (9, 4, 16), (33, 1, 1), (64, 8, 8), (1, 8, 8), (5, 7, 9)])
def test_chaotic_single_tile_every_workgroup_size(dims, waves):
    """One tile holds all lines: chaotic GS is the two-colour block GS sweep;
    with several wavefronts the colour-1 lines read colour-0 values other
    wavefronts stored before the barrier."""
    p = small_patch(*dims, seed=71, eps=(1.0, 3.0, 7.0))
    for nsweeps in (1, 2):
        log("register x-lines chaotic %s waves=%d nsweeps=%d" % (dims, waves, nsweeps))
        s = Single(p)
        s.ps.set_xline_config("chaotic", waves=waves)
        s.line(0, "chaotic", 1.0, nsweeps)
        ref = oracle.line_sweeps(p.u0, p.f, p.eps, p.h, 0, oracle.COLORED_GS, 1.0, nsweeps)
        assert relerr(s.u_np(), ref) < TOL, (dims, waves, nsweeps)


def test_forms_agree_on_a_patch_set():
    """Uneven patches (edges 16..64): register form with 1, 2, 4 wavefronts,
    chunked form with 1 and 4 chunks, one and a persistent grid: all equal
    the oracle per patch."""
    s = c4_patchset(npatch=24, seed=17)
    ps = bs.PatchSet([tuple(d) for d in s.dims], [tuple(e) for e in s.eps], list(s.h))
    f = ps.pack_f(s.f)
    refs = {}
    for scheme, om, osch in (("jacobi", 0.8, oracle.JACOBI), ("colored", 1.0, oracle.COLORED_GS)):
        refs[scheme] = [oracle.line_sweeps(s.u0[p], s.f[p], tuple(s.eps[p]), s.h[p], 0, osch, om, 2)
                        for p in range(ps.npatch)]
        configs = [("xreg", 1, 0), ("xreg", 2, 0), ("xreg", 4, 0), ("xreg", 4, 300), ("chunk", 1, 0),
                   ("chunk", 4, 0)]
        outs = []
        for kind, n, grid in configs:
            if kind == "xreg":
                ps.set_xline_config(scheme, waves=n, grid=grid)
            else:
                ps.set_line_config(0, scheme, n, tile=64, grid=grid)
            u = ps.pack_u(s.u0)
            w = ps.empty_u()
            ps.line_relax(0, scheme, om, 2, u, f, w)
            torch.cuda.synchronize()
            log("forms %s %s n=%d grid=%d" % (scheme, kind, n, grid))
            for p in range(ps.npatch):
                assert relerr(ps.view_u(u, p).cpu().numpy(), refs[scheme][p]) < TOL, (scheme, kind, n, grid, p)
            outs.append(u)
        # the register form's result does not depend on the workgroup size or grid
        assert all(torch.equal(outs[0], o) for o in outs[1:4]), scheme


def test_fp32_register_x_lines():
    """FP32 block solve (FP64 residual and update) in the register form:
    within the FP32 bound of the FP64 result."""
    p = small_patch(40, 12, 11, seed=5, eps=(1.0, 3.0, 7.0))
    ref = oracle.line_sweeps(p.u0, p.f, p.eps, p.h, 0, oracle.JACOBI, 0.8, 3)
    s = Single(p)
    s.ps.set_xline_config("jacobi", waves=4)
    assert s.ps.line_config(0, "jacobi")["form"] == 1
    s.line(0, "jacobi", 0.8, 3, prec="fp32")
    err = relerr(s.u_np(), ref)
    log("fp32 register x-lines relerr %.3e" % err)
    assert 1e-10 < err < 3 * 0.8 * 1e-6     # k omega eta_32, eta_32 = 1e-6
