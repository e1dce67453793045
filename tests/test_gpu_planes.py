"""GPU parity of the plane-block path (fast diagonalisation on the matrix
cores) against the oracle (partial diagonalisation, a different algorithm).

FP64 Jacobi and two-colour GS: max-norm relative error <= 1e-12 (the plane
blocks are well conditioned, kappa <= 3 for the tested weights).  The chaotic
scheme for planes runs the same colour-major order as the two-colour scheme,
so it is checked against the oracle's two-colour GS too."""
import numpy as np
import pytest

import oracle
from conftest import relerr
from gpu_util import Single, log, need_gpu
from workloads import c3_patch, small_patch

pytestmark = pytest.mark.gpu

TOL = 1e-12
SHAPES = [(5, 4, 3), (7, 6, 5), (1, 1, 1), (2, 3, 1), (1, 5, 2), (33, 17, 9), (64, 8, 70), (130, 3, 67),
          (20, 65, 3), (100, 100, 2)]


@pytest.fixture(scope="module", autouse=True)
def _setup():
    need_gpu()
    oracle.set_threads(0)
    yield


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("normal", [0, 1, 2])
@pytest.mark.parametrize("scheme", ["jacobi", "colored", "chaotic"])
def test_plane_parity_small(dims, normal, scheme):
    p = small_patch(*dims, seed=51 + normal, eps=(1.0, 3.0, 7.0))
    omega = 0.8 if scheme == "jacobi" else 1.0
    osch = oracle.JACOBI if scheme == "jacobi" else oracle.COLORED_GS
    for nsweeps in (1, 2, 3):
        log("plane %s normal=%d %s nsweeps=%d" % (dims, normal, scheme, nsweeps))
        s = Single(p)
        s.plane(normal, scheme, omega, nsweeps)
        got = s.u_np()
        ref = oracle.plane_sweeps(p.u0, p.f, p.eps, p.h, normal, osch, omega, nsweeps)
        assert relerr(got, ref) < TOL, (dims, normal, scheme, nsweeps)
        gm = ~np.pad(np.ones(p.f.shape, bool), 1, constant_values=False)
        assert np.array_equal(got[gm], p.u0[gm])


def test_plane_fixed_point():
    p = small_patch(24, 20, 18, seed=9, eps=(2.0, 1.0, 5.0))
    r, _ = oracle.residual(p.u0, np.zeros_like(p.f), p.eps, p.h)
    f_exact = -r / (p.h * p.h)
    for normal in (0, 1, 2):
        for scheme in ("jacobi", "colored"):
            s = Single(p)
            s.f = s.ps.pack_f([f_exact])
            s.plane(normal, scheme, 1.0, 2)
            assert relerr(s.u_np(), p.u0) < 1e-13, (normal, scheme)


@pytest.mark.timeout(900)
def test_c3_xy_plane_jacobi_sampled():
    """512^3, eps (1,100,100), xy-plane Jacobi omega 1: two sweeps; for each
    sweep, sampled planes of the GPU result equal the oracle's update of those
    planes computed from the GPU's previous iterate."""
    p = c3_patch()
    s = Single(p)
    planes = [0, 1, 255, 256, 510, 511]
    prev = p.u0
    for sweep in (1, 2):
        log("C3 sweep %d: gpu" % sweep)
        s.plane(2, "jacobi", 1.0, 1)
        got = s.u_np()
        log("C3 sweep %d: oracle on planes %s" % (sweep, planes))
        ref = oracle.plane_update_some(prev, p.f, p.eps, p.h, 2, 1.0, planes)
        for k in planes:
            e = relerr(got[k + 1], ref[k + 1])
            log("  plane %d relerr %.3e" % (k, e))
            assert e < TOL
        prev = got
