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


# Stated bound for the mixed forms: each low-precision solve returns the
# correction with relative error at most eta (FP32 transforms: 1e-6, BF16
# transforms with FP32 accumulation: 1.5e-2), each defect-correction step
# multiplies it by eta, and the iteration contracts, so after k sweeps the
# deviation from the FP64 iterate is at most about k * omega * eta^(refine+1)
# relative to max|u| (the first correction is of the size of u).
ETA = {"fp32": 1e-6, "bf16": 1.5e-2}


def mixed_bound(prec, refine, k, omega=1.0):
    return k * omega * ETA[prec] ** (refine + 1)


MIXED = [("fp32", 0), ("fp32", 1), ("bf16", 0), ("bf16", 1), ("bf16", 2)]


@pytest.mark.parametrize("prec,refine", MIXED)
@pytest.mark.parametrize("normal", [0, 1, 2])
def test_mixed_plane_error_vs_fp64(prec, refine, normal):
    """Mixed plane Jacobi (FP64 residual and update): the error against the FP64
    oracle after three sweeps stays within the stated bound."""
    p = small_patch(40, 36, 33, seed=81 + normal, eps=(1.0, 100.0, 100.0))
    bound = mixed_bound(prec, refine, 3)
    s = Single(p)
    s.plane(normal, "jacobi", 1.0, 3, prec=prec, refine=refine)
    got = s.u_np()
    ref = oracle.plane_sweeps(p.u0, p.f, p.eps, p.h, normal, oracle.JACOBI, 1.0, 3)
    e = relerr(got, ref)
    log("mixed %s refine %d normal %d: relerr vs FP64 %.3e (bound %.0e)" % (prec, refine, normal, e, bound))
    assert e < bound


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_plane_fixed_point(prec):
    """With the exact solution the FP64 residual is at rounding level, so the
    low-precision correction cannot move u beyond it."""
    p = small_patch(24, 20, 18, seed=9, eps=(2.0, 1.0, 5.0))
    r, _ = oracle.residual(p.u0, np.zeros_like(p.f), p.eps, p.h)
    f_exact = -r / (p.h * p.h)
    for normal in (0, 2):
        s = Single(p)
        s.f = s.ps.pack_f([f_exact])
        s.plane(normal, "colored", 1.0, 2, prec=prec, refine=1)
        assert relerr(s.u_np(), p.u0) < 1e-13


@pytest.mark.timeout(900)
def test_c3_mixed_forms_error_statement():
    """512^3, eps (1,100,100), xy-plane Jacobi omega 1: five sweeps per form;
    error of each mixed form against the FP64 GPU result (itself checked
    against the oracle plane by plane above)."""
    p = c3_patch()
    ref = Single(p)
    ref.plane(2, "jacobi", 1.0, 5)
    u64 = ref.u_np()
    r64 = ref.rnorm()
    for prec, refine in (("fp32", 0), ("fp32", 1), ("bf16", 1), ("bf16", 2)):
        bound = mixed_bound(prec, refine, 5)
        s = Single(p)
        s.plane(2, "jacobi", 1.0, 5, prec=prec, refine=refine)
        e = relerr(s.u_np(), u64)
        rr = s.rnorm() / r64
        log("C3 %s refine %d: relerr vs FP64 %.3e (bound %.1e), residual ratio %.6f" % (prec, refine, e, bound, rr))
        assert e < bound
        assert abs(rr - 1.0) < 1e-3
