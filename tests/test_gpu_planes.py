"""GPU parity of the plane-block path (fast diagonalisation on the matrix
cores) against the oracle (partial diagonalisation, a different algorithm).

FP64 Jacobi and two-colour GS: max-norm relative error <= 1e-12 (the plane
blocks are well conditioned, kappa <= 3 for the tested weights).  The chaotic
scheme for planes runs the same colour-major order as the two-colour scheme,
so it is checked against the oracle's two-colour GS too."""
import math

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
# relative to max|u| (the first correction is of the size of u).  The BF16
# chain stores the residual and the correction in FP32, which adds a rounding
# of at most 2^-24 of each to every step's correction.
ETA = {"fp32": 1e-6, "bf16": 1.5e-2}
STORE = {"fp32": 0.0, "bf16": 2.0 ** -24}


def mixed_bound(prec, refine, k, omega=1.0):
    return k * omega * (ETA[prec] ** (refine + 1) + 2 * STORE[prec])


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


def _dev_relerr(a, b):
    return float((a - b).abs().max() / b.abs().max())


@pytest.mark.timeout(900)
def test_c3_mixed_forms_error_statement():
    """512^3, eps (1,100,100), xy-plane Jacobi omega 1, the full 50 sweeps:
    every 10 sweeps, the max-norm error of each mixed form against the FP64
    GPU iterate (itself checked against the oracle plane by plane above) stays
    within k * omega * eta^(refine+1), and its residual within 1e-3 of the FP64
    one.  BF16 without refinement is logged but carries no bound: its solve
    error (about 3e-3) exceeds the 1.9e-5 stability margin of the
    z-checkerboard mode at omega 1, so the iteration is not a contraction."""
    import torch
    p = c3_patch()
    ref = Single(p)
    u64, r64 = {}, {}
    for k in range(10, 51, 10):
        ref.plane(2, "jacobi", 1.0, 10)
        u64[k] = ref.u.clone()
        r64[k] = ref.rnorm()
    del ref
    for prec, refine in (("fp32", 0), ("fp32", 1), ("bf16", 1), ("bf16", 2), ("bf16", 0)):
        s = Single(p)
        for k in range(10, 51, 10):
            s.plane(2, "jacobi", 1.0, 10, prec=prec, refine=refine)
            torch.cuda.synchronize()
            e = _dev_relerr(s.u, u64[k])
            rr = s.rnorm() / r64[k]
            if prec == "bf16" and refine == 0:
                log("C3 bf16 refine 0 sweep %d: relerr vs FP64 %.3e (no bound), residual ratio %.6f" % (k, e, rr))
                continue
            bound = mixed_bound(prec, refine, k)
            log("C3 %s refine %d sweep %d: relerr vs FP64 %.3e (bound %.1e), residual ratio %.6f"
                % (prec, refine, k, e, bound, rr))
            assert e < bound, (prec, refine, k)
            assert abs(rr - 1.0) < 1e-3, (prec, refine, k)
        del s


@pytest.mark.timeout(600)
def test_c3_z_checkerboard_amplification():
    """Stability of the mixed forms at omega 1 (the residual-correction form of
    eq. blockiteration2 with an inexact block solve): on 512^3 with eps
    (1,100,100), f = 0 and zero ghosts, the mode sin((i+1)pi/513)
    sin((j+1)pi/513) sin(512(k+1)pi/513) is damped by one xy-plane Jacobi sweep
    to g u with g = nu/mu = -(1 - 3.77e-5) (closed form, which the FP64 sweep
    must reproduce).  The low-precision solves must not amplify it:
    ||u_1|| / ||u_0|| <= 1 for FP32 (refine 0, 1) and BF16 with refine 2.
    BF16 with refine 0 and 1 are logged (predicted unstable / borderline)."""
    import torch

    import paper_1208_1975_amd as bs
    n = 512
    eps = (1.0, 100.0, 100.0)
    h = 1.0 / n
    th = [math.pi / (n + 1), math.pi / (n + 1), n * math.pi / (n + 1)]
    mu = 4 * eps[0] * math.sin(th[0] / 2) ** 2 + 4 * eps[1] * math.sin(th[1] / 2) ** 2 + 2 * eps[2]
    nu = 2 * eps[2] * math.cos(th[2])
    g = nu / mu
    log("z-checkerboard: g = %.10f, 1 - |g| = %.3e" % (g, 1 - abs(g)))
    ps = bs.PatchSet([(n, n, n)], [eps], [h])
    idx = torch.arange(1, n + 1, dtype=torch.float64, device="cuda")
    sx = torch.sin(th[0] * idx)
    sz = torch.sin(th[2] * idx)
    f = ps.empty_f()
    u0 = ps.empty_u()
    ps.view_u(u0, 0)[1:-1, 1:-1, 1:-1] = sz[:, None, None] * sx[None, :, None] * sx[None, None, :]
    n0 = float(torch.linalg.vector_norm(u0))
    w = ps.empty_u()
    for prec, refine, must in (("fp64", 0, True), ("fp32", 0, True), ("fp32", 1, True), ("bf16", 2, True),
                               ("bf16", 1, False), ("bf16", 0, False)):
        u = u0.clone()
        ps.plane_relax(2, "jacobi", 1.0, 1, u, f, w, prec=prec, refine=refine)
        torch.cuda.synchronize()
        amp = float(torch.linalg.vector_norm(u)) / n0
        dev = float(torch.linalg.vector_norm(u - g * u0)) / n0
        log("z-checkerboard %s refine %d: ||u1||/||u0|| = %.10f (1 - amp %.3e), ||u1 - g u0||/||u0|| = %.3e"
            % (prec, refine, amp, 1 - amp, dev))
        if prec == "fp64":
            assert dev < 1e-10
        elif must:
            assert amp <= 1.0, (prec, refine, amp)
        del u
    ps.close()
