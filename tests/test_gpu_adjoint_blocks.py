"""GPU parity of the adjoint of line and plane block sweeps under damped
Jacobi and two-colour GS (bs_block_backward) against the oracle's reverse
mode, which is pinned by dense Jacobians and central differences: gradients in
u0 (interior and face ghosts) and f to 1e-10 relative, in eps to 1e-9, with
checkpoint intervals that split the sweeps into several recomputed segments;
and the autograd form through BlockSmoothFn."""
import numpy as np
import pytest
import torch

import oracle
import paper_1208_1975_amd as bs
from conftest import relerr
from gpu_util import log, need_gpu
from workloads import small_patch

pytestmark = pytest.mark.gpu

OS = {"jacobi": oracle.JACOBI, "colored": oracle.COLORED_GS}


@pytest.fixture(scope="module", autouse=True)
def _setup():
    need_gpu()
    oracle.set_threads(0)
    yield


def _grads(p, kind, axis, scheme, omega, K, ckpt, gK):
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    u0, f = ps.pack_u([p.u0]), ps.pack_f([p.f])
    g = ps.pack_u([gK])
    nbytes = bs.bs_block_backward_workspace_bytes(ps.handle, kind, axis, scheme, K, ckpt)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    gu0, gf = torch.zeros_like(u0), torch.zeros_like(f)
    geps = torch.zeros(3, dtype=torch.float64, device="cuda")
    bs.bs_block_backward(ps.handle, kind, axis, scheme, omega, K, ckpt, u0, f, g, gu0, gf, geps, ws)
    torch.cuda.synchronize()
    out = (ps.view_u(gu0, 0).cpu().numpy().copy(), ps.view_f(gf, 0).cpu().numpy().copy(), geps.cpu().numpy())
    ps.close()
    return out


def _face_mask(shape):
    nz, ny, nx = (s - 2 for s in shape)
    m = np.zeros(shape, dtype=bool)
    m[1:-1, 1:-1, 0] = m[1:-1, 1:-1, -1] = True
    m[1:-1, 0, 1:-1] = m[1:-1, -1, 1:-1] = True
    m[0, 1:-1, 1:-1] = m[-1, 1:-1, 1:-1] = True
    return m


@pytest.mark.parametrize("kind,axis", [("line", 0), ("line", 1), ("line", 2), ("plane", 0), ("plane", 1),
                                       ("plane", 2)])
@pytest.mark.parametrize("scheme,omega", [("jacobi", 0.8), ("colored", 1.0), ("colored", 1.2)])
@pytest.mark.parametrize("dims", [(9, 7, 6), (20, 5, 33)])
def test_block_adjoint_matches_oracle(kind, axis, scheme, omega, dims):
    p = small_patch(*dims, seed=71 + axis, eps=(1.0, 3.0, 7.0))
    K, ckpt = 5, 2
    gK = np.random.default_rng(3).uniform(-1, 1, p.u0.shape)
    log("adjoint %s %d %s %.1f %s" % (kind, axis, scheme, omega, dims))
    gu, gf, ge = _grads(p, kind, axis, scheme, omega, K, ckpt, gK)
    ru, rf, re = oracle.block_adjoint(p.u0, p.f, p.eps, p.h, kind, axis, OS[scheme], omega, K, gK)
    assert relerr(gu[1:-1, 1:-1, 1:-1], ru[1:-1, 1:-1, 1:-1]) < 1e-10
    m = _face_mask(gu.shape)
    assert relerr(gu[m], ru[m]) < 1e-10
    assert relerr(gf, rf) < 1e-10
    assert relerr(ge, re) < 1e-9


@pytest.mark.parametrize("ckpt", [1, 3, 7])
def test_checkpoint_interval_does_not_change_gradients(ckpt):
    p = small_patch(24, 16, 12, seed=5, eps=(1.0, 1.0, 10.0))
    gK = np.random.default_rng(4).uniform(-1, 1, p.u0.shape)
    ref = _grads(p, "plane", 2, "colored", 1.0, 6, 6, gK)
    got = _grads(p, "plane", 2, "colored", 1.0, 6, ckpt, gK)
    for a, b in zip(got, ref):
        assert relerr(a, b) < 1e-13


def test_autograd_block_smoother():
    p = small_patch(16, 12, 10, seed=6, eps=(1.0, 2.0, 5.0))
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    f = ps.pack_f([p.f]).requires_grad_(True)
    u0 = ps.pack_u([p.u0]).requires_grad_(True)
    eps = torch.tensor([p.eps], dtype=torch.float64, device="cuda", requires_grad=True)
    uK = bs.block_smooth(f, u0, eps, ps, kind="plane", axis=1, scheme="colored", omega=1.0, K=4, ckpt=2)
    target = torch.zeros_like(uK)
    loss = ((uK - target) ** 2).sum()
    loss.backward()
    gK = 2 * ps.view_u(uK.detach(), 0).cpu().numpy()
    gK_full = np.zeros_like(p.u0)
    gK_full[1:-1, 1:-1, 1:-1] = gK[1:-1, 1:-1, 1:-1]
    ru, rf, re = oracle.block_adjoint(p.u0, p.f, p.eps, p.h, "plane", 1, oracle.COLORED_GS, 1.0, 4, gK_full)
    assert relerr(ps.view_f(f.grad, 0).cpu().numpy(), rf) < 1e-10
    assert relerr(ps.view_u(u0.grad, 0).cpu().numpy()[1:-1, 1:-1, 1:-1], ru[1:-1, 1:-1, 1:-1]) < 1e-10
    assert relerr(eps.grad.cpu().numpy().reshape(-1), re) < 1e-9
    ps.close()


def test_block_backward_refusals():
    p = small_patch(8, 8, 8, seed=1)
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    u0, f = ps.pack_u([p.u0]), ps.pack_f([p.f])
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    with pytest.raises(bs.BSError) as ei:
        bs.bs_block_backward(ps.handle, "line", 2, "chaotic", 1.0, 2, 1, u0, f, u0, None, None, None, ws)
    assert ei.value.status == bs.BS_ERR_UNSUPPORTED
    with pytest.raises(bs.BSError) as ei:
        bs.bs_block_backward(ps.handle, "line", 2, "jacobi", 0.8, 2, 1, u0, f, u0, None, None, None,
                             ws[:16])
    assert ei.value.status == bs.BS_ERR_INVALID
    assert bs.bs_block_backward_workspace_bytes(ps.handle, "line", 2, "chaotic", 2, 1) == 0
    ps.close()


@pytest.mark.parametrize("kind,axis,scheme,omega", [("line", 2, "jacobi", 0.8), ("line", 1, "colored", 1.0),
                                                    ("line", 0, "jacobi", 1.1), ("plane", 2, "jacobi", 1.0),
                                                    ("plane", 0, "colored", 1.2)])
@pytest.mark.parametrize("K,ckpt", [(7, 3), (4, 5), (1, 1)])
def test_forward_checkpoints_then_backward(kind, axis, scheme, omega, K, ckpt):
    """bs_block_forward_ckpt + bs_block_backward_ckpt: the forward's u_K is
    the smoother's (the same sweeps as line_relax / plane_relax, to rounding
    order), and the backward from its checkpoints gives bit for bit the
    gradients of bs_block_backward, twice in a row (the checkpoints stay)."""
    p = small_patch(19, 13, 22, seed=17 + axis, eps=(1.0, 4.0, 9.0))
    gK = np.random.default_rng(8).uniform(-1, 1, p.u0.shape)
    log("forward ckpt %s %d %s %.1f K %d ckpt %d" % (kind, axis, scheme, omega, K, ckpt))
    ref = _grads(p, kind, axis, scheme, omega, K, ckpt, gK)
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    u0, f, g = ps.pack_u([p.u0]), ps.pack_f([p.f]), ps.pack_u([gK])
    nbytes = bs.bs_block_backward_workspace_bytes(ps.handle, kind, axis, scheme, K, ckpt)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    u = u0.clone()
    bs.bs_block_forward_ckpt(ps.handle, kind, axis, scheme, omega, K, ckpt, u, f, ws)
    uref, w = u0.clone(), ps.empty_u()
    if kind == "line":
        ps.line_relax(axis, scheme, omega, K, uref, f, w)
    else:
        ps.plane_relax(axis, scheme, omega, K, uref, f, w)
    torch.cuda.synchronize()
    assert relerr(ps.view_u(u, 0).cpu().numpy(), ps.view_u(uref, 0).cpu().numpy()) < 1e-13
    for rep in range(2):
        gu0, gf = torch.zeros_like(u0), torch.zeros_like(f)
        geps = torch.zeros(3, dtype=torch.float64, device="cuda")
        bs.bs_block_backward_ckpt(ps.handle, kind, axis, scheme, omega, K, ckpt, f, g, gu0, gf, geps, ws)
        torch.cuda.synchronize()
        got = (ps.view_u(gu0, 0).cpu().numpy(), ps.view_f(gf, 0).cpu().numpy(), geps.cpu().numpy())
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), rep
    ps.close()


@pytest.mark.parametrize("kind,axis,scheme", [("line", 2, "jacobi"), ("line", 1, "colored"), ("plane", 1, "jacobi")])
def test_forward_checkpoints_patch_set(kind, axis, scheme):
    """Three patches of different shapes and eps: the checkpoint-split adjoint
    gives bit for bit the gradients of bs_block_backward on the same set."""
    ps_ = [small_patch(*d, seed=90 + i, eps=e) for i, (d, e) in
           enumerate([((12, 9, 30), (1.0, 2.0, 20.0)), ((7, 16, 11), (3.0, 1.0, 5.0)), ((20, 5, 8), (1.0, 1.0, 1.0))])]
    ps = bs.PatchSet([p.dims for p in ps_], [p.eps for p in ps_], [p.h for p in ps_])
    u0, f = ps.pack_u([p.u0 for p in ps_]), ps.pack_f([p.f for p in ps_])
    rng = np.random.default_rng(12)
    g = ps.pack_u([rng.uniform(-1, 1, p.u0.shape) for p in ps_])
    K, ckpt, omega = 6, 4, 0.9
    nbytes = bs.bs_block_backward_workspace_bytes(ps.handle, kind, axis, scheme, K, ckpt)
    outs = []
    for split in (False, True):
        log("forward ckpt patch set %s %d %s split=%s" % (kind, axis, scheme, split))
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        gu0, gf = torch.zeros_like(u0), torch.zeros_like(f)
        geps = torch.zeros(3 * ps.npatch, dtype=torch.float64, device="cuda")
        if split:
            u = u0.clone()
            bs.bs_block_forward_ckpt(ps.handle, kind, axis, scheme, omega, K, ckpt, u, f, ws)
            uref, w = u0.clone(), ps.empty_u()
            if kind == "line":
                ps.line_relax(axis, scheme, omega, K, uref, f, w)
            else:
                ps.plane_relax(axis, scheme, omega, K, uref, f, w)
            bs.bs_block_backward_ckpt(ps.handle, kind, axis, scheme, omega, K, ckpt, f, g, gu0, gf, geps, ws)
            torch.cuda.synchronize()
            for i in range(ps.npatch):
                assert relerr(ps.view_u(u, i).cpu().numpy(), ps.view_u(uref, i).cpu().numpy()) < 1e-13
        else:
            bs.bs_block_backward(ps.handle, kind, axis, scheme, omega, K, ckpt, u0, f, g, gu0, gf, geps, ws)
            torch.cuda.synchronize()
        outs.append((gu0.cpu().numpy(), gf.cpu().numpy(), geps.cpu().numpy()))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    ps.close()
