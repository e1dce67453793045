"""Helpers for the GPU parity tests: run the HIP library on patches built by
the seeded generators and bring results back as NumPy arrays."""
import sys

import numpy as np
import pytest
import torch

import paper_1208_1975_amd as bs


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bs.lib()   # raises if the HIP library is missing: no fallback


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


class Single:
    """One patch on the device: u, f, work tensors in the library layout."""

    def __init__(self, patch, eps=None):
        need_gpu()
        self.patch = patch
        nx, ny, nz = patch.dims
        self.ps = bs.PatchSet([(nx, ny, nz)], [eps or patch.eps], [patch.h])
        self.u = self.ps.pack_u([patch.u0])
        self.f = self.ps.pack_f([patch.f])
        self.work = self.ps.empty_u()

    def u_np(self):
        torch.cuda.synchronize()
        return self.ps.view_u(self.u, 0).cpu().numpy().copy()

    def set_u(self, arr):
        self.ps.pack_u([arr], out=self.u)

    def line(self, axis, scheme, omega, nsweeps, prec="fp64"):
        self.ps.line_relax(axis, scheme, omega, nsweeps, self.u, self.f, self.work, prec=prec)

    def plane(self, normal, scheme, omega, nsweeps, prec="fp64", refine=0):
        self.ps.plane_relax(normal, scheme, omega, nsweeps, self.u, self.f, self.work, prec=prec, refine=refine)

    def residual(self):
        r = self.ps.empty_f()
        n2 = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.ps.residual(self.u, self.f, r, n2)
        torch.cuda.synchronize()
        return self.ps.view_f(r, 0).cpu().numpy().copy(), float(n2.item())

    def rnorm(self):
        n2 = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.ps.residual(self.u, self.f, None, n2)
        torch.cuda.synchronize()
        return float(np.sqrt(n2.item()))
