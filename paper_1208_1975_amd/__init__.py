"""Python binding of libblocksmooth.so (line- and plane-block relaxation of the
constant-coefficient 7-point stencil on MI355X).

Argument marshalling only: every step of every sweep runs in the library's
HIP kernels.  PyTorch supplies device memory (float64 CUDA tensors) and the
current stream.  The functions carry the C names (``bs_line_relax`` ...) and
raise ``BSError`` on a non-OK status.  If the library has not been built the
first call raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must be loaded first: the library binds to torch's HIP runtime)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libblocksmooth.so")

BS_OK, BS_ERR_INVALID, BS_ERR_UNSUPPORTED, BS_ERR_OOM, BS_ERR_HIP = range(5)
BS_JACOBI, BS_CHAOTIC_GS, BS_COLORED_GS = range(3)
BS_FP64, BS_MIXED_FP32, BS_MIXED_BF16 = range(3)

SCHEMES = {"jacobi": BS_JACOBI, "chaotic": BS_CHAOTIC_GS, "chaotic_gs": BS_CHAOTIC_GS,
           "colored": BS_COLORED_GS, "colored_gs": BS_COLORED_GS}
PRECISIONS = {"fp64": BS_FP64, "fp32": BS_MIXED_FP32, "bf16": BS_MIXED_BF16}

_STATUS = {1: "BS_ERR_INVALID", 2: "BS_ERR_UNSUPPORTED", 3: "BS_ERR_OOM", 4: "BS_ERR_HIP"}

# Every symbol the public header declares.
EXPORTS = ("bs_layout_plan", "bs_create_patchset", "bs_destroy_patchset", "bs_set_eps", "bs_layout",
           "bs_residual", "bs_line_relax", "bs_plane_relax", "bs_cube_prepare", "bs_cube_relax",
           "bs_autotune_line", "bs_line_config", "bs_set_bc", "bs_set_links", "bs_exchange_ghosts",
           "bs_mg_create", "bs_mg_destroy", "bs_mg_levels", "bs_vcycle", "bs_block_backward_workspace_bytes",
           "bs_block_backward", "bs_block_forward_ckpt", "bs_block_backward_ckpt", "bs_backward_workspace_bytes",
           "bs_relax_backward", "bs_residual_noalloc", "bs_last_error")


class BSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, str(status)), msg))
        self.status = status


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libblocksmooth.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, dbl, vp, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
    P = ctypes.POINTER
    L.bs_layout_plan.argtypes = [i32, vp, P(i64), P(i64), vp, vp]
    L.bs_create_patchset.argtypes = [i32, vp, vp, vp, P(vp)]
    L.bs_destroy_patchset.argtypes = [vp]
    L.bs_destroy_patchset.restype = None
    L.bs_set_eps.argtypes = [vp, vp]
    L.bs_layout.argtypes = [vp, P(i64), P(i64), vp, vp]
    L.bs_residual.argtypes = [vp, vp, vp, vp, vp, vp]
    L.bs_line_relax.argtypes = [vp, i32, ctypes.c_int, dbl, i32, ctypes.c_int, vp, vp, vp, vp]
    L.bs_plane_relax.argtypes = [vp, i32, ctypes.c_int, dbl, i32, ctypes.c_int, i32, vp, vp, vp, vp]
    L.bs_cube_prepare.argtypes = [vp, i32, i32, i32]
    L.bs_cube_relax.argtypes = [vp, i32, i32, i32, ctypes.c_int, dbl, i32, ctypes.c_int, vp, vp, vp, vp]
    L.bs_autotune_line.argtypes = [vp, i32, ctypes.c_int, vp, vp, vp]
    L.bs_line_config.argtypes = [vp, i32, ctypes.c_int, vp]
    L.bsi_set_line_cfg.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.bsi_set_line_cfg.restype = ctypes.c_int
    L.bsi_set_xline_cfg.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.bsi_set_xline_cfg.restype = ctypes.c_int
    L.bsi_set_xz_cfg.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.bsi_set_xz_cfg.restype = ctypes.c_int
    L.bsi_set_pair.argtypes = [vp, ctypes.c_int]
    L.bsi_set_pair.restype = ctypes.c_int
    L.bsi_set_line_direct.argtypes = [vp, ctypes.c_int]
    L.bsi_set_line_direct.restype = ctypes.c_int
    L.bsi_set_chaotic_chunk.argtypes = [vp, ctypes.c_int]
    L.bsi_set_chaotic_chunk.restype = ctypes.c_int
    L.bsi_set_graphs.argtypes = [vp, ctypes.c_int]
    L.bsi_set_graphs.restype = ctypes.c_int
    L.bsi_line_relax_per_patch.argtypes = [vp, i32, ctypes.c_int, dbl, i32, vp, vp, vp, vp]
    L.bsi_line_relax_per_patch.restype = ctypes.c_int
    L.bsi_stream_triad.argtypes = [vp, vp, vp, i64, ctypes.c_int, vp]
    L.bsi_stream_triad.restype = ctypes.c_int
    L.bs_backward_workspace_bytes.argtypes = [vp, i32, i32, i32]
    L.bs_backward_workspace_bytes.restype = sz
    L.bs_relax_backward.argtypes = [vp, i32, dbl, i32, i32, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.bs_set_bc.argtypes = [vp, vp]
    L.bs_set_links.argtypes = [vp, i32, vp]
    L.bs_exchange_ghosts.argtypes = [vp, vp, vp]
    L.bs_mg_create.argtypes = [vp, i32, i32, ctypes.c_int, dbl, i32, i32, i32, i32, i32, P(vp)]
    L.bs_mg_destroy.argtypes = [vp]
    L.bs_mg_destroy.restype = None
    L.bs_mg_levels.argtypes = [vp, P(i32)]
    L.bs_vcycle.argtypes = [vp, vp, vp, vp, vp]
    L.bs_block_backward_workspace_bytes.argtypes = [vp, i32, i32, ctypes.c_int, i32, i32]
    L.bs_block_backward_workspace_bytes.restype = sz
    L.bs_block_backward.argtypes = [vp, i32, i32, ctypes.c_int, dbl, i32, i32, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.bs_block_forward_ckpt.argtypes = [vp, i32, i32, ctypes.c_int, dbl, i32, i32, vp, vp, vp, sz, vp]
    L.bs_block_backward_ckpt.argtypes = [vp, i32, i32, ctypes.c_int, dbl, i32, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    L.bs_last_error.argtypes = []
    L.bs_last_error.restype = ctypes.c_char_p
    for name in ("bs_layout_plan", "bs_create_patchset", "bs_set_eps", "bs_layout", "bs_residual",
                 "bs_line_relax", "bs_plane_relax", "bs_autotune_line", "bs_line_config", "bs_relax_backward",
                 "bs_set_bc", "bs_set_links", "bs_exchange_ghosts", "bs_mg_create", "bs_mg_levels", "bs_vcycle",
                 "bs_block_backward", "bs_block_forward_ckpt", "bs_block_backward_ckpt"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(st):
    if st != BS_OK:
        raise BSError(st, lib().bs_last_error().decode(errors="replace"))


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch.Tensor")
    if not t.is_cuda:
        raise ValueError("buffers must be device (cuda) tensors")
    if not t.is_contiguous():
        raise ValueError("buffers must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _f64(t, numel, name):
    if t is None:
        return None
    if t.dtype != torch.float64:
        raise TypeError("%s must be float64" % name)
    if t.numel() < numel:
        raise ValueError("%s has %d elements, needs %d" % (name, t.numel(), numel))
    return _ptr(t)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _host_array(ctype, values):
    values = list(values)
    return (ctype * len(values))(*values)


def _scheme(s):
    return SCHEMES[s] if isinstance(s, str) else int(s)


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


# --- the C names -------------------------------------------------------------

def bs_layout_plan(dims):
    """(u_numel, f_numel, u_offsets, f_offsets) for patches dims = [(nx,ny,nz), ...]."""
    n = len(dims)
    d = _host_array(ctypes.c_int32, [int(v) for t in dims for v in t])
    un, fn = ctypes.c_int64(), ctypes.c_int64()
    uo = (ctypes.c_int64 * max(n, 1))()
    fo = (ctypes.c_int64 * max(n, 1))()
    _check(lib().bs_layout_plan(n, d, ctypes.byref(un), ctypes.byref(fn), uo, fo))
    return un.value, fn.value, list(uo)[:n], list(fo)[:n]


def bs_create_patchset(dims, eps, h):
    """Opaque handle for patches dims [(nx,ny,nz)], eps [(ex,ey,ez)], h [h]."""
    n = len(dims)
    d = _host_array(ctypes.c_int32, [int(v) for t in dims for v in t])
    e = _host_array(ctypes.c_double, [float(v) for t in eps for v in t])
    hh = _host_array(ctypes.c_double, [float(v) for v in h])
    out = ctypes.c_void_p()
    _check(lib().bs_create_patchset(n, d, e, hh, ctypes.byref(out)))
    return out


def bs_destroy_patchset(ps):
    lib().bs_destroy_patchset(ps)


def bs_set_eps(ps, eps):
    e = _host_array(ctypes.c_double, [float(v) for t in eps for v in t])
    _check(lib().bs_set_eps(ps, e))


def bs_set_bc(ps, bc):
    """Per patch the 6-bit mask of extrapolated-Dirichlet faces (bit 2a: low
    face of axis a, bit 2a+1: high face)."""
    b = _host_array(ctypes.c_int32, [int(v) for v in bc])
    _check(lib().bs_set_bc(ps, b))


def bs_set_links(ps, links):
    """Face-adjacent patches [(a, axis, b)]: b lies on a's high side along axis."""
    flat = [int(v) for t in links for v in t]
    arr = _host_array(ctypes.c_int32, flat) if flat else None
    _check(lib().bs_set_links(ps, len(flat) // 3, arr))


def bs_exchange_ghosts(ps, u, stream=None):
    _check(lib().bs_exchange_ghosts(ps, _ptr(u), _stream(stream)))


def bs_mg_create(ps, kind, arg, scheme, omega, nu1, nu2, ncoarse, levels=0, coarse_bc=0):
    """Multigrid cycle object over patch set ps: kind 'line' (axis arg) or
    'plane' (normal arg) block smoothing."""
    k = {"line": 0, "plane": 1}[kind] if isinstance(kind, str) else int(kind)
    out = ctypes.c_void_p()
    _check(lib().bs_mg_create(ps, k, int(arg), _scheme(scheme), float(omega), int(nu1), int(nu2), int(ncoarse),
                              int(levels), int(coarse_bc), ctypes.byref(out)))
    return out


def bs_mg_destroy(mg):
    lib().bs_mg_destroy(mg)


def bs_mg_levels(mg):
    n = ctypes.c_int32()
    _check(lib().bs_mg_levels(mg, ctypes.byref(n)))
    return n.value


def bs_vcycle(mg, u, f, work=None, stream=None):
    _check(lib().bs_vcycle(mg, _ptr(u), _ptr(f), _ptr(work), _stream(stream)))


def bs_layout(ps, npatch):
    un, fn = ctypes.c_int64(), ctypes.c_int64()
    uo = (ctypes.c_int64 * npatch)()
    fo = (ctypes.c_int64 * npatch)()
    _check(lib().bs_layout(ps, ctypes.byref(un), ctypes.byref(fn), uo, fo))
    return un.value, fn.value, list(uo), list(fo)


def bs_residual(ps, u, f, r=None, rnorm2=None, stream=None):
    _check(lib().bs_residual(ps, _ptr(u), _ptr(f), _ptr(r), _ptr(rnorm2), _stream(stream)))


def bs_line_relax(ps, axis, scheme, omega, nsweeps, prec, u, f, work=None, stream=None):
    _check(lib().bs_line_relax(ps, int(axis), _scheme(scheme), float(omega), int(nsweeps), _prec(prec),
                               _ptr(u), _ptr(f), _ptr(work), _stream(stream)))


def bs_plane_relax(ps, normal_axis, scheme, omega, nsweeps, prec, refine, u, f, work=None, stream=None):
    _check(lib().bs_plane_relax(ps, int(normal_axis), _scheme(scheme), float(omega), int(nsweeps),
                                _prec(prec), int(refine), _ptr(u), _ptr(f), _ptr(work), _stream(stream)))


def bs_cube_prepare(ps, bx, by, bz):
    _check(lib().bs_cube_prepare(ps, int(bx), int(by), int(bz)))


def bs_cube_relax(ps, bx, by, bz, scheme, omega, nsweeps, prec, u, f, work=None, stream=None):
    _check(lib().bs_cube_relax(ps, int(bx), int(by), int(bz), _scheme(scheme), float(omega), int(nsweeps),
                               _prec(prec), _ptr(u), _ptr(f), _ptr(work), _stream(stream)))


def bs_autotune_line(ps, axis, scheme, u, f, stream=None):
    _check(lib().bs_autotune_line(ps, int(axis), _scheme(scheme), _ptr(u), _ptr(f), _stream(stream)))


def bs_line_config(ps, axis, scheme):
    """dict(chunks, chunk_len, tile, grid, tuned, form) of the launch configuration
    in use (forms 1 and 2, register x-lines: chunks = wavefronts per workgroup,
    chunk_len = cells per lane; form 2, marched along z: tile = planes per item)."""
    out = (ctypes.c_int32 * 6)()
    _check(lib().bs_line_config(ps, int(axis), _scheme(scheme), out))
    return dict(zip(("chunks", "chunk_len", "tile", "grid", "tuned", "form"), list(out)))


def bs_backward_workspace_bytes(ps, axis, nsweeps, ckpt_every):
    return int(lib().bs_backward_workspace_bytes(ps, int(axis), int(nsweeps), int(ckpt_every)))


def bs_relax_backward(ps, axis, omega, nsweeps, ckpt_every, u0, f, grad_uK, grad_u0=None, grad_f=None,
                      grad_eps=None, workspace=None, stream=None):
    wb = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _check(lib().bs_relax_backward(ps, int(axis), float(omega), int(nsweeps), int(ckpt_every), _ptr(u0),
                                   _ptr(f), _ptr(grad_uK), _ptr(grad_u0), _ptr(grad_f), _ptr(grad_eps),
                                   _ptr(workspace), wb, _stream(stream)))


def _kind(kind):
    return {"line": 0, "plane": 1}[kind] if isinstance(kind, str) else int(kind)


def bs_block_backward_workspace_bytes(ps, kind, axis, scheme, nsweeps, ckpt_every):
    return int(lib().bs_block_backward_workspace_bytes(ps, _kind(kind), int(axis), _scheme(scheme), int(nsweeps),
                                                       int(ckpt_every)))


def bs_block_backward(ps, kind, axis, scheme, omega, nsweeps, ckpt_every, u0, f, grad_uK, grad_u0=None,
                      grad_f=None, grad_eps=None, workspace=None, stream=None):
    wb = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _check(lib().bs_block_backward(ps, _kind(kind), int(axis), _scheme(scheme), float(omega), int(nsweeps),
                                   int(ckpt_every), _ptr(u0), _ptr(f), _ptr(grad_uK), _ptr(grad_u0), _ptr(grad_f),
                                   _ptr(grad_eps), _ptr(workspace), wb, _stream(stream)))


def bs_block_forward_ckpt(ps, kind, axis, scheme, omega, nsweeps, ckpt_every, u, f, workspace, stream=None):
    """u (in: u0, out: u_K) after the sweeps bs_block_backward differentiates,
    with the checkpoints left in `workspace` for bs_block_backward_ckpt."""
    wb = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _check(lib().bs_block_forward_ckpt(ps, _kind(kind), int(axis), _scheme(scheme), float(omega), int(nsweeps),
                                       int(ckpt_every), _ptr(u), _ptr(f), _ptr(workspace), wb, _stream(stream)))


def bs_block_backward_ckpt(ps, kind, axis, scheme, omega, nsweeps, ckpt_every, f, grad_uK, grad_u0=None,
                           grad_f=None, grad_eps=None, workspace=None, stream=None):
    """bs_block_backward from the checkpoints bs_block_forward_ckpt left in `workspace`."""
    wb = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _check(lib().bs_block_backward_ckpt(ps, _kind(kind), int(axis), _scheme(scheme), float(omega), int(nsweeps),
                                        int(ckpt_every), _ptr(f), _ptr(grad_uK), _ptr(grad_u0), _ptr(grad_f),
                                        _ptr(grad_eps), _ptr(workspace), wb, _stream(stream)))


def stream_triad(a, b, c, mode=0, stream=None):
    """Device streaming probe c = a + b (float64, n even): the 24 bytes per
    element of a line sweep at the HBM ceiling (mode 1: nontemporal b)."""
    n = c.numel()
    if a.numel() < n or b.numel() < n or not all(t.dtype == torch.float64 for t in (a, b, c)):
        raise ValueError("stream_triad: float64 buffers of at least c's size")
    st = lib().bsi_stream_triad(_ptr(a), _ptr(b), _ptr(c), n, int(mode), _stream(stream))
    if st != 0:
        raise BSError(st, "bsi_stream_triad failed")


def bs_last_error():
    return lib().bs_last_error().decode(errors="replace")


# --- a small owner of a patch set and its device buffers ---------------------

class PatchSet:
    """Owns a patch set handle; packs / unpacks per-patch arrays into the
    library's concatenated layout (u padded, f unpadded)."""

    def __init__(self, dims, eps, h, device="cuda"):
        self.dims = [tuple(int(v) for v in t) for t in dims]
        self.eps = [tuple(float(v) for v in t) for t in eps]
        self.h = [float(v) for v in h]
        self.device = torch.device(device)
        self.handle = bs_create_patchset(self.dims, self.eps, self.h)
        self.u_numel, self.f_numel, self.u_off, self.f_off = bs_layout(self.handle, len(self.dims))

    @property
    def npatch(self):
        return len(self.dims)

    def close(self):
        if self.handle is not None:
            bs_destroy_patchset(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_eps(self, eps):
        new = [tuple(float(v) for v in t) for t in eps]
        bs_set_eps(self.handle, new)   # raises on failure; the library then keeps its old eps
        self.eps = new

    def set_bc(self, bc):
        bs_set_bc(self.handle, bc)

    def set_links(self, links):
        bs_set_links(self.handle, links)

    def exchange_ghosts(self, u, stream=None):
        bs_exchange_ghosts(self.handle, u, stream)

    def empty_u(self):
        return torch.zeros(self.u_numel, dtype=torch.float64, device=self.device)

    def empty_f(self):
        return torch.zeros(self.f_numel, dtype=torch.float64, device=self.device)

    def pack_u(self, arrays, out=None):
        out = self.empty_u() if out is None else out
        for p, a in enumerate(arrays):
            nx, ny, nz = self.dims[p]
            n = (nx + 2) * (ny + 2) * (nz + 2)
            out[self.u_off[p]:self.u_off[p] + n].copy_(torch.as_tensor(a).reshape(-1))
        return out

    def pack_f(self, arrays, out=None):
        out = self.empty_f() if out is None else out
        for p, a in enumerate(arrays):
            nx, ny, nz = self.dims[p]
            n = nx * ny * nz
            out[self.f_off[p]:self.f_off[p] + n].copy_(torch.as_tensor(a).reshape(-1))
        return out

    def view_u(self, t, p):
        nx, ny, nz = self.dims[p]
        n = (nx + 2) * (ny + 2) * (nz + 2)
        return t[self.u_off[p]:self.u_off[p] + n].view(nz + 2, ny + 2, nx + 2)

    def view_f(self, t, p):
        nx, ny, nz = self.dims[p]
        return t[self.f_off[p]:self.f_off[p] + nx * ny * nz].view(nz, ny, nx)

    # thin method forms of the C calls
    def residual(self, u, f, r=None, rnorm2=None, stream=None):
        bs_residual(self.handle, u, f, r, rnorm2, stream)

    def line_relax(self, axis, scheme, omega, nsweeps, u, f, work=None, prec="fp64", stream=None):
        bs_line_relax(self.handle, axis, scheme, omega, nsweeps, prec, u, f, work, stream)

    def plane_relax(self, normal_axis, scheme, omega, nsweeps, u, f, work=None, prec="fp64", refine=0,
                    stream=None):
        bs_plane_relax(self.handle, normal_axis, scheme, omega, nsweeps, prec, refine, u, f, work, stream)

    def cube_prepare(self, block):
        bs_cube_prepare(self.handle, *block)

    def cube_relax(self, block, scheme, omega, nsweeps, u, f, work=None, prec="fp64", stream=None):
        bs_cube_relax(self.handle, *block, scheme, omega, nsweeps, prec, u, f, work, stream)

    def autotune_line(self, axis, scheme, u, f, stream=None):
        bs_autotune_line(self.handle, axis, scheme, u, f, stream)

    def line_config(self, axis, scheme):
        return bs_line_config(self.handle, axis, scheme)

    # tuning and comparison hooks of the library (not part of the C header)
    def set_line_config(self, axis, scheme, chunks, tile=64, grid=0):
        popt = (1, 2, 4, 8, 16).index(int(chunks))
        _check(lib().bsi_set_line_cfg(self.handle, int(axis), _scheme(scheme), popt, int(tile), int(grid)))

    def set_xline_config(self, scheme, waves=4, grid=0):
        """Register x-line kernel (x-lines of up to 64 cells across the lanes of
        a 16-lane row) with `waves` wavefronts per workgroup."""
        _check(lib().bsi_set_xline_cfg(self.handle, _scheme(scheme), int(waves), int(grid)))

    def set_xz_config(self, scheme, waves=4, planes=0, grid=0):
        """z-marching x-line kernel (x-lines of up to 64 cells, items of rows by
        `planes` planes marched along z; 0 = the default) for Jacobi or chaotic GS."""
        _check(lib().bsi_set_xz_cfg(self.handle, _scheme(scheme), int(waves), int(planes), int(grid)))

    def set_pair(self, enable):
        """Chaotic GS on y/z lines with omega 1: two x-cells per lane (True, the
        default) or one line per lane with the in-tile correction solve."""
        _check(lib().bsi_set_pair(self.handle, 1 if enable else 0))

    def set_line_direct(self, enable):
        """Jacobi on y/z lines: the direct form M^{-1}(omega b + (1 - omega) M u)
        (True, the default) or u + omega M^{-1} r with u kept for the update."""
        _check(lib().bsi_set_line_direct(self.handle, 1 if enable else 0))

    def set_chaotic_chunk(self, tiles):
        """Tiles per even/odd chunk of the one-launch chaotic order (0: default)."""
        _check(lib().bsi_set_chaotic_chunk(self.handle, int(tiles)))

    def set_graphs(self, enable):
        _check(lib().bsi_set_graphs(self.handle, 1 if enable else 0))

    def line_relax_per_patch(self, axis, scheme, omega, nsweeps, u, f, work=None, stream=None):
        _check(lib().bsi_line_relax_per_patch(self.handle, int(axis), _scheme(scheme), float(omega), int(nsweeps),
                                             _ptr(u), _ptr(f), _ptr(work), _stream(stream)))


class Multigrid:
    """Owns a V-cycle object over a PatchSet (which must outlive it)."""

    def __init__(self, ps, kind, arg, scheme, omega, nu1=1, nu2=1, ncoarse=10, levels=0, coarse_bc=0):
        self.ps = ps
        self.handle = bs_mg_create(ps.handle, kind, arg, scheme, omega, nu1, nu2, ncoarse, levels, coarse_bc)
        self.levels = bs_mg_levels(self.handle)

    def vcycle(self, u, f, work=None, stream=None):
        bs_vcycle(self.handle, u, f, work, stream)

    def close(self):
        if self.handle is not None:
            bs_mg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --- differentiable smoother ---------------------------------------------------

class LineJacobiFn(torch.autograd.Function):
    """u_K = K damped Jacobi line sweeps along `axis` from (f, u0) with axis
    weights eps, differentiable in f, u0 (incl. face ghosts) and eps through
    the library's adjoint kernels, recomputing states from checkpoints taken
    every `ckpt` sweeps.

    apply(f, u0, eps, ps, axis, omega, K, ckpt): f and u0 in the patch set's
    f / u layouts (float64, on the device), eps a (npatch, 3) float64 tensor,
    ps a PatchSet whose eps is reset to `eps` when it differs."""

    @staticmethod
    def forward(ctx, f, u0, eps, ps, axis, omega, K, ckpt):
        _sync_eps(ps, eps)
        u = u0.detach().clone()
        # the forward keeps its checkpoints for the backward (workspace held
        # until then)
        nbytes = bs_backward_workspace_bytes(ps.handle, axis, K, ckpt)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=u0.device)
        bs_block_forward_ckpt(ps.handle, "line", axis, "jacobi", omega, K, ckpt, u, f.detach(), ws)
        ctx.save_for_backward(f, u0, eps)
        ctx.ws = ws
        ctx.cfg = (ps, int(axis), float(omega), int(K), int(ckpt))
        return u

    @staticmethod
    def backward(ctx, grad_uK):
        f, u0, eps = ctx.saved_tensors
        ps, axis, omega, K, ckpt = ctx.cfg
        _sync_eps(ps, eps)
        g_u0 = torch.zeros_like(u0)     # alignment gaps between patches stay 0
        g_f = torch.zeros_like(f)
        g_eps = torch.empty(ps.npatch * 3, dtype=torch.float64, device=u0.device)
        bs_block_backward_ckpt(ps.handle, "line", axis, "jacobi", omega, K, ckpt, f.detach(), grad_uK.contiguous(),
                               g_u0, g_f, g_eps, ctx.ws)
        ctx.ws = None
        return g_f, g_u0, g_eps.view(eps.shape).to(eps.device), None, None, None, None, None


class BlockSmoothFn(torch.autograd.Function):
    """u_K = K sweeps of line blocks (kind 'line', along axis) or plane blocks
    (kind 'plane', normal to axis) under 'jacobi' or 'colored' GS from (f, u0)
    with axis weights eps, differentiable in f, u0 (incl. face ghosts) and eps
    through the library's adjoint, recomputing states from checkpoints taken
    every `ckpt` sweeps.  Arguments as LineJacobiFn plus kind and scheme."""

    @staticmethod
    def forward(ctx, f, u0, eps, ps, kind, axis, scheme, omega, K, ckpt):
        _sync_eps(ps, eps)
        u = u0.detach().clone()
        # the forward keeps its checkpoints for the backward
        nbytes = bs_block_backward_workspace_bytes(ps.handle, kind, axis, scheme, K, ckpt)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=u0.device)
        bs_block_forward_ckpt(ps.handle, kind, axis, scheme, omega, K, ckpt, u, f.detach(), ws)
        ctx.save_for_backward(f, u0, eps)
        ctx.ws = ws
        ctx.cfg = (ps, kind, int(axis), scheme, float(omega), int(K), int(ckpt))
        return u

    @staticmethod
    def backward(ctx, grad_uK):
        f, u0, eps = ctx.saved_tensors
        ps, kind, axis, scheme, omega, K, ckpt = ctx.cfg
        _sync_eps(ps, eps)
        g_u0 = torch.zeros_like(u0)
        g_f = torch.zeros_like(f)
        g_eps = torch.empty(ps.npatch * 3, dtype=torch.float64, device=u0.device)
        bs_block_backward_ckpt(ps.handle, kind, axis, scheme, omega, K, ckpt, f.detach(), grad_uK.contiguous(),
                               g_u0, g_f, g_eps, ctx.ws)
        ctx.ws = None
        return g_f, g_u0, g_eps.view(eps.shape).to(eps.device), None, None, None, None, None, None, None


def block_smooth(f, u0, eps, ps, kind="line", axis=2, scheme="jacobi", omega=0.8, K=20, ckpt=5):
    """Differentiable K-sweep block smoother (see BlockSmoothFn)."""
    return BlockSmoothFn.apply(f, u0, eps, ps, kind, axis, scheme, omega, K, ckpt)


def _sync_eps(ps, eps):
    e = [tuple(float(v) for v in row) for row in eps.detach().cpu().reshape(-1, 3).tolist()]
    if e != ps.eps:
        ps.set_eps(e)


def line_jacobi(f, u0, eps, ps, axis=2, omega=0.8, K=20, ckpt=5):
    """Differentiable K-sweep damped Jacobi line smoother (see LineJacobiFn)."""
    return LineJacobiFn.apply(f, u0, eps, ps, axis, omega, K, ckpt)
