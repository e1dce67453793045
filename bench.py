#!/usr/bin/env python3
"""Benchmark of the line-block smoother on one MI355X.

Workload (one step): a 256^3 patch, eps = (1,1,100), h = 1/256, zero ghosts,
f, u0 ~ U[-1,1] (seed 2); 100 z-line block Jacobi sweeps (omega 0.8) and 100
chaotic z-line block Gauss-Seidel sweeps (omega 1), with the residual norm
taken every 10 sweeps.  value = interior cells x sweeps / wall time (GLUP/s).

Also reported: the roofline of the dominant kernel (a z-line sweep; bytes per
launch = 24 B/cell algorithmic: read u, read f, write u) from HIP events on
the launch stream, and the oracle timed on the host cores on a bounded sample.
Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per sweep (GLUP/s) + % HBM roofline; mixed/batched vs plain FP64"
HBM_PEAK_GBS = 8000.0
N = 256
EPS = (1.0, 1.0, 100.0)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle time for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the other configurations")
    ap.add_argument("--profile-c4", action="store_true",
                    help="fixed batched sequence for rocprofv3 (3000 AMR patches: 1 GiB copy, 3 x-line chaotic GS sweeps)")
    ap.add_argument("--profile-planes", action="store_true",
                    help="fixed plane-sweep sequence for rocprofv3 (512^3: FP64, FP32, BF16 refine 1 and 2; 2 sweeps each)")
    ap.add_argument("--cubes", action="store_true",
                    help="only the cube-block timings (64 patches of 64^3), printed as JSON")
    ap.add_argument("--profile-cubes", action="store_true",
                    help="fixed cube-block sequence for rocprofv3 (64 patches of 64^3: 1 GiB copy, then one "
                         "Jacobi sweep each with 8^3 and 4^3 blocks)")
    ap.add_argument("--profile-mg", action="store_true",
                    help="fixed multigrid sequence for rocprofv3 (three V-cycles of the multigrid form)")
    ap.add_argument("--profile", action="store_true",
                    help="for rocprofv3 counter runs: a 1 GiB device copy (reference for FETCH_SIZE / "
                         "WRITE_SIZE scaling), then 10 z-line Jacobi and 10 chaotic GS sweep launches; no JSON")
    return ap.parse_args()


def profile_run():
    """Fixed kernel sequence for counter collection: copy of known size, then sweeps."""
    import torch

    import paper_1208_1975_amd as bs
    from workloads import c2_patch

    torch.cuda.set_device(0)
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)   # 1 GiB
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    patch = c2_patch(N)
    ps = bs.PatchSet([patch.dims], [patch.eps], [patch.h])
    u = ps.pack_u([patch.u0])
    f = ps.pack_f([patch.f])
    work = ps.empty_u()
    uc = u.clone()
    torch.cuda.synchronize()
    ps.line_relax(2, "jacobi", 0.8, 10, u, f, work)
    ps.line_relax(2, "chaotic", 1.0, 10, uc, f)
    n2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    ps.residual(u, f, None, n2)
    torch.cuda.synchronize()
    print("profile run done", flush=True)


def profile_c4_run():
    """Fixed batched sequence for counters: a 1 GiB copy (scale), then the
    autotuner's trials and three x-line chaotic GS sweeps of the 3000-patch
    set in the configuration it picks, one launch each."""
    import torch

    import paper_1208_1975_amd as bs
    from workloads import c4_patchset

    torch.cuda.set_device(0)
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    s = c4_patchset()
    ps = bs.PatchSet([tuple(d) for d in s.dims], [tuple(e) for e in s.eps], list(s.h))
    u = ps.pack_u(s.u0)
    f = ps.pack_f(s.f)
    ps.autotune_line(0, "chaotic", u, f)
    torch.cuda.synchronize()
    print("profile c4 config %s" % json.dumps(ps.line_config(0, "chaotic")), flush=True)
    ps.set_graphs(False)
    for _ in range(3):
        ps.line_relax(0, "chaotic", 1.0, 1, u, f)
    torch.cuda.synchronize()
    print("profile c4 done", flush=True)


def profile_planes_run():
    """Fixed plane-sweep sequence for kernel traces: 512^3 xy-plane Jacobi,
    two sweeps each in FP64, FP32 (refine 0) and BF16 (refine 1 and 2)."""
    import torch

    import paper_1208_1975_amd as bs
    from workloads import c3_patch

    torch.cuda.set_device(0)
    p = c3_patch()
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    f = ps.pack_f([p.f])
    u0 = ps.pack_u([p.u0])
    w = ps.empty_u()
    for prec, refine in (("fp64", 0), ("fp32", 0), ("bf16", 1), ("bf16", 2)):
        u = u0.clone()
        ps.plane_relax(2, "jacobi", 1.0, 2, u, f, w, prec=prec, refine=refine)
        torch.cuda.synchronize()
        print("profile planes %s refine %d done" % (prec, refine), flush=True)
        del u


def profile_cubes_run():
    """Fixed cube-block sequence for kernel traces and counters."""
    import torch

    import paper_1208_1975_amd as bs
    from workloads import uniform_patchset

    torch.cuda.set_device(0)
    x = torch.empty(2 ** 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    y.copy_(x)
    torch.cuda.synchronize()
    s = uniform_patchset()
    ps = bs.PatchSet([tuple(d) for d in s.dims], [tuple(e) for e in s.eps], list(s.h))
    ps.set_graphs(False)
    u, f, w = ps.pack_u(s.u0), ps.pack_f(s.f), ps.empty_u()
    for blk in ((8, 8, 8), (4, 4, 4)):
        ps.cube_prepare(blk)
        ps.cube_relax(blk, "jacobi", 0.8, 1, u, f, w)
        torch.cuda.synchronize()
        print("profile cubes %s done" % (blk,), flush=True)


def profile_mg_run():
    """Fixed V-cycle sequence for kernel traces: the multigrid form's cycle
    (256^3, z-line two-colour GS with extrapolated faces), three cycles, the
    last two replayed from the captured graph."""
    import torch

    import paper_1208_1975_amd as bs
    from workloads import make_patch

    p = make_patch(256, 256, 256, (1.0, 1.0, 100.0), 1.0 / 256, seed=2, f="zero", u0="uniform")
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    ps.set_bc([63])
    mg = bs.Multigrid(ps, "line", 2, "colored", 1.0, 1, 1, 20, 0, 63)
    u, f = ps.pack_u([p.u0]), ps.pack_f([p.f])
    for c in range(3):
        mg.vcycle(u, f)
        torch.cuda.synchronize()
        print("profile mg cycle %d done" % c, flush=True)
    mg.close()
    ps.close()


def measured_traffic():
    """HBM bytes per launch of the z-line sweep kernel from the committed
    counter summary (FETCH_SIZE / WRITE_SIZE, scaled by a copy of known size),
    used only while the kernel sources are the ones the counters were taken on
    (SHA-256 of the listed files, concatenated in order)."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    prof = os.path.join(here, "profiles", "zline_256cube_hbm_counters.md")
    try:
        for ln in open(prof):
            if ln.startswith("traffic-json: "):
                t = json.loads(ln[len("traffic-json: "):])
                h = hashlib.sha256()
                for rel in t.get("sources", []):
                    h.update(open(os.path.join(here, rel), "rb").read())
                return t if t.get("sources") and t.get("source_sha256") == h.hexdigest() else None
    except OSError:
        return None
    return None


def timed_sweeps(fn, nsweeps_list, reps=5):
    """Median event time of fn(n) for each n (ms); events on the launch stream."""
    import torch
    out = {}
    for n in nsweeps_list:
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn(n)
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        ts.sort()
        out[n] = ts[len(ts) // 2]
    return out


def ev_ms(fn, reps=3):
    """Median HIP-event time (ms) of fn() on the current stream."""
    import torch
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def cube_forms(blocks=((2, 2, 2), (4, 2, 2), (4, 4, 2), (4, 4, 4), (8, 4, 4), (8, 8, 4), (8, 8, 8)), nsweeps=3):
    """Cube-block sweeps on 64 patches of 64^3 for the block sizes of the
    paper's study: ms per sweep, cells per second, and the block products'
    rate (2 nb flop per cell for blocks of nb cells)."""
    import paper_1208_1975_amd as bs
    from workloads import uniform_patchset

    s = uniform_patchset()
    ps = bs.PatchSet([tuple(d) for d in s.dims], [tuple(e) for e in s.eps], list(s.h))
    u0, f, w = ps.pack_u(s.u0), ps.pack_f(s.f), ps.empty_u()
    u = u0.clone()
    cells = s.cells()
    res = {}
    for blk in blocks:
        nb = blk[0] * blk[1] * blk[2]
        ps.cube_prepare(blk)
        for scheme, omega in (("jacobi", 0.8), ("chaotic", 1.0)):
            ps.cube_relax(blk, scheme, omega, nsweeps, u, f, w)   # capture the graph
            ms = ev_ms(lambda: ps.cube_relax(blk, scheme, omega, nsweeps, u, f, w), reps=5)
            per = ms / nsweeps
            res["%dx%dx%d_%s" % (blk + (scheme,))] = {
                "ms_per_sweep": round(per, 4), "glups": round(cells / (per * 1e-3) / 1e9, 3),
                "product_tflops": round(2.0 * nb * cells / (per * 1e-3) / 1e12, 2),
                "mfma_frac_fp64": round(2.0 * nb * cells / (per * 1e-3) / 78.6e12, 4),
                "hbm_frac_24B": round(24.0 * cells / (per * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}
            u.copy_(u0)
    ps.close()
    return res


def cube_convergence(n=64, long_sweeps=10000):
    """The block-size study (section 3) on the GPU: one 64^3 patch, eps = 1,
    f = 0, random initial guess, zero ghosts.  Relative residual after 3
    sweeps per block size and scheme, and the convergence factor
    (r_{2K} / r_K)^(1/K): Jacobi with K = long_sweeps / 2, the window starting
    near sweep 5000 as in the paper (point blocks: closed form
    1 - 1.6 sin^2(pi / (2 (n + 1)))); chaotic GS with half that K (it
    converges about twice as fast, so the residual stays far above rounding)."""
    import torch

    import paper_1208_1975_amd as bs
    from workloads import make_patch

    p = make_patch(n, n, n, (1.0, 1.0, 1.0), 1.0 / n, seed=8, f="zero", u0="uniform", ghosts="zero")
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    u0, f, w = ps.pack_u([p.u0]), ps.pack_f([p.f]), ps.empty_u()
    n2 = torch.zeros(1, dtype=torch.float64, device="cuda")

    def rnorm(u):
        ps.residual(u, f, None, n2)
        return math.sqrt(float(n2.item()))

    r0 = rnorm(u0)
    half = long_sweeps // 2
    res = {"closed_form_point_jacobi_factor": 1.0 - 1.6 * math.sin(math.pi / (2 * (n + 1))) ** 2}
    for b in ((1, 1, 1), (2, 2, 2), (4, 2, 2), (4, 4, 2), (4, 4, 4), (8, 4, 4), (8, 8, 4), (8, 8, 8)):
        ps.cube_prepare(b)
        e = {}
        for scheme, omega in (("jacobi", 0.8), ("chaotic", 1.0)):
            u = u0.clone()
            ps.cube_relax(b, scheme, omega, 3, u, f, w)
            e[scheme + "_rel_residual_3"] = round(rnorm(u) / r0, 6)
        for scheme, omega, k in (("jacobi", 0.8, half), ("chaotic", 1.0, half // 2)):
            u = u0.clone()
            ps.cube_relax(b, scheme, omega, k, u, f, w)
            ra = rnorm(u)
            ps.cube_relax(b, scheme, omega, k, u, f, w)
            e[scheme + "_factor"] = round((rnorm(u) / ra) ** (1.0 / k), 7)
        res["%dx%dx%d" % b] = e
    ps.close()
    return res


def forms():
    """The other configurations on the same GPU: timings, rates and errors."""
    import torch

    import paper_1208_1975_amd as bs
    from workloads import c1_patch, c2_patch, c3_patch, c4_patchset, c5_patch

    out = {}
    # 256^3 z-line Jacobi with the line solve in FP32 (FP64 residual and update)
    # against the FP64 form: 20 sweeps from the same state
    p = c2_patch(256)
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    u0, f, w = ps.pack_u([p.u0]), ps.pack_f([p.f]), ps.empty_u()
    res = {}
    u64 = None
    for prec in ("fp64", "fp32"):
        u = u0.clone()
        ps.line_relax(2, "jacobi", 0.8, 20, u, f, w, prec=prec)   # warm (graph capture)
        u.copy_(u0)
        ms = ev_ms(lambda: ps.line_relax(2, "jacobi", 0.8, 20, u, f, w, prec=prec), reps=1)
        entry = {"ms_per_sweep": round(ms / 20, 4), "glups": round(256 ** 3 * 20 / (ms * 1e-3) / 1e9, 3)}
        if prec == "fp64":
            u64 = u.clone()
        else:
            entry["relerr_vs_fp64_20_sweeps"] = float((u - u64).abs().max() / u64.abs().max())
        res[prec] = entry
        del u
    out["c2_zline_jacobi_line_solve_precision"] = res
    ps.close()
    del u0, f, w, u64

    # 32^3 x-line Jacobi, 10 sweeps (cache resident, launch bound)
    p = c1_patch()
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    u, f, w = ps.pack_u([p.u0]), ps.pack_f([p.f]), ps.empty_u()
    ps.line_relax(0, "jacobi", 1.0, 10, u, f, w)
    ms = ev_ms(lambda: ps.line_relax(0, "jacobi", 1.0, 10, u, f, w), reps=7)
    out["c1_xline_jacobi_32"] = {"ms_10_sweeps": round(ms, 4), "glups": round(32 ** 3 * 10 / (ms * 1e-3) / 1e9, 3)}
    ps.close()
    del u, f, w

    # 512^3 xy-plane Jacobi, the full 50 sweeps: FP64 fast diagonalisation vs
    # mixed forms; errors against the FP64 iterate and residual ratios every
    # 10 sweeps
    p = c3_patch()
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    f = ps.pack_f([p.f])
    u0 = ps.pack_u([p.u0])
    w = ps.empty_u()
    n2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    cells = 512 ** 3
    # four products per plane over 512 planes; the FP64 chain folds each about
    # the sine basis's even/odd symmetry (half of 2 n^3 per product and plane)
    flops = 4 * 512 ** 4 * 1.0
    res = {}
    u64, r64 = {}, {}
    for name, prec, refine in (("fp64", "fp64", 0), ("fp32", "fp32", 0), ("fp32_r1", "fp32", 1),
                               ("bf16", "bf16", 0), ("bf16_r1", "bf16", 1), ("bf16_r2", "bf16", 2)):
        u = u0.clone()
        ps.plane_relax(2, "jacobi", 1.0, 10, u, f, w, prec=prec, refine=refine)   # warm (tables, scratch, graph)
        u.copy_(u0)
        ms = 0.0
        errs, rrat = [], []
        for k in range(10, 51, 10):
            ms += ev_ms(lambda: ps.plane_relax(2, "jacobi", 1.0, 10, u, f, w, prec=prec, refine=refine), reps=1)
            ps.residual(u, f, None, n2)
            rk = math.sqrt(float(n2.item()))
            if name == "fp64":
                u64[k] = u.clone()
                r64[k] = rk
            else:
                errs.append(float((u - u64[k]).abs().max() / u64[k].abs().max()))
                rrat.append(round(rk / r64[k], 7))
        entry = {"ms_per_sweep": round(ms / 50, 3), "glups": round(cells * 50 / (ms * 1e-3) / 1e9, 3)}
        if name == "fp64":
            entry["mfma_tflops"] = round(flops * 50 / (ms * 1e-3) / 1e12, 2)
            entry["mfma_frac_fp64"] = round(flops * 50 / (ms * 1e-3) / 78.6e12, 4)
            entry["flop_per_sweep"] = flops
        else:
            entry["relerr_vs_fp64_at_sweeps_10_20_30_40_50"] = errs
            entry["residual_ratio_vs_fp64_at_sweeps_10_20_30_40_50"] = rrat
            if name == "bf16":
                entry["caveat"] = ("no error bound: the BF16 solve error (~3e-3) exceeds the 1.9e-5 stability "
                                   "margin of the z-checkerboard mode at omega 1, so the iteration is not a "
                                   "contraction")
        res[name] = entry
        del u
    out["c3_xyplane_jacobi_512_50_sweeps"] = res
    ps.close()
    del f, u0, w, u64
    torch.cuda.empty_cache()

    # 3000 uneven AMR patches, x-line chaotic GS, 20 sweeps
    s = c4_patchset()
    ps = bs.PatchSet([tuple(d) for d in s.dims], [tuple(e) for e in s.eps], list(s.h))
    u = ps.pack_u(s.u0)
    f = ps.pack_f(s.f)
    cells = s.cells()
    ps.autotune_line(0, "chaotic", u, f)
    ps.line_relax(0, "chaotic", 1.0, 20, u, f)                        # capture the graph
    ms_one = ev_ms(lambda: ps.line_relax(0, "chaotic", 1.0, 20, u, f), reps=3)
    ms_pp = ev_ms(lambda: ps.line_relax_per_patch(0, "chaotic", 1.0, 20, u, f), reps=1)
    out["c4_amr3000_xline_chaotic"] = {
        "cells": cells, "config": ps.line_config(0, "chaotic"),
        "one_graph_launch_ms": round(ms_one, 3), "glups": round(cells * 20 / (ms_one * 1e-3) / 1e9, 3),
        "hbm_frac": round((24.0 * cells * 20) / (ms_one * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
        "per_patch_launches_ms": round(ms_pp, 3), "launches_per_patch_path": 20 * 2 * s.npatch,
        "speedup_vs_per_patch": round(ms_pp / ms_one, 2)}
    # the same set with 4^3 cube blocks (every patch its own inverse): one fused
    # launch per colour pass for all 3000 patches, 20 chaotic sweeps
    t0 = time.time()
    ps.cube_prepare((4, 4, 4))
    prep_s = time.time() - t0
    ps.cube_relax((4, 4, 4), "chaotic", 1.0, 20, u, f)                 # capture the graph
    ms_c = ev_ms(lambda: ps.cube_relax((4, 4, 4), "chaotic", 1.0, 20, u, f), reps=3)
    out["c4_amr3000_cube4_chaotic"] = {
        "cells": cells, "prepare_s": round(prep_s, 3), "ms_20_sweeps": round(ms_c, 3),
        "glups": round(cells * 20 / (ms_c * 1e-3) / 1e9, 3),
        "hbm_frac": round((24.0 * cells * 20) / (ms_c * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}
    ps.close()
    del u, f
    torch.cuda.empty_cache()

    out["c4_adjacent_2940_xline_chaotic_exchange"] = exchange_form()
    torch.cuda.empty_cache()
    out["mg_vcycle_256_zline"] = mg_form()
    torch.cuda.empty_cache()

    # geometric cube blocks (the paper's own block kind) on the block-size
    # study's 64 patches of 64^3, eps = 1: 3 sweeps per block size and scheme
    out["cube_blocks_64x64cube"] = cube_forms()
    out["cube_block_size_study_64"] = cube_convergence()
    torch.cuda.empty_cache()

    # 128^3 differentiable smoother: K = 20 z-line Jacobi, checkpoint every 5
    p = c5_patch()
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    u0, f, w = ps.pack_u([p.u0]), ps.pack_f([p.f]), ps.empty_u()
    u = u0.clone()
    ps.line_relax(2, "jacobi", 0.8, 20, u, f, w)                       # capture the graph
    ms_f = ev_ms(lambda: (u.copy_(u0), ps.line_relax(2, "jacobi", 0.8, 20, u, f, w)), reps=5)
    g = torch.randn_like(u0)
    nbytes = bs.bs_backward_workspace_bytes(ps.handle, 2, 20, 5)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    gu0, gf = torch.zeros_like(u0), torch.zeros_like(f)
    geps = torch.zeros(3, dtype=torch.float64, device="cuda")
    bwd = lambda: bs.bs_relax_backward(ps.handle, 2, 0.8, 20, 5, u0, f, g, gu0, gf, geps, ws)
    bwd()
    ms_b = ev_ms(bwd, reps=5)
    # the autograd form: the forward keeps its checkpoints, the backward starts from them
    fwd_c = lambda: (u.copy_(u0), bs.bs_block_forward_ckpt(ps.handle, "line", 2, "jacobi", 0.8, 20, 5, u, f, ws))
    fwd_c()
    ms_fc = ev_ms(fwd_c, reps=5)
    bwd_c = lambda: bs.bs_block_backward_ckpt(ps.handle, "line", 2, "jacobi", 0.8, 20, 5, f, g, gu0, gf, geps, ws)
    bwd_c()
    ms_bc = ev_ms(bwd_c, reps=5)
    cells = 128 ** 3
    out["c5_adjoint_128_K20"] = {"forward_ms": round(ms_f, 3), "backward_ms": round(ms_b, 3),
                                 "backward_over_forward": round(ms_b / ms_f, 2),
                                 "forward_keeping_checkpoints_ms": round(ms_fc, 3),
                                 "backward_from_checkpoints_ms": round(ms_bc, 3),
                                 "backward_from_checkpoints_over_forward": round(ms_bc / ms_f, 2),
                                 "forward_glups": round(cells * 20 / (ms_f * 1e-3) / 1e9, 3),
                                 "workspace_MiB": round(nbytes / 2 ** 20, 1)}
    ps.close()
    return out


def exchange_form():
    """The adjacent version of the uneven AMR set (2940 patches tiling a box face
    to face): 20 x-line chaotic GS sweeps in one graph launch with the ghost
    exchange after every sweep, against the same sweeps without links, and the
    exchange alone (its share of the smoothing step)."""
    import torch

    import paper_1208_1975_amd as bs
    from workloads import c4_adjacent_patchset

    s = c4_adjacent_patchset()
    ps = bs.PatchSet(s.dims, s.eps, s.h)
    u0, f = ps.pack_u(s.u0), ps.pack_f(s.f)
    u = u0.clone()
    cells = s.cells()
    ps.autotune_line(0, "chaotic", u, f)
    ps.line_relax(0, "chaotic", 1.0, 20, u, f)                          # capture
    ms_plain = ev_ms(lambda: ps.line_relax(0, "chaotic", 1.0, 20, u, f), reps=3)
    ps.set_links(s.links)
    u.copy_(u0)
    ps.line_relax(0, "chaotic", 1.0, 20, u, f)                          # capture with the exchange
    ms_x = ev_ms(lambda: ps.line_relax(0, "chaotic", 1.0, 20, u, f), reps=3)
    ps.exchange_ghosts(u)
    ms_e = ev_ms(lambda: [ps.exchange_ghosts(u) for _ in range(20)], reps=3)
    ghost_cells = 2 * sum(int(s.dims[a][(ax + 1) % 3]) * int(s.dims[a][(ax + 2) % 3]) for a, ax, _ in s.links)
    res = {"patches": int(s.npatch), "links": len(s.links), "cells": int(cells), "exchanged_ghost_cells": ghost_cells,
           "ms_20_sweeps_with_exchange": round(ms_x, 3), "ms_20_sweeps_without": round(ms_plain, 3),
           "ms_20_exchanges_alone": round(ms_e, 3),
           "exchange_share_of_step": round((ms_x - ms_plain) / ms_x, 4),
           "glups_with_exchange": round(cells * 20 / (ms_x * 1e-3) / 1e9, 3),
           "exchange_GBs": round(16.0 * ghost_cells * 20 / (ms_e * 1e-3) / 1e9, 1)}
    ps.close()
    return res


def mg_form():
    """One V(1,1) cycle with z-line two-colour GS smoothing on the 256^3
    eps (1,1,100) patch with extrapolated faces on every level: time per cycle
    and the residual reduction per cycle (f = 0, random initial guess)."""
    import torch

    import paper_1208_1975_amd as bs
    from workloads import make_patch

    p = make_patch(256, 256, 256, (1.0, 1.0, 100.0), 1.0 / 256, seed=2, f="zero", u0="uniform")
    ps = bs.PatchSet([p.dims], [p.eps], [p.h])
    ps.set_bc([63])
    mg = bs.Multigrid(ps, "line", 2, "colored", 1.0, 1, 1, 20, 0, 63)
    u0, f = ps.pack_u([p.u0]), ps.pack_f([p.f])
    u = u0.clone()
    n2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    rs = []
    for _ in range(8):
        ps.residual(u, f, None, n2)
        rs.append(math.sqrt(float(n2.item())))
        mg.vcycle(u, f)
    ms = ev_ms(lambda: mg.vcycle(u, f), reps=5)
    # a cycle smooths each level twice (coarsest: 20 sweeps): fine-grid sweep equivalents
    fine_eq = sum(2.0 / 8 ** l for l in range(mg.levels - 1)) + 20.0 / 8 ** (mg.levels - 1)
    res = {"levels": int(mg.levels), "ms_per_cycle": round(ms, 3),
           "residual_factor_per_cycle": [round(rs[i + 1] / rs[i], 4) for i in range(len(rs) - 1)],
           "fine_sweep_equivalents_per_cycle": round(fine_eq, 3),
           "glups_equivalent": round(256 ** 3 * fine_eq / (ms * 1e-3) / 1e9, 2)}
    mg.close()
    ps.close()
    return res


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(patch, target_s):
    """The oracle on the host: z-line Jacobi + lexicographic GS sweep pairs of
    the full grid, at the default thread count and at 1 thread, median of 3
    timed runs each; target_s bounds the whole measurement."""
    import oracle
    cells = patch.f.size
    runs = {}
    for label, nt, share in (("all", 0, 0.45), ("one", 1, 0.55)):
        oracle.set_threads(nt)
        threads = oracle.get_threads()
        t0 = time.perf_counter()
        u = oracle.line_sweeps(patch.u0, patch.f, patch.eps, patch.h, 2, oracle.JACOBI, 0.8, 1)
        u = oracle.line_sweeps(patch.u0, patch.f, patch.eps, patch.h, 2, oracle.LEX_GS, 1.0, 1, lex_form=1)
        per_pair = time.perf_counter() - t0
        k = max(1, int(target_s * share / 3 / per_pair))
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            u = oracle.line_sweeps(patch.u0, patch.f, patch.eps, patch.h, 2, oracle.JACOBI, 0.8, k)
            u = oracle.line_sweeps(patch.u0, patch.f, patch.eps, patch.h, 2, oracle.LEX_GS, 1.0, k, lex_form=1)
            ts.append(time.perf_counter() - t0)
        del u
        ts.sort()
        runs[label] = {"threads": threads, "pairs": k, "median_s": ts[1], "glups": cells * 2 * k / ts[1] / 1e9}
    oracle.set_threads(0)
    a, o = runs["all"], runs["one"]
    return {"value": round(a["glups"], 5), "unit": "GLUP/s", "cores": a["threads"], "kind": "oracle",
            "value_1_thread": round(o["glups"], 5), "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": "%d^3 z-lines, eps (1,1,100): %d Jacobi + %d lexicographic GS sweeps (anti-diagonal form) "
                      "of the full grid, median of 3 runs (%.2f s) at %d threads; %d + %d sweeps, median of 3 "
                      "(%.2f s) at 1 thread" % (N, a["pairs"], a["pairs"], a["median_s"], a["threads"], o["pairs"],
                                                o["pairs"], o["median_s"])}


def stream_ceiling(n, reps=7):
    """Measured streaming ceiling (GB/s) for 24 bytes per element over n
    doubles per operand (the size of one sweep's u, f and v): the library's
    triad probe, plain and with nontemporal loads of the second operand."""
    import torch

    import paper_1208_1975_amd as bs
    n += n & 1
    a = torch.rand(n, dtype=torch.float64, device="cuda")
    b = torch.rand(n, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    out = {}
    for mode, name in ((0, "triad"), (1, "triad_nontemporal")):
        bs.stream_triad(a, b, c, mode)
        ms = ev_ms(lambda: bs.stream_triad(a, b, c, mode), reps=reps)
        out[name + "_GBs"] = round(24.0 * n / (ms * 1e-3) / 1e9, 1)
    del a, b, c
    return out


def main():
    args = parse()
    if args.profile_planes:
        profile_planes_run()
        return
    if args.profile_c4:
        profile_c4_run()
        return
    if args.profile_cubes:
        profile_cubes_run()
        return
    if args.profile_mg:
        profile_mg_run()
        return
    if args.cubes:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"timings": cube_forms(), "block_size_study": cube_convergence()}), flush=True)
        return
    if args.profile:
        profile_run()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU; --gpus %d is not supported" % args.gpus)
        sys.exit(2)

    import torch

    import paper_1208_1975_amd as bs
    from workloads import c2_patch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU")
        sys.exit(1)
    torch.cuda.set_device(0)
    patch = c2_patch(N)
    ps = bs.PatchSet([patch.dims], [patch.eps], [patch.h])
    u0 = ps.pack_u([patch.u0])
    f = ps.pack_f([patch.f])
    uj = u0.clone()
    uc = u0.clone()
    work = ps.empty_u()
    norms = torch.zeros(20, dtype=torch.float64, device="cuda")
    cells = N ** 3
    sweeps_per_step = 200

    def step():
        for blk in range(10):
            ps.line_relax(2, "jacobi", 0.8, 10, uj, f, work)
            ps.residual(uj, f, None, norms[blk:blk + 1])
        for blk in range(10):
            ps.line_relax(2, "chaotic", 1.0, 10, uc, f)
            ps.residual(uc, f, None, norms[10 + blk:11 + blk])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    value = cells * sweeps_per_step * args.steps / dt / 1e9

    # per-launch kernel time from the difference of two sweep counts (removes fixed costs)
    tj = timed_sweeps(lambda n: ps.line_relax(2, "jacobi", 0.8, n, uj, f, work), (10, 40))
    tc = timed_sweeps(lambda n: ps.line_relax(2, "chaotic", 1.0, n, uc, f), (10, 40))
    jac_us = (tj[40] - tj[10]) / 30 * 1e3
    cha_us = (tc[40] - tc[10]) / 30 * 1e3
    bytes_per_launch = 24.0 * cells
    dom_name, dom_us = ("z-line Jacobi sweep", jac_us) if jac_us >= cha_us else ("z-line chaotic GS sweep", cha_us)
    achieved = bytes_per_launch / (dom_us * 1e-6) / 1e9
    mt = measured_traffic()
    traffic = None
    if mt is not None:
        k = "jacobi" if dom_name.startswith("z-line Jacobi") else "chaotic"
        traffic = mt[k + "_read_bytes"] + mt[k + "_write_bytes"]
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": dom_name, "us_per_launch": round(dom_us, 2),
            "bytes_per_launch": bytes_per_launch,
            "other": {"jacobi_us": round(jac_us, 2), "chaotic_us": round(cha_us, 2),
                      "jacobi_frac": round(bytes_per_launch / (jac_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                      "chaotic_frac": round(bytes_per_launch / (cha_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}}
    rn = norms.cpu().numpy()
    ceil = stream_ceiling(cells)
    best = max(ceil.values())
    roof["measured_ceiling"] = dict(ceil, frac_of_measured=round(achieved / best, 4),
                                    note="triad c = a + b over %d doubles per operand on this GPU" % cells)

    ps.close()
    del uj, uc, u0, f, work
    torch.cuda.empty_cache()
    other = None if args.no_forms else forms()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(patch, args.cpu_seconds)

    line = {"metric": METRIC, "value": round(value, 3), "unit": "GLUP/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "256^3 patch, eps (1,1,100): 100 z-line block Jacobi sweeps (omega 0.8) + "
                                   "100 chaotic z-line block GS sweeps (omega 1), residual norm every 10 sweeps",
                       "cells": cells, "sweeps_per_step": sweeps_per_step, "parallelism": "single GPU"},
            "roofline": roof, "cpu_baseline": cpu,
            "residual_last": {"jacobi": float(math.sqrt(rn[9])), "chaotic": float(math.sqrt(rn[19]))},
            "forms": other}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
