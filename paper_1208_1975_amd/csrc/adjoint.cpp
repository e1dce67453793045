// Backward of K damped Jacobi or two-colour GS sweeps of line or plane blocks
// with checkpointing: states at sweeps 0, c, 2c, ... are kept (taken here, or
// left in the workspace by a forward call that keeps them, so that the
// backward need not run the forward again); each segment
// is recomputed forward and then walked in reverse, one half-step at a time
// (a Jacobi sweep is one half-step over all blocks, a two-colour sweep colour
// 0 then colour 1, undone colour 1 first), with the adjoint step of
// k_adjoint.hip.  Its two block solves, w = P M^{-1} r(U) and
// lambda = M^{-1} P gbar, reuse the line kernels (solve-only output, right-hand
// side from a field) or the plane chain.
#include <algorithm>

#include "patchset.h"
#include "relax.h"

namespace bs {

namespace {

struct BackwardPlan {
    int ncp = 0, nseg = 0;       // checkpoints, recomputed states per segment
    int nw = 0;                  // the recomputed sweeps' corrections w (Jacobi on y/z lines)
    int extra = 0;               // lambda, w, gbar, plus the mid-sweep state of two-colour GS
    size_t state_bytes = 0;      // one u-layout buffer, 256-byte aligned
    size_t acc_bytes = 0;
    size_t total = 0;
};

// Jacobi on y/z lines recomputes each segment with sweeps that also write
// their correction w = M^{-1} r(U), so the reverse steps need no w solve but
// the segment's last.
bool keeps_w(int kind, int axis, bool gs)
{
    return kind == 0 && axis != 0 && !gs;
}

BackwardPlan plan_backward(const bs_patchset *ps, int K, int c, bool gs, bool keep_w)
{
    BackwardPlan b;
    b.ncp = K > 0 ? (K + c - 1) / c : 1;
    b.nseg = std::max(0, std::min(c, K) - 1);
    b.nw = keep_w ? b.nseg : 0;
    b.extra = gs ? 4 : 3;
    b.state_bytes = (static_cast<size_t>(ps->u_numel) * sizeof(double) + 255) / 256 * 256;
    b.acc_bytes = (static_cast<size_t>(ps->nrtiles) * 3 * sizeof(double) + 255) / 256 * 256;
    b.total = static_cast<size_t>(b.ncp + b.nseg + b.nw + b.extra) * b.state_bytes + b.acc_bytes;
    return b;
}

bs_status check_backward(const bs_patchset *ps, int32_t kind, int32_t axis, bs_scheme scheme, int32_t nsweeps,
                         int32_t ckpt_every, const char *fn)
{
    if (kind != 0 && kind != 1) return fail(BS_ERR_INVALID, "%s: kind must be 0 (lines) or 1 (planes)", fn);
    if (axis < 0 || axis > 2) return fail(BS_ERR_INVALID, "%s: axis must be 0, 1 or 2", fn);
    if (nsweeps < 0 || ckpt_every < 1) return fail(BS_ERR_INVALID, "%s: bad nsweeps or ckpt_every", fn);
    if (scheme != BS_JACOBI && scheme != BS_COLORED_GS && scheme != BS_CHAOTIC_GS)
        return fail(BS_ERR_INVALID, "%s: unknown scheme", fn);
    if (scheme == BS_CHAOTIC_GS)
        return fail(BS_ERR_UNSUPPORTED, "%s: chaotic GS has no unique forward map to differentiate", fn);
    if (!ps) return fail(BS_ERR_INVALID, "%s: null patch set", fn);
    return BS_OK;
}

// What one call of block_adjoint does.
enum class AdjMode {
    full,       // forward to the checkpoints, then the reverse pass
    forward,    // only the forward: u0 -> u_K, checkpoints left in the workspace
    reverse     // only the reverse pass, from checkpoints a forward call left
};

}  // namespace

}  // namespace bs

using namespace bs;

namespace {

// u: u0 (full mode), u0 in / u_K out (forward mode), unused (reverse mode).
bs_status block_adjoint(AdjMode mode, const char *fn, bs_patchset *ps, int32_t kind, int32_t axis, bs_scheme scheme,
                        double omega, int32_t nsweeps, int32_t ckpt_every, double *u, const double *f,
                        const double *grad_uK, double *grad_u0, double *grad_f, double *grad_eps, void *workspace,
                        size_t workspace_bytes, hipStream_t stream)
{
    bs_status st = check_backward(ps, kind, axis, scheme, nsweeps, ckpt_every, fn);
    if (st != BS_OK) return st;
    if (!(omega > 0.0 && omega < 2.0)) return fail(BS_ERR_INVALID, "%s: omega must be in (0, 2)", fn);
    if (!f || (mode != AdjMode::reverse && !u) || (mode != AdjMode::forward && !grad_uK))
        return fail(BS_ERR_INVALID, "%s: null argument", fn);
    if (!workspace) return fail(BS_ERR_INVALID, "%s: null workspace", fn);
    if (ghost_active(ps)) return fail(BS_ERR_UNSUPPORTED, "%s: patch sets with links or extrapolated faces", fn);
    const bool gs = scheme == BS_COLORED_GS;
    const bool keep_w = keeps_w(kind, axis, gs);
    const BackwardPlan bp = plan_backward(ps, nsweeps, ckpt_every, gs, keep_w);
    if (workspace_bytes < bp.total)
        return fail(BS_ERR_INVALID, "%s: workspace of %zu bytes, needs %zu", fn, workspace_bytes, bp.total);
    const double *u0 = u;
    LineCfg cj, cc;
    if (kind == 0) {
        if ((st = check_line_ps_ext(ps, axis, fn)) != BS_OK) return st;
        cj = line_cfg(ps, axis, 0);
        cc = line_cfg(ps, axis, 1);
        // most line passes here are block solves, not direct-form sweeps (and
        // the z-marching x-line form runs plain sweeps only)
        if (cj.deflt || cj.form == 2) cj = default_line_cfg(ps, axis, 0, false);
        if ((st = check_line_cfg(ps, axis, cj)) != BS_OK) return st;
        if ((st = check_line_cfg(ps, axis, cc)) != BS_OK) return st;
        if ((st = prepare_lists(ps, axis, cj, 0)) != BS_OK) return st;
        if ((st = prepare_lists(ps, axis, cc, 1)) != BS_OK) return st;
        hipError_t e = prepare_line_kernels();
        if (e != hipSuccess) return hip_fail(e, "line kernel attributes");
    } else {
        for (int a = 0; a < 3; ++a)
            if (a != axis && ps->max_n[a] > 1024) return fail(BS_ERR_UNSUPPORTED, "%s: an in-plane edge exceeds 1024", fn);
    }

    // carve the workspace
    char *wsp = static_cast<char *>(workspace);
    std::vector<double *> ckpt(bp.ncp), seg(bp.nseg), wseg(bp.nw);
    for (int i = 0; i < bp.ncp; ++i, wsp += bp.state_bytes) ckpt[i] = reinterpret_cast<double *>(wsp);
    for (int i = 0; i < bp.nseg; ++i, wsp += bp.state_bytes) seg[i] = reinterpret_cast<double *>(wsp);
    for (int i = 0; i < bp.nw; ++i, wsp += bp.state_bytes) wseg[i] = reinterpret_cast<double *>(wsp);
    double *lam = reinterpret_cast<double *>(wsp);
    wsp += bp.state_bytes;
    double *w = reinterpret_cast<double *>(wsp);
    wsp += bp.state_bytes;
    double *gbar_ws = reinterpret_cast<double *>(wsp);
    wsp += bp.state_bytes;
    double *mid = nullptr;   // two-colour GS: the state after a sweep's colour-0 half-step
    if (gs) {
        mid = reinterpret_cast<double *>(wsp);
        wsp += bp.state_bytes;
    }
    double *acc = reinterpret_cast<double *>(wsp);
    double *gbar = grad_u0 ? grad_u0 : gbar_ws;

    const PatchDesc *pdd = static_cast<const PatchDesc *>(ps->desc_d.p);
    const ResidTile *tiles = static_cast<const ResidTile *>(ps->rtile_d.p);
    const int32_t *pfirst = static_cast<const int32_t *>(ps->rtile_first_d.p);
    const int spans = kind == 0 ? (1 << axis) : (7 & ~(1 << axis));
    auto chk = [&](hipError_t err, const char *what) -> bs_status {
        return err == hipSuccess ? BS_OK : hip_fail(err, what);
    };
    // one half-step in place on x (colour -1: a Jacobi step src -> dst)
    auto half = [&](int colour, const double *src, double *dst) -> bs_status {
        if (kind == 1) return plane_step(ps, axis, colour, src, dst, f, omega, stream);
        if (colour < 0) return line_pass(ps, axis, cj, 0, 0, src, dst, f, omega, stream, -1, 0, 0);
        return line_pass(ps, axis, cc, 1, colour, src, dst, f, omega, stream, -1, 0, 0);
    };
    // one sweep src -> dst (dst carries u0's ghosts)
    auto sweep = [&](const double *src, double *dst) -> bs_status {
        if (!gs) return half(-1, src, dst);
        bs_status s2 = chk(launch_interior_copy(src, dst, pdd, ps->npatch, stream), "copy");
        if (s2 == BS_OK) s2 = half(0, dst, dst);
        if (s2 == BS_OK) s2 = half(1, dst, dst);
        return s2;
    };
    // out = M^{-1} P rhs on colour's blocks, rhs = r(src) (with f) or src
    auto solve = [&](int colour, const double *src, bool residual, double *out) -> bs_status {
        if (kind == 1) return plane_solve(ps, axis, colour, src, residual ? f : nullptr, out, stream);
        const int cm = colour < 0 ? 0 : 1;
        return line_pass(ps, axis, cm ? cc : cj, cm, cm ? colour : 0, src, out, f, omega, stream, -1,
                         residual ? 0 : 1, 1);
    };
    // the reverse of one half-step from state U for colour (-1: all blocks);
    // wk: U's correction w when a recomputing sweep kept it
    auto reverse = [&](int colour, const double *U, const double *wk) -> bs_status {
        bs_status s2;
        // blocks of the other colour (and every ghost) must read zero in lambda;
        // w only matters on the half-step's blocks (the planes' solve adds into it)
        if (colour >= 0 || kind == 1) {
            if ((s2 = chk(launch_fill(lam, ps->u_numel, 0.0, stream), "fill")) != BS_OK) return s2;
            if (kind == 1 && (s2 = chk(launch_fill(w, ps->u_numel, 0.0, stream), "fill")) != BS_OK) return s2;
        }
        if (!wk) {
            if ((s2 = solve(colour, U, true, w)) != BS_OK) return s2;
            wk = w;
        }
        if ((s2 = solve(colour, gbar, false, lam)) != BS_OK) return s2;
        return chk(launch_adj_step(lam, U, wk, gbar, grad_f, acc, pdd, tiles, ps->nrtiles, spans, omega, stream),
                   "adjoint step");
    };

    if (mode != AdjMode::reverse) {
        // every state buffer carries u0's ghosts; checkpoint 0 is u0
        for (double *bf : ckpt)
            if ((st = chk(launch_ghost_copy(u0, bf, pdd, ps->npatch, stream), "ghost copy")) != BS_OK) return st;
        for (double *bf : seg)
            if ((st = chk(launch_ghost_copy(u0, bf, pdd, ps->npatch, stream), "ghost copy")) != BS_OK) return st;
        if (mid && (st = chk(launch_ghost_copy(u0, mid, pdd, ps->npatch, stream), "ghost copy")) != BS_OK) return st;
        if ((st = chk(launch_interior_copy(u0, ckpt[0], pdd, ps->npatch, stream), "copy")) != BS_OK) return st;
        // forward: checkpoints at sweeps c, 2c, ...
        for (int s = 0; s + 1 < bp.ncp; ++s) {
            const double *src = ckpt[s];
            for (int j = 1; j <= ckpt_every; ++j) {
                double *dst = j == ckpt_every ? ckpt[s + 1] : seg[j - 1];
                if ((st = sweep(src, dst)) != BS_OK) return st;
                src = dst;
            }
        }
    }
    if (mode == AdjMode::forward) {
        // the sweeps after the last checkpoint, the last one into u
        const int rest = nsweeps - (bp.ncp - 1) * ckpt_every;
        const double *src = ckpt[bp.ncp - 1];
        for (int j = 1; j <= rest; ++j) {
            double *dst = j == rest ? u : seg[j - 1];
            if ((st = sweep(src, dst)) != BS_OK) return st;
            src = dst;
        }
        return BS_OK;
    }
    // adjoint state (lambda and w start at zero, ghosts included)
    if ((st = chk(launch_fill(lam, ps->u_numel, 0.0, stream), "fill")) != BS_OK) return st;
    if ((st = chk(launch_fill(w, ps->u_numel, 0.0, stream), "fill")) != BS_OK) return st;
    for (double *bf : wseg)
        if ((st = chk(launch_fill(bf, ps->u_numel, 0.0, stream), "fill")) != BS_OK) return st;
    if ((st = chk(launch_fill(acc, static_cast<int64_t>(ps->nrtiles) * 3, 0.0, stream), "fill")) != BS_OK) return st;
    if (grad_f && (st = chk(launch_fill(grad_f, ps->f_numel, 0.0, stream), "fill")) != BS_OK) return st;
    if ((st = chk(launch_adj_init(grad_uK, gbar, pdd, ps->npatch, stream), "adjoint init")) != BS_OK) return st;
    // reverse, one segment at a time
    for (int s = bp.ncp - 1; s >= 0; --s) {
        const int k0 = s * ckpt_every, k1 = std::min(nsweeps, k0 + ckpt_every);
        for (int j = 1; j < k1 - k0; ++j) {
            const double *src = j == 1 ? ckpt[s] : seg[j - 2];
            // state k0 + j, and (keep_w) the correction of state k0 + j - 1
            st = keep_w ? line_pass(ps, axis, cj, 0, 0, src, seg[j - 1], f, omega, stream, -1, 0, 2, 0, wseg[j - 1])
                        : sweep(src, seg[j - 1]);
            if (st != BS_OK) return st;
        }
        for (int k = k1 - 1; k >= k0; --k) {
            const double *Uk = k == k0 ? ckpt[s] : seg[k - k0 - 1];
            if (!gs) {
                const double *wk = (keep_w && k < k1 - 1) ? wseg[k - k0] : nullptr;
                if ((st = reverse(-1, Uk, wk)) != BS_OK) return st;
                continue;
            }
            // the mid-sweep state, then colour 1 undone before colour 0
            if ((st = chk(launch_interior_copy(Uk, mid, pdd, ps->npatch, stream), "copy")) != BS_OK) return st;
            if ((st = half(0, mid, mid)) != BS_OK) return st;
            if ((st = reverse(1, mid, nullptr)) != BS_OK) return st;
            if ((st = reverse(0, Uk, nullptr)) != BS_OK) return st;
        }
    }
    if (grad_eps && (st = chk(launch_eps_final(acc, pfirst, ps->npatch, omega, grad_eps, stream), "eps reduce")) != BS_OK)
        return st;
    return BS_OK;
}

}  // namespace

extern "C" {

size_t bs_block_backward_workspace_bytes(const bs_patchset *ps, int32_t kind, int32_t axis, bs_scheme scheme,
                                         int32_t nsweeps, int32_t ckpt_every)
{
    if (!ps || (kind != 0 && kind != 1) || axis < 0 || axis > 2 || nsweeps < 0 || ckpt_every < 1) return 0;
    if (scheme != BS_JACOBI && scheme != BS_COLORED_GS) return 0;
    const bool gs = scheme == BS_COLORED_GS;
    return plan_backward(ps, nsweeps, ckpt_every, gs, keeps_w(kind, axis, gs)).total;
}

size_t bs_backward_workspace_bytes(const bs_patchset *ps, int32_t axis, int32_t nsweeps, int32_t ckpt_every)
{
    return bs_block_backward_workspace_bytes(ps, 0, axis, BS_JACOBI, nsweeps, ckpt_every);
}

bs_status bs_block_backward(bs_patchset *ps, int32_t kind, int32_t axis, bs_scheme scheme, double omega,
                            int32_t nsweeps, int32_t ckpt_every, const double *u0, const double *f,
                            const double *grad_uK, double *grad_u0, double *grad_f, double *grad_eps,
                            void *workspace, size_t workspace_bytes, hipStream_t stream)
{
    return block_adjoint(AdjMode::full, "bs_block_backward", ps, kind, axis, scheme, omega, nsweeps, ckpt_every,
                         const_cast<double *>(u0), f, grad_uK, grad_u0, grad_f, grad_eps, workspace, workspace_bytes,
                         stream);
}

bs_status bs_block_forward_ckpt(bs_patchset *ps, int32_t kind, int32_t axis, bs_scheme scheme, double omega,
                                int32_t nsweeps, int32_t ckpt_every, double *u, const double *f, void *workspace,
                                size_t workspace_bytes, hipStream_t stream)
{
    return block_adjoint(AdjMode::forward, "bs_block_forward_ckpt", ps, kind, axis, scheme, omega, nsweeps,
                         ckpt_every, u, f, nullptr, nullptr, nullptr, nullptr, workspace, workspace_bytes, stream);
}

bs_status bs_block_backward_ckpt(bs_patchset *ps, int32_t kind, int32_t axis, bs_scheme scheme, double omega,
                                 int32_t nsweeps, int32_t ckpt_every, const double *f, const double *grad_uK,
                                 double *grad_u0, double *grad_f, double *grad_eps, void *workspace,
                                 size_t workspace_bytes, hipStream_t stream)
{
    return block_adjoint(AdjMode::reverse, "bs_block_backward_ckpt", ps, kind, axis, scheme, omega, nsweeps,
                         ckpt_every, nullptr, f, grad_uK, grad_u0, grad_f, grad_eps, workspace, workspace_bytes,
                         stream);
}

bs_status bs_relax_backward(bs_patchset *ps, int32_t axis, double omega, int32_t nsweeps, int32_t ckpt_every,
                            const double *u0, const double *f, const double *grad_uK, double *grad_u0,
                            double *grad_f, double *grad_eps, void *workspace, size_t workspace_bytes,
                            hipStream_t stream)
{
    return bs_block_backward(ps, 0, axis, BS_JACOBI, omega, nsweeps, ckpt_every, u0, f, grad_uK, grad_u0, grad_f,
                             grad_eps, workspace, workspace_bytes, stream);
}

}  // extern "C"
