// Backward of K damped Jacobi line sweeps with checkpointing: states at
// sweeps 0, c, 2c, ... are kept; each segment is recomputed forward and then
// walked in reverse with the adjoint step (k_adjoint.hip), whose two block
// solves (w = M^{-1} r(U^k) and lambda = M^{-1} gbar) reuse the line kernels.
#include <algorithm>

#include "patchset.h"
#include "relax.h"

namespace bs {

namespace {

struct BackwardPlan {
    int ncp = 0, nseg = 0;       // checkpoints, recomputed states per segment
    size_t state_bytes = 0;      // one u-layout buffer, 256-byte aligned
    size_t acc_bytes = 0;
    size_t total = 0;
};

BackwardPlan plan_backward(const bs_patchset *ps, int K, int c)
{
    BackwardPlan b;
    b.ncp = K > 0 ? (K + c - 1) / c : 1;
    b.nseg = std::max(0, std::min(c, K) - 1);
    b.state_bytes = (static_cast<size_t>(ps->u_numel) * sizeof(double) + 255) / 256 * 256;
    b.acc_bytes = (static_cast<size_t>(ps->nrtiles) * 3 * sizeof(double) + 255) / 256 * 256;
    // checkpoints + segment states + lambda + w + gbar (when grad_u0 is not given) + accumulators
    b.total = static_cast<size_t>(b.ncp + b.nseg + 3) * b.state_bytes + b.acc_bytes;
    return b;
}

}  // namespace

}  // namespace bs

using namespace bs;

extern "C" {

size_t bs_backward_workspace_bytes(const bs_patchset *ps, int32_t axis, int32_t nsweeps, int32_t ckpt_every)
{
    if (!ps || axis < 0 || axis > 2 || nsweeps < 0 || ckpt_every < 1) return 0;
    return plan_backward(ps, nsweeps, ckpt_every).total;
}

bs_status bs_relax_backward(bs_patchset *ps, int32_t axis, double omega, int32_t nsweeps, int32_t ckpt_every,
                            const double *u0, const double *f, const double *grad_uK, double *grad_u0,
                            double *grad_f, double *grad_eps, void *workspace, size_t workspace_bytes,
                            hipStream_t stream)
{
    if (axis < 0 || axis > 2) return fail(BS_ERR_INVALID, "bs_relax_backward: axis must be 0, 1 or 2");
    if (!(omega > 0.0 && omega < 2.0)) return fail(BS_ERR_INVALID, "bs_relax_backward: omega must be in (0, 2)");
    if (nsweeps < 0 || ckpt_every < 1) return fail(BS_ERR_INVALID, "bs_relax_backward: bad nsweeps or ckpt_every");
    if (!ps || !u0 || !f || !grad_uK) return fail(BS_ERR_INVALID, "bs_relax_backward: null argument");
    if (!workspace) return fail(BS_ERR_INVALID, "bs_relax_backward: null workspace");
    bs_status st = check_line_ps_ext(ps, axis, "bs_relax_backward");
    if (st != BS_OK) return st;
    const BackwardPlan bp = plan_backward(ps, nsweeps, ckpt_every);
    if (workspace_bytes < bp.total)
        return fail(BS_ERR_INVALID, "bs_relax_backward: workspace of %zu bytes, needs %zu", workspace_bytes, bp.total);
    const LineCfg c = line_cfg(ps, axis, 0);
    if ((st = check_line_cfg(ps, axis, c)) != BS_OK) return st;
    if ((st = prepare_lists(ps, axis, c, 0)) != BS_OK) return st;
    hipError_t e = prepare_line_kernels();
    if (e != hipSuccess) return hip_fail(e, "line kernel attributes");

    // carve the workspace
    char *wsp = static_cast<char *>(workspace);
    std::vector<double *> ckpt(bp.ncp), seg(bp.nseg);
    for (int i = 0; i < bp.ncp; ++i, wsp += bp.state_bytes) ckpt[i] = reinterpret_cast<double *>(wsp);
    for (int i = 0; i < bp.nseg; ++i, wsp += bp.state_bytes) seg[i] = reinterpret_cast<double *>(wsp);
    double *lam = reinterpret_cast<double *>(wsp);
    wsp += bp.state_bytes;
    double *w = reinterpret_cast<double *>(wsp);
    wsp += bp.state_bytes;
    double *gbar_ws = reinterpret_cast<double *>(wsp);
    wsp += bp.state_bytes;
    double *acc = reinterpret_cast<double *>(wsp);
    double *gbar = grad_u0 ? grad_u0 : gbar_ws;

    const PatchDesc *pdd = static_cast<const PatchDesc *>(ps->desc_d.p);
    const ResidTile *tiles = static_cast<const ResidTile *>(ps->rtile_d.p);
    const int32_t *pfirst = static_cast<const int32_t *>(ps->rtile_first_d.p);
    auto chk = [&](hipError_t err, const char *what) -> bs_status {
        return err == hipSuccess ? BS_OK : hip_fail(err, what);
    };
    auto sweep = [&](const double *src, double *dst) {
        return line_pass(ps, axis, c, 0, 0, src, dst, f, omega, stream, -1, 0, 0);
    };

    // every state buffer carries u0's ghosts; checkpoint 0 is u0
    for (double *bf : ckpt)
        if ((st = chk(launch_ghost_copy(u0, bf, pdd, ps->npatch, stream), "ghost copy")) != BS_OK) return st;
    for (double *bf : seg)
        if ((st = chk(launch_ghost_copy(u0, bf, pdd, ps->npatch, stream), "ghost copy")) != BS_OK) return st;
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
    // adjoint state
    if ((st = chk(launch_fill(lam, ps->u_numel, 0.0, stream), "fill")) != BS_OK) return st;
    if ((st = chk(launch_fill(w, ps->u_numel, 0.0, stream), "fill")) != BS_OK) return st;
    if ((st = chk(launch_fill(acc, static_cast<int64_t>(ps->nrtiles) * 3, 0.0, stream), "fill")) != BS_OK) return st;
    if (grad_f && (st = chk(launch_fill(grad_f, ps->f_numel, 0.0, stream), "fill")) != BS_OK) return st;
    if ((st = chk(launch_adj_init(grad_uK, gbar, pdd, ps->npatch, stream), "adjoint init")) != BS_OK) return st;
    // reverse, one segment at a time
    for (int s = bp.ncp - 1; s >= 0; --s) {
        const int k0 = s * ckpt_every, k1 = std::min(nsweeps, k0 + ckpt_every);
        for (int j = 1; j < k1 - k0; ++j)
            if ((st = sweep(j == 1 ? ckpt[s] : seg[j - 2], seg[j - 1])) != BS_OK) return st;
        for (int k = k1 - 1; k >= k0; --k) {
            const double *Uk = k == k0 ? ckpt[s] : seg[k - k0 - 1];
            if ((st = line_pass(ps, axis, c, 0, 0, Uk, w, f, omega, stream, -1, 0, 1)) != BS_OK) return st;
            if ((st = line_pass(ps, axis, c, 0, 0, gbar, lam, f, omega, stream, -1, 1, 1)) != BS_OK) return st;
            if ((st = chk(launch_adj_step(lam, Uk, w, gbar, grad_f, acc, pdd, tiles, ps->nrtiles, axis, omega,
                                          stream),
                          "adjoint step")) != BS_OK)
                return st;
        }
    }
    if (grad_eps && (st = chk(launch_eps_final(acc, pfirst, ps->npatch, omega, grad_eps, stream), "eps reduce")) != BS_OK)
        return st;
    return BS_OK;
}

}  // extern "C"
