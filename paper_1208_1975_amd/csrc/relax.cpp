// Sweep drivers: launch configuration, work lists and the sweep sequences of
// the three schemes (section 2: Jacobi with a second vector and pointer swap;
// chaotic block Gauss-Seidel in place, Algorithm 1; plus two-colour GS).
#include <algorithm>
#include <cmath>
#include <numeric>

#include "patchset.h"
#include "relax.h"

namespace bs {

namespace {

int pow2_ceil(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

int lmax_for(int Lr)
{
    if (Lr <= 8) return 8;
    if (Lr <= 16) return 16;
    if (Lr <= 32) return 32;
    return 64;
}

// Tiles of one patch for a line kernel.
int tiles_of(const bs_patchset *ps, int p, int kind, int axis, int tx, int colour_mode)
{
    const int nx = ps->dims[3 * p], ny = ps->dims[3 * p + 1], nz = ps->dims[3 * p + 2];
    if (kind == 1) {
        const int64_t rows = static_cast<int64_t>(colour_mode ? (ny + 1) / 2 : ny) * nz;
        return static_cast<int>((rows + 63) / 64);
    }
    const int no = axis == 2 ? ny : nz;
    const int span = colour_mode ? (nx + 1) / 2 : nx;
    const int nti = (span + tx - 1) / tx;
    const int nto = (no + 64 / tx - 1) / (64 / tx);
    return nti * nto;
}

// XCD-aware order: the hardware hands workgroup b to XCD b mod 8, so item j of
// a run (in spatial order) is placed at b = (j mod chunk) * 8 + j / chunk,
// giving each XCD a contiguous block of tiles that shares its L2.
void xcd_order(std::vector<WorkItem> &run)
{
    const size_t n = run.size();
    const size_t full = n / 8 * 8;
    if (full < 16) return;
    const size_t chunk = full / 8;
    std::vector<WorkItem> out(run);
    for (size_t j = 0; j < full; ++j) out[(j % chunk) * 8 + j / chunk] = run[j];
    run.swap(out);
}

}  // namespace

bs_status get_worklist(bs_patchset *ps, int kind, int axis, int popt, int tx, int colour_mode, WorkList **out)
{
    const WorkKey key{kind, axis, popt, tx, colour_mode};
    auto itr = ps->lists.find(key);
    if (itr != ps->lists.end()) {
        *out = itr->second.get();
        return BS_OK;
    }
    // LPT: larger patches first
    std::vector<int> order(ps->npatch);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const int64_t ca = static_cast<int64_t>(ps->dims[3 * a]) * ps->dims[3 * a + 1] * ps->dims[3 * a + 2];
        const int64_t cb = static_cast<int64_t>(ps->dims[3 * b]) * ps->dims[3 * b + 1] * ps->dims[3 * b + 2];
        return ca > cb;
    });
    auto wl = std::make_unique<WorkList>();
    std::vector<WorkItem> all;
    const int ncol = colour_mode ? 2 : 1;
    for (int c = 0; c < ncol; ++c) {
        std::vector<WorkItem> run;
        for (int p : order) {
            const int nt = tiles_of(ps, p, kind, axis, tx, colour_mode);
            for (int t = 0; t < nt; ++t) run.push_back(WorkItem{p, t, c, 0});
        }
        if (ps->npatch == 1) xcd_order(run);
        wl->count[c] = static_cast<int>(run.size());
        all.insert(all.end(), run.begin(), run.end());
    }
    bs_status st = upload(wl->buf, all.data(), all.size() * sizeof(WorkItem), "work list");
    if (st != BS_OK) return st;
    *out = wl.get();
    ps->lists.emplace(key, std::move(wl));
    return BS_OK;
}

LineCfg default_line_cfg(const bs_patchset *ps, int axis, int colour_mode)
{
    LineCfg c;
    const int nmax = ps->max_n[axis];
    // the fewest chunks whose length stays <= 16 (registers: about 122 VGPRs
    // at 1024 threads); longer lines take 32-cell chunks
    for (int o = 0; o < kNumPOpt; ++o) {
        const int Lr = (nmax + kPOpts[o] - 1) / kPOpts[o];
        if (Lr <= 16 || o == kNumPOpt - 1) {
            c.popt = o;
            break;
        }
    }
    int lr_max = 0;
    for (int p = 0; p < ps->npatch; ++p) lr_max = std::max(lr_max, ps->desc[p].line[axis][c.popt].Lr);
    c.Lmax = lmax_for(lr_max);
    c.nwaves = kPOpts[c.popt];
    if (axis != 0) {
        const int span = colour_mode ? (ps->max_n[0] + 1) / 2 : ps->max_n[0];
        c.tx = std::min(64, pow2_ceil(std::max(1, span)));
    } else {
        c.tx = 64;
    }
    return c;
}

bs_status check_line_cfg(const bs_patchset *ps, int axis, const LineCfg &c)
{
    if (c.popt < 0 || c.popt >= kNumPOpt) return fail(BS_ERR_INVALID, "line config: bad chunk option");
    if (c.nwaves != kPOpts[c.popt]) return fail(BS_ERR_INVALID, "line config: waves != chunk count");
    if (c.tx < 1 || c.tx > 64 || (c.tx & (c.tx - 1))) return fail(BS_ERR_INVALID, "line config: bad tile width");
    if (c.Lmax != 8 && c.Lmax != 16 && c.Lmax != 32 && c.Lmax != 64)
        return fail(BS_ERR_INVALID, "line config: bad register chunk");
    for (int p = 0; p < ps->npatch; ++p) {
        const LineTabRef &r = ps->desc[p].line[axis][c.popt];
        if (r.off < 0 || r.Lr > c.Lmax)
            return fail(BS_ERR_UNSUPPORTED, "line config: patch %d axis %d has no chunk table for %d chunks", p, axis,
                        kPOpts[c.popt]);
    }
    return BS_OK;
}

size_t line_lds_bytes(const bs_patchset *ps, int axis, const LineCfg &c)
{
    int tsz = 0, sd = 1;
    for (int p = 0; p < ps->npatch; ++p) {
        const LineTabRef &r = ps->desc[p].line[axis][c.popt];
        tsz = std::max(tsz, line_table_size(r.Lr, r.P));
        sd = std::max(sd, ps->dims[3 * p] | 1);
    }
    size_t n = static_cast<size_t>((tsz + 1) & ~1) + 2 * 64 * static_cast<size_t>(c.nwaves);
    if (axis == 0) n += 64 * static_cast<size_t>(sd) + 128;
    return n * sizeof(double);
}

// One pass over the lines of `axis`: colour_mode 0 = all lines (one run);
// colour_mode 1 with run = 0 / 1 = that colour only, run = 2 = both colours in
// one launch, colour 0 dispatched first (chaotic).
bs_status line_pass(bs_patchset *ps, int axis, const LineCfg &c, int colour_mode, int run, const double *src,
                    double *dst, const double *f, double omega, hipStream_t stream)
{
    const int kind = axis == 0 ? 1 : 0;
    WorkList *wl = nullptr;
    bs_status st = get_worklist(ps, kind, axis, c.popt, c.tx, colour_mode, &wl);
    if (st != BS_OK) return st;
    int first = 0, count = wl->count[0];
    if (colour_mode) {
        if (run == 1) {
            first = wl->count[0];
            count = wl->count[1];
        } else if (run == 2) {
            count = wl->count[0] + wl->count[1];
        }
    }
    if (count == 0) return BS_OK;
    LineArgs a{};
    a.src = src;
    a.dst = dst;
    a.f = f;
    a.pd = static_cast<const PatchDesc *>(ps->desc_d.p);
    a.tab = static_cast<const double *>(ps->tab_d.p);
    a.items = static_cast<const WorkItem *>(wl->buf.p) + first;
    a.axis = axis;
    a.popt = c.popt;
    a.tx = c.tx;
    a.colour_mode = colour_mode;
    a.omega = omega;
    const size_t lds = line_lds_bytes(ps, axis, c);
    if (lds > 160 * 1024) return fail(BS_ERR_UNSUPPORTED, "line sweep needs %zu bytes of LDS", lds);
    hipError_t e = axis == 0 ? launch_line_x(a, count, c.Lmax, c.nwaves, lds, stream)
                             : launch_line_strided(a, count, c.Lmax, c.nwaves, lds, stream);
    if (e != hipSuccess) return hip_fail(e, "line sweep kernel");
    return BS_OK;
}

const LineCfg &line_cfg(bs_patchset *ps, int axis, int colour_mode)
{
    auto key = std::make_pair(axis, colour_mode);
    auto itr = ps->line_cfg.find(key);
    if (itr == ps->line_cfg.end()) itr = ps->line_cfg.emplace(key, default_line_cfg(ps, axis, colour_mode)).first;
    return itr->second;
}

}  // namespace bs

using namespace bs;

extern "C" {

bs_status bs_line_relax(bs_patchset *ps, int32_t axis, bs_scheme scheme, double omega, int32_t nsweeps,
                        bs_precision prec, double *u, const double *f, double *work, hipStream_t stream)
{
    if (axis < 0 || axis > 2) return fail(BS_ERR_INVALID, "bs_line_relax: axis must be 0, 1 or 2");
    if (scheme != BS_JACOBI && scheme != BS_CHAOTIC_GS && scheme != BS_COLORED_GS)
        return fail(BS_ERR_INVALID, "bs_line_relax: unknown scheme");
    if (!(omega > 0.0 && omega < 2.0)) return fail(BS_ERR_INVALID, "bs_line_relax: omega must be in (0, 2)");
    if (nsweeps < 0) return fail(BS_ERR_INVALID, "bs_line_relax: nsweeps < 0");
    if (prec != BS_FP64 && prec != BS_MIXED_FP32 && prec != BS_MIXED_BF16)
        return fail(BS_ERR_INVALID, "bs_line_relax: unknown precision");
    if (prec == BS_MIXED_BF16) return fail(BS_ERR_UNSUPPORTED, "bs_line_relax: BF16 is offered for planes only");
    if (prec == BS_MIXED_FP32) return fail(BS_ERR_UNSUPPORTED, "bs_line_relax: FP32 line solves are not provided");
    if (!ps || !u || !f) return fail(BS_ERR_INVALID, "bs_line_relax: null patch set, u or f");
    if (scheme == BS_JACOBI && !work) return fail(BS_ERR_INVALID, "bs_line_relax: Jacobi needs a work buffer");
    if (ps->max_n[axis] > 16 * kMaxChunkLen)
        return fail(BS_ERR_UNSUPPORTED, "bs_line_relax: lines longer than %d cells", 16 * kMaxChunkLen);
    if (axis == 0 && ps->max_n[0] > 256)
        return fail(BS_ERR_UNSUPPORTED, "bs_line_relax: x-lines longer than 256 cells");
    if (nsweeps == 0) return BS_OK;

    const int cm = scheme == BS_JACOBI ? 0 : 1;
    const LineCfg &c = line_cfg(ps, axis, cm);
    bs_status st = check_line_cfg(ps, axis, c);
    if (st != BS_OK) return st;
    const PatchDesc *pdd = static_cast<const PatchDesc *>(ps->desc_d.p);

    if (scheme == BS_JACOBI) {
        hipError_t e = launch_ghost_copy(u, work, pdd, ps->npatch, stream);
        if (e != hipSuccess) return hip_fail(e, "ghost copy");
        for (int s = 0; s < nsweeps; ++s) {
            const double *src = (s & 1) ? work : u;
            double *dst = (s & 1) ? u : work;
            if ((st = line_pass(ps, axis, c, 0, 0, src, dst, f, omega, stream)) != BS_OK) return st;
        }
        if (nsweeps & 1) {
            e = launch_interior_copy(work, u, pdd, ps->npatch, stream);
            if (e != hipSuccess) return hip_fail(e, "interior copy");
        }
        return BS_OK;
    }
    for (int s = 0; s < nsweeps; ++s) {
        if (scheme == BS_COLORED_GS) {
            if ((st = line_pass(ps, axis, c, 1, 0, u, u, f, omega, stream)) != BS_OK) return st;
            if ((st = line_pass(ps, axis, c, 1, 1, u, u, f, omega, stream)) != BS_OK) return st;
        } else {
            if ((st = line_pass(ps, axis, c, 1, 2, u, u, f, omega, stream)) != BS_OK) return st;
        }
    }
    return BS_OK;
}

size_t bs_backward_workspace_bytes(const bs_patchset *ps, int32_t axis, int32_t nsweeps, int32_t ckpt_every)
{
    (void)ps;
    (void)axis;
    (void)nsweeps;
    (void)ckpt_every;
    return 0;
}

bs_status bs_relax_backward(bs_patchset *ps, int32_t axis, double omega, int32_t nsweeps, int32_t ckpt_every,
                            const double *u0, const double *f, const double *grad_uK, double *grad_u0,
                            double *grad_f, double *grad_eps, void *workspace, size_t workspace_bytes,
                            hipStream_t stream)
{
    (void)grad_u0;
    (void)grad_f;
    (void)grad_eps;
    (void)workspace;
    (void)workspace_bytes;
    (void)stream;
    if (axis < 0 || axis > 2) return fail(BS_ERR_INVALID, "bs_relax_backward: axis must be 0, 1 or 2");
    if (!(omega > 0.0 && omega < 2.0)) return fail(BS_ERR_INVALID, "bs_relax_backward: omega must be in (0, 2)");
    if (nsweeps < 0 || ckpt_every < 1) return fail(BS_ERR_INVALID, "bs_relax_backward: bad nsweeps or ckpt_every");
    if (!ps || !u0 || !f || !grad_uK) return fail(BS_ERR_INVALID, "bs_relax_backward: null argument");
    return fail(BS_ERR_UNSUPPORTED, "bs_relax_backward: not built yet");
}

// Host-side tuning hook (not part of the public header): set the launch
// configuration of line sweeps along `axis` for the Jacobi (colour_mode 0) or
// Gauss-Seidel (colour_mode 1) kernels.  popt indexes the chunk counts
// {1,2,4,8,16}; tx is the strided kernel's lanes per row (power of two <= 64).
int bsi_set_line_cfg(bs_patchset *ps, int axis, int colour_mode, int popt, int tx)
{
    if (!ps || axis < 0 || axis > 2 || colour_mode < 0 || colour_mode > 1) return BS_ERR_INVALID;
    if (popt < 0 || popt >= kNumPOpt) return BS_ERR_INVALID;
    LineCfg c;
    c.popt = popt;
    c.nwaves = kPOpts[popt];
    c.tx = tx;
    int lr_max = 0;
    for (int p = 0; p < ps->npatch; ++p) {
        if (ps->desc[p].line[axis][popt].off < 0) return BS_ERR_UNSUPPORTED;
        lr_max = std::max(lr_max, ps->desc[p].line[axis][popt].Lr);
    }
    c.Lmax = lr_max <= 8 ? 8 : lr_max <= 16 ? 16 : lr_max <= 32 ? 32 : 64;
    bs_status st = check_line_cfg(ps, axis, c);
    if (st != BS_OK) return st;
    ps->line_cfg[std::make_pair(axis, colour_mode)] = c;
    return BS_OK;
}

}  // extern "C"
