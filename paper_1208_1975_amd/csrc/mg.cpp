// Geometric multigrid V-cycle with the line and plane block smoothers
// (section 1: line and plane smoothers are the components that make geometric
// multigrid robust for anisotropic problems; section 5: multilevel use).
//
// Every patch of the fine set is coarsened on its own by factors of two (cell
// width 2h, the same eps): the defect d = h^2 f - A u is restricted to the
// right-hand side f_c = R(d / h^2) of the coarse error equation
// A e = (2h)^2 f_c, whose ghosts carry the error's homogeneous condition
// (zero ghosts, or the extrapolated faces of coarse_bc), and the coarse
// correction is interpolated back trilinearly.
#include <cstring>
#include <memory>
#include <vector>

#include "patchset.h"
#include "relax.h"

struct bs_mg {
    bs_patchset *fine = nullptr;                   // the caller's, level 0
    std::vector<bs_patchset *> lv;                 // owned: levels 1 .. L-1
    std::vector<bs::DevBuf *> u, f, w, d;          // per level (u, f, w from 1; d up to L-2)
    int kind = 0, arg = 0, nu1 = 1, nu2 = 1, ncoarse = 1, coarse_bc = 0, levels = 1;
    bs_scheme scheme = BS_COLORED_GS;
    double omega = 1.0;
    std::vector<std::pair<std::vector<int64_t>, hipGraphExec_t>> graphs;
    std::vector<std::vector<int64_t>> seen;        // sequences run eagerly once
    uint64_t gen = 0;                              // the fine set's generation the graphs were captured at
    std::vector<double> eps0;                      // the fine set's eps and faces at creation
    std::vector<int32_t> bc0;
    hipStream_t cap = nullptr;
    ~bs_mg()
    {
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
        if (cap) (void)hipStreamDestroy(cap);
        for (bs_patchset *p : lv) bs_destroy_patchset(p);
        for (auto *v : {&u, &f, &w, &d})
            for (bs::DevBuf *b : *v) delete b;
    }
};

namespace bs {

namespace {

bs_patchset *level_ps(bs_mg *mg, int l) { return l == 0 ? mg->fine : mg->lv[l - 1]; }

int64_t max_cells(const bs_patchset *ps)
{
    int64_t m = 0;
    for (int p = 0; p < ps->npatch; ++p)
        m = std::max<int64_t>(m, int64_t(ps->dims[3 * p]) * ps->dims[3 * p + 1] * ps->dims[3 * p + 2]);
    return m;
}

bs_status smooth(bs_mg *mg, int l, int nsweeps, double *u, const double *f, double *w, hipStream_t s)
{
    bs_patchset *ps = level_ps(mg, l);
    if (mg->kind == 0)
        return line_relax_impl(ps, mg->arg, mg->scheme, mg->omega, nsweeps, BS_FP64, u, f, w, s, false);
    return bs_plane_relax(ps, mg->arg, mg->scheme, mg->omega, nsweeps, BS_FP64, 0, u, f, w, s);
}

bs_status cycle(bs_mg *mg, int l, double *u, const double *f, double *w, hipStream_t s)
{
    bs_status st;
    if (l == mg->levels - 1) return smooth(mg, l, mg->ncoarse, u, f, w, s);
    if ((st = smooth(mg, l, mg->nu1, u, f, w, s)) != BS_OK) return st;
    bs_patchset *ps = level_ps(mg, l), *pc = mg->lv[l];
    double *d = static_cast<double *>(mg->d[l]->p);
    if ((st = bs_residual(ps, u, f, d, nullptr, s)) != BS_OK) return st;
    const PatchDesc *dF = static_cast<const PatchDesc *>(ps->desc_d.p);
    const PatchDesc *dC = static_cast<const PatchDesc *>(pc->desc_d.p);
    double *uc = static_cast<double *>(mg->u[l + 1]->p);
    double *fc = static_cast<double *>(mg->f[l + 1]->p);
    double *wc = static_cast<double *>(mg->w[l + 1]->p);
    hipError_t e = launch_restrict(d, fc, dF, dC, ps->npatch, max_cells(pc), s);
    if (e != hipSuccess) return hip_fail(e, "restriction");
    if ((e = launch_fill(uc, pc->u_numel, 0.0, s)) != hipSuccess) return hip_fail(e, "coarse zero");
    if ((st = cycle(mg, l + 1, uc, fc, wc, s)) != BS_OK) return st;
    if ((e = launch_prolong_add(uc, u, dF, dC, ps->npatch, max_cells(ps), mg->coarse_bc, s)) != hipSuccess)
        return hip_fail(e, "prolongation");
    return smooth(mg, l, mg->nu2, u, f, w, s);
}

}  // namespace

}  // namespace bs

using namespace bs;

extern "C" {

bs_status bs_mg_create(bs_patchset *fine, int32_t kind, int32_t arg, bs_scheme scheme, double omega, int32_t nu1,
                       int32_t nu2, int32_t ncoarse, int32_t levels, int32_t coarse_bc, bs_mg **out)
{
    if (!out) return fail(BS_ERR_INVALID, "bs_mg_create: out is null");
    *out = nullptr;
    if (!fine) return fail(BS_ERR_INVALID, "bs_mg_create: null patch set");
    if (kind != 0 && kind != 1) return fail(BS_ERR_INVALID, "bs_mg_create: kind must be 0 (lines) or 1 (planes)");
    if (arg < 0 || arg > 2) return fail(BS_ERR_INVALID, "bs_mg_create: axis must be 0, 1 or 2");
    if (scheme != BS_JACOBI && scheme != BS_CHAOTIC_GS && scheme != BS_COLORED_GS)
        return fail(BS_ERR_INVALID, "bs_mg_create: unknown scheme");
    if (!(omega > 0.0 && omega < 2.0)) return fail(BS_ERR_INVALID, "bs_mg_create: omega must be in (0, 2)");
    if (nu1 < 0 || nu2 < 0 || ncoarse < 0 || levels < 0)
        return fail(BS_ERR_INVALID, "bs_mg_create: negative sweep or level count");
    if (coarse_bc < 0 || coarse_bc > 63) return fail(BS_ERR_INVALID, "bs_mg_create: coarse_bc is not a 6-bit mask");
    if (!fine->links.empty()) return fail(BS_ERR_UNSUPPORTED, "bs_mg_create: patch sets with links");
    // levels: halve while every edge of every patch is even and >= 2
    int maxl = 1;
    std::vector<int32_t> dims(fine->dims);
    while (true) {
        bool ok = true;
        for (int32_t v : dims) ok = ok && v >= 2 && v % 2 == 0;
        if (!ok) break;
        for (int32_t &v : dims) v /= 2;
        ++maxl;
    }
    const int L = levels == 0 ? maxl : std::min<int>(levels, maxl);
    std::unique_ptr<bs_mg> mg(new (std::nothrow) bs_mg);
    if (!mg) return fail(BS_ERR_OOM, "bs_mg_create: host allocation");
    mg->fine = fine;
    mg->kind = kind;
    mg->arg = arg;
    mg->scheme = scheme;
    mg->omega = omega;
    mg->nu1 = nu1;
    mg->nu2 = nu2;
    mg->ncoarse = ncoarse;
    mg->coarse_bc = coarse_bc;
    mg->levels = L;
    mg->eps0 = fine->eps;
    mg->bc0 = fine->bc;
    mg->gen = fine->gen;
    mg->u.assign(L, nullptr);
    mg->f.assign(L, nullptr);
    mg->w.assign(L, nullptr);
    mg->d.assign(L, nullptr);
    dims = fine->dims;
    std::vector<double> h(fine->h);
    const int np = fine->npatch;
    const std::vector<int32_t> cbc(np, coarse_bc);
    bs_status st;
    for (int l = 1; l < L; ++l) {
        for (int32_t &v : dims) v /= 2;
        for (double &v : h) v *= 2.0;
        bs_patchset *pc = nullptr;
        if ((st = bs_create_patchset(np, dims.data(), fine->eps.data(), h.data(), &pc)) != BS_OK) return st;
        mg->lv.push_back(pc);
        if (coarse_bc && (st = bs_set_bc(pc, cbc.data())) != BS_OK) return st;
        for (auto *v : {&mg->u, &mg->f, &mg->w}) (*v)[l] = new DevBuf;
        if ((st = dev_alloc(*mg->u[l], pc->u_numel * sizeof(double), "multigrid level")) != BS_OK) return st;
        if ((st = dev_alloc(*mg->f[l], pc->f_numel * sizeof(double), "multigrid level")) != BS_OK) return st;
        if ((st = dev_alloc(*mg->w[l], pc->u_numel * sizeof(double), "multigrid level")) != BS_OK) return st;
        hipError_t e = launch_fill(static_cast<double *>(mg->w[l]->p), pc->u_numel, 0.0, nullptr);
        if (e != hipSuccess) return hip_fail(e, "multigrid level");
    }
    for (int l = 0; l + 1 < L; ++l) {
        mg->d[l] = new DevBuf;
        const bs_patchset *ps = l == 0 ? fine : mg->lv[l - 1];
        if ((st = dev_alloc(*mg->d[l], ps->f_numel * sizeof(double), "multigrid defect")) != BS_OK) return st;
    }
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    *out = mg.release();
    return BS_OK;
}

void bs_mg_destroy(bs_mg *mg)
{
    if (!mg) return;
    (void)hipDeviceSynchronize();
    delete mg;
}

bs_status bs_mg_levels(const bs_mg *mg, int32_t *levels)
{
    if (!mg || !levels) return fail(BS_ERR_INVALID, "bs_mg_levels: null argument");
    *levels = mg->levels;
    return BS_OK;
}

bs_status bs_vcycle(bs_mg *mg, double *u, const double *f, double *work, hipStream_t stream)
{
    if (!mg || !u || !f) return fail(BS_ERR_INVALID, "bs_vcycle: null multigrid, u or f");
    if (mg->scheme == BS_JACOBI && !work) return fail(BS_ERR_INVALID, "bs_vcycle: Jacobi smoothing needs a work buffer");
    if (mg->fine->eps != mg->eps0 || mg->fine->bc != mg->bc0)
        return fail(BS_ERR_INVALID, "bs_vcycle: the fine patch set's eps or faces changed; create the cycle again");
    if (mg->fine->gen != mg->gen) {
        // the fine set replaced tables the captured cycles refer to
        for (auto &g : mg->graphs) (void)hipGraphExecDestroy(g.second);
        mg->graphs.clear();
        mg->seen.clear();
        mg->gen = mg->fine->gen;
    }
    const std::vector<int64_t> key{reinterpret_cast<int64_t>(u), reinterpret_cast<int64_t>(f),
                                   reinterpret_cast<int64_t>(work)};
    for (auto &g : mg->graphs)
        if (g.first == key) {
            hipError_t e = hipGraphLaunch(g.second, stream);
            return e == hipSuccess ? BS_OK : hip_fail(e, "hipGraphLaunch");
        }
    bool seen = false;
    for (auto &k : mg->seen) seen = seen || k == key;
    if (!seen || !mg->fine->use_graphs) {
        // the first cycle with these buffers runs eagerly: it builds every
        // table and work list the levels need, so that the next one can be
        // captured
        if (!seen) mg->seen.push_back(key);
        bs_status st = cycle(mg, 0, u, f, work, stream);
        mg->gen = mg->fine->gen;   // tables built on the way are part of the state to capture
        return st;
    }
    hipError_t e;
    if (!mg->cap && (e = hipStreamCreateWithFlags(&mg->cap, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "capture stream");
    hipGraph_t graph = nullptr;
    if ((e = hipStreamBeginCapture(mg->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, "hipStreamBeginCapture");
    bs_status st = cycle(mg, 0, u, f, work, mg->cap);
    e = hipStreamEndCapture(mg->cap, &graph);
    if (st != BS_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    if (mg->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(mg->graphs.front().second);
        mg->graphs.erase(mg->graphs.begin());
    }
    mg->graphs.emplace_back(key, exec);
    if ((e = hipGraphLaunch(exec, stream)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return BS_OK;
}

}  // extern "C"
