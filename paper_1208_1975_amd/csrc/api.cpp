// C ABI of the block-smoothing library: argument validation, patch-set
// ownership, layout, precomputed tables and the residual.  The sweep drivers
// are in relax.cpp.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "patchset.h"
#include "relax.h"
#include "tables.h"

namespace bs {

namespace {
thread_local std::string g_err;
}

bs_status fail(bs_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

bs_status hip_fail(hipError_t e, const char *what)
{
    return fail(BS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bs_status dev_alloc(DevBuf &b, size_t bytes, const char *what)
{
    b.reset();
    if (bytes == 0) return BS_OK;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return fail(BS_ERR_OOM, "%s: hipMalloc(%zu) failed: %s", what, bytes, hipGetErrorString(e));
    }
    b.bytes = bytes;
    return BS_OK;
}

bs_status upload(DevBuf &b, const void *src, size_t bytes, const char *what)
{
    bs_status st = dev_alloc(b, bytes, what);
    if (st != BS_OK || bytes == 0) return st;
    hipError_t e = hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, what);
    return BS_OK;
}

const char *last_error_str() { return g_err.c_str(); }

}  // namespace bs

using namespace bs;

namespace {

constexpr int64_t kAlign = 32;   // doubles (256 bytes)

int64_t align_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool valid_dims(int32_t npatch, const int32_t *dims)
{
    if (npatch < 1 || !dims) return false;
    for (int64_t t = 0; t < 3 * static_cast<int64_t>(npatch); ++t)
        if (dims[t] < 1) return false;
    return true;
}

void plan_layout(int32_t npatch, const int32_t *dims, std::vector<int64_t> &uoff, std::vector<int64_t> &foff,
                 int64_t &un, int64_t &fn)
{
    uoff.resize(npatch);
    foff.resize(npatch);
    un = fn = 0;
    for (int p = 0; p < npatch; ++p) {
        const int64_t nx = dims[3 * p], ny = dims[3 * p + 1], nz = dims[3 * p + 2];
        uoff[p] = un;
        foff[p] = fn;
        un = align_up(un + (nx + 2) * (ny + 2) * (nz + 2));
        fn = align_up(fn + nx * ny * nz);
    }
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// (Re)build every table that depends on eps and upload descriptors + tables.
// The new device buffers are built aside and swapped in only once every
// allocation and copy has succeeded, so a failure leaves the patch set exactly
// as it was (old tables, work lists and captured graphs all still valid).
bs_status build_tables(bs_patchset *ps)
{
    std::vector<double> tab;
    tab.reserve(4096);
    std::vector<PatchDesc> desc(ps->npatch, PatchDesc{});
    for (int p = 0; p < ps->npatch; ++p) {
        PatchDesc &d = desc[p];
        for (int a = 0; a < 3; ++a) d.n[a] = ps->dims[3 * p + a];
        d.uoff = ps->uoff[p];
        d.foff = ps->foff[p];
        for (int a = 0; a < 3; ++a) d.eps[a] = ps->eps[3 * p + a];
        d.h2 = ps->h[p] * ps->h[p];
        d.bc = ps->bc[p];
        const double dd = 2.0 * (d.eps[0] + d.eps[1] + d.eps[2]);
        for (int a = 0; a < 3; ++a) {
            for (int o = 0; o < kNumPOpt; ++o) {
                LineTabRef &r = d.line[a][o];
                int Lr, P, Ll;
                r.off = -1;
                r.Lr = r.P = r.Llast = r.pad = 0;
                if (!line_split(d.n[a], kPOpts[o], Lr, P, Ll)) continue;
                std::vector<double> t;
                try {
                    // an extrapolated face at a line's end raises that end's diagonal by eps_a
                    const int bcm = ps->bc[p];
                    t = build_line_table(d.n[a], d.eps[a], dd, kPOpts[o], ((bcm >> (2 * a)) & 1) ? d.eps[a] : 0.0,
                                         ((bcm >> (2 * a + 1)) & 1) ? d.eps[a] : 0.0);
                } catch (const std::exception &ex) {
                    return fail(BS_ERR_INVALID, "line table for patch %d axis %d: %s", p, a, ex.what());
                }
                r.off = static_cast<int64_t>(tab.size());
                r.Lr = Lr;
                r.P = P;
                r.Llast = Ll;
                tab.insert(tab.end(), t.begin(), t.end());
                while (tab.size() % 4) tab.push_back(0.0);
            }
            d.plane[a].off = -1;
            d.plane[a].na = d.plane[a].nb = 0;
        }
    }
    DevBuf tab_d, tab32_d, desc_d;
    bs_status st = upload(tab_d, tab.data(), tab.size() * sizeof(double), "tables");
    if (st != BS_OK) return st;
    const std::vector<float> tab32(tab.begin(), tab.end());   // for FP32 block solves
    if ((st = upload(tab32_d, tab32.data(), tab32.size() * sizeof(float), "tables")) != BS_OK) return st;
    if ((st = upload(desc_d, desc.data(), desc.size() * sizeof(PatchDesc), "patch descriptors")) != BS_OK)
        return st;
    // commit: work lists and graphs refer to the old buffers, which are freed
    // when the locals go out of scope
    ps->lists.clear();
    clear_graphs(ps);
    ps->plane_ready = false;   // plane tables depend on eps; rebuilt on next use
    ps->tab_d.swap(tab_d);
    ps->tab32_d.swap(tab32_d);
    ps->desc_d.swap(desc_d);
    ps->desc.swap(desc);
    return BS_OK;
}

}  // namespace

extern "C" {

const char *bs_last_error(void) { return last_error_str(); }

bs_status bs_layout_plan(int32_t npatch, const int32_t *dims_host, int64_t *u_numel, int64_t *f_numel,
                         int64_t *u_off_host, int64_t *f_off_host)
{
    if (!u_numel || !f_numel) return fail(BS_ERR_INVALID, "bs_layout_plan: null numel pointer");
    if (!valid_dims(npatch, dims_host))
        return fail(BS_ERR_INVALID, "bs_layout_plan: npatch < 1, null dims or dims < 1");
    std::vector<int64_t> uo, fo;
    plan_layout(npatch, dims_host, uo, fo, *u_numel, *f_numel);
    if (u_off_host) std::copy(uo.begin(), uo.end(), u_off_host);
    if (f_off_host) std::copy(fo.begin(), fo.end(), f_off_host);
    return BS_OK;
}

bs_status bs_create_patchset(int32_t npatch, const int32_t *dims_host, const double *eps_host,
                             const double *h_host, bs_patchset **out)
{
    if (!out) return fail(BS_ERR_INVALID, "bs_create_patchset: out is null");
    *out = nullptr;
    if (!valid_dims(npatch, dims_host))
        return fail(BS_ERR_INVALID, "bs_create_patchset: npatch < 1, null dims or dims < 1");
    if (!eps_host || !h_host) return fail(BS_ERR_INVALID, "bs_create_patchset: null eps or h");
    for (int64_t t = 0; t < 3 * static_cast<int64_t>(npatch); ++t)
        if (!finite_pos(eps_host[t]))
            return fail(BS_ERR_INVALID, "bs_create_patchset: eps[%lld] must be finite and > 0", (long long)t);
    for (int p = 0; p < npatch; ++p)
        if (!finite_pos(h_host[p])) return fail(BS_ERR_INVALID, "bs_create_patchset: h[%d] must be finite and > 0", p);
    for (int64_t t = 0; t < 3 * static_cast<int64_t>(npatch); ++t)
        if (dims_host[t] > 4096) return fail(BS_ERR_UNSUPPORTED, "bs_create_patchset: an edge exceeds 4096");
    // the line kernels address a patch with 32-bit byte offsets
    for (int p = 0; p < npatch; ++p) {
        const int64_t padded = static_cast<int64_t>(dims_host[3 * p] + 2) * (dims_host[3 * p + 1] + 2) *
                               (dims_host[3 * p + 2] + 2);
        if (padded >= (int64_t(1) << 29))
            return fail(BS_ERR_UNSUPPORTED, "bs_create_patchset: patch %d's padded u reaches 4 GiB; split it", p);
    }

    std::unique_ptr<bs_patchset> ps(new (std::nothrow) bs_patchset);
    if (!ps) return fail(BS_ERR_OOM, "bs_create_patchset: host allocation");
    hipError_t e = hipGetDevice(&ps->device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    ps->npatch = npatch;
    ps->dims.assign(dims_host, dims_host + 3 * static_cast<size_t>(npatch));
    ps->eps.assign(eps_host, eps_host + 3 * static_cast<size_t>(npatch));
    ps->h.assign(h_host, h_host + npatch);
    ps->bc.assign(npatch, 0);
    for (int p = 0; p < npatch; ++p)
        for (int a = 0; a < 3; ++a) ps->max_n[a] = std::max(ps->max_n[a], ps->dims[3 * p + a]);
    plan_layout(npatch, dims_host, ps->uoff, ps->foff, ps->u_numel, ps->f_numel);
    bs_status st = build_tables(ps.get());
    if (st != BS_OK) return st;

    // residual (and adjoint) tiles: tx x ty columns (tx the power of two in
    // [1, 64] nearest above nx, ty = 256 / tx) by kz planes, in patch order;
    // the per-patch sums add the patch's tiles in order.  kz starts at
    // kResidPlanes and halves while the set has fewer than kResidMinTiles.
    std::vector<ResidTile> tl;
    std::vector<int32_t> tf(npatch + 1);
    auto tile_pass = [&](int kz, bool emit) -> int64_t {
        int64_t n = 0;
        for (int p = 0; p < npatch; ++p) {
            if (emit) tf[p] = static_cast<int32_t>(tl.size());
            const int nx = ps->dims[3 * p], ny = ps->dims[3 * p + 1], nz = ps->dims[3 * p + 2];
            int tx = 64;
            while (tx > 1 && (tx >> 1) >= nx) tx >>= 1;
            const int ty = 256 / tx;
            for (int z0 = 0; z0 < nz; z0 += kz)
                for (int y0 = 0; y0 < ny; y0 += ty)
                    for (int x0 = 0; x0 < nx; x0 += tx) {
                        ++n;
                        if (emit) tl.push_back(ResidTile{p, x0, y0, z0, std::min(nz, z0 + kz)});
                    }
        }
        return n;
    };
    int kz = kResidPlanes;
    while (kz > 4 && tile_pass(kz, false) < kResidMinTiles) kz >>= 1;
    if (tile_pass(kz, false) > INT32_MAX) return fail(BS_ERR_UNSUPPORTED, "bs_create_patchset: too many tiles");
    tile_pass(kz, true);
    tf[npatch] = static_cast<int32_t>(tl.size());
    ps->nrtiles = static_cast<int32_t>(tl.size());
    if ((st = upload(ps->rtile_d, tl.data(), tl.size() * sizeof(ResidTile), "residual tiles")) != BS_OK) return st;
    if ((st = upload(ps->rtile_first_d, tf.data(), tf.size() * 4, "residual tiles")) != BS_OK) return st;
    if ((st = dev_alloc(ps->rpartial_d, tl.size() * 8, "residual partials")) != BS_OK) return st;
    *out = ps.release();
    return BS_OK;
}

void bs_destroy_patchset(bs_patchset *ps)
{
    if (!ps) return;
    (void)hipDeviceSynchronize();
    delete ps;
}

bs_status bs_set_eps(bs_patchset *ps, const double *eps_host)
{
    if (!ps || !eps_host) return fail(BS_ERR_INVALID, "bs_set_eps: null argument");
    for (int64_t t = 0; t < 3 * static_cast<int64_t>(ps->npatch); ++t)
        if (!finite_pos(eps_host[t]))
            return fail(BS_ERR_INVALID, "bs_set_eps: eps[%lld] must be finite and > 0", (long long)t);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    std::vector<double> old(ps->eps);
    ps->eps.assign(eps_host, eps_host + 3 * static_cast<size_t>(ps->npatch));
    bs_status st = build_tables(ps);
    if (st != BS_OK) {
        ps->eps.swap(old);   // the old tables are untouched: the set keeps its old eps
        return st;
    }
    return cube_rebuild_all(ps);   // block inverses depend on eps
}

bs_status bs_set_bc(bs_patchset *ps, const int32_t *bc_host)
{
    if (!ps || !bc_host) return fail(BS_ERR_INVALID, "bs_set_bc: null argument");
    for (int p = 0; p < ps->npatch; ++p)
        if (bc_host[p] < 0 || bc_host[p] > 63) return fail(BS_ERR_INVALID, "bs_set_bc: bc[%d] is not a 6-bit mask", p);
    for (size_t t = 0; t < ps->links.size() / 3; ++t) {
        const int a = ps->links[3 * t], axis = ps->links[3 * t + 1], b = ps->links[3 * t + 2];
        if (((bc_host[a] >> (2 * axis + 1)) & 1) || ((bc_host[b] >> (2 * axis)) & 1))
            return fail(BS_ERR_INVALID, "bs_set_bc: link %zu joins a face that would be extrapolated", t);
    }
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    std::vector<int32_t> nb(bc_host, bc_host + ps->npatch);
    FaceOpsBuild fb;
    bs_status st = make_face_ops(ps, nb, ps->links, fb);
    if (st != BS_OK) return st;   // nothing changed
    ps->bc.swap(nb);
    if ((st = build_tables(ps)) != BS_OK) {
        ps->bc.swap(nb);   // the old tables were kept: the set keeps its old conditions
        return st;
    }
    commit_face_ops(ps, fb);
    reset_bc_state(ps);
    ps->cube.clear();   // block inverses depend on the conditions: prepare again
    return BS_OK;
}

bs_status bs_layout(const bs_patchset *ps, int64_t *u_numel, int64_t *f_numel, int64_t *u_off_host,
                    int64_t *f_off_host)
{
    if (!ps || !u_numel || !f_numel) return fail(BS_ERR_INVALID, "bs_layout: null argument");
    *u_numel = ps->u_numel;
    *f_numel = ps->f_numel;
    if (u_off_host) std::copy(ps->uoff.begin(), ps->uoff.end(), u_off_host);
    if (f_off_host) std::copy(ps->foff.begin(), ps->foff.end(), f_off_host);
    return BS_OK;
}

bs_status bs_residual(const bs_patchset *ps, const double *u, const double *f, double *r, double *rnorm2,
                      hipStream_t stream)
{
    if (!r && !rnorm2) return fail(BS_ERR_INVALID, "bs_residual: r and rnorm2 are both null");
    if (!ps || !u || !f) return fail(BS_ERR_INVALID, "bs_residual: null patch set, u or f");
    ResidArgs a{};
    a.u = u;
    a.f = f;
    a.r = r;
    a.partial = rnorm2 ? static_cast<double *>(ps->rpartial_d.p) : nullptr;
    a.pd = static_cast<const PatchDesc *>(ps->desc_d.p);
    a.tiles = static_cast<const ResidTile *>(ps->rtile_d.p);
    hipError_t e = launch_residual(a, ps->nrtiles, stream);
    if (e != hipSuccess) return hip_fail(e, "residual kernel");
    if (rnorm2) {
        e = launch_residual_final(a.partial, static_cast<const int32_t *>(ps->rtile_first_d.p), ps->npatch,
                                  rnorm2, stream);
        if (e != hipSuccess) return hip_fail(e, "residual reduction kernel");
    }
    return BS_OK;
}

// Host-side test hook (not part of the public header): the line table that
// bs_create_patchset would build for one line (end diagonals raised by dlo /
// dhi for extrapolated faces), copied to out[cap].  Returns the number of
// doubles (or -1); info = {Lr, P, Llast}.
int bsi_line_table(int n, double eps_a, double d, int preq, double dlo, double dhi, double *out, int cap, int *info)
{
    int Lr, P, Ll;
    if (!line_split(n, preq, Lr, P, Ll)) return -1;
    std::vector<double> t;
    try {
        t = build_line_table(n, eps_a, d, preq, dlo, dhi);
    } catch (...) {
        return -1;
    }
    if (info) {
        info[0] = Lr;
        info[1] = P;
        info[2] = Ll;
    }
    if (out && cap >= static_cast<int>(t.size())) std::copy(t.begin(), t.end(), out);
    return static_cast<int>(t.size());
}

}  // extern "C"
