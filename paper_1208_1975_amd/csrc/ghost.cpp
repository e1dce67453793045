// Boundary conditions and adjacency of a patch set: the extrapolated-Dirichlet
// faces (section 1.1: boundary conditions are extrapolated into the ghost
// layer), the links between face-adjacent patches whose ghosts are exchanged
// after every smoothing step (section 2), the face operations of one ghost
// update, and the line blocks next to extrapolated faces.
#include <algorithm>
#include <set>
#include <tuple>

#include "patchset.h"
#include "relax.h"

namespace bs {

namespace {

// Element offset in u of interior cell (idx[0], idx[1], idx[2]) of patch p
// (indices may be -1 or n: the ghost layer).
int64_t ucell(const bs_patchset *ps, int p, const int idx[3])
{
    const int64_t nx = ps->dims[3 * p], ny = ps->dims[3 * p + 1];
    const int64_t sx = nx + 2, sy = sx * (ny + 2);
    return ps->uoff[p] + (idx[2] + 1) * sy + (idx[1] + 1) * sx + (idx[0] + 1);
}

int64_t ustride(const bs_patchset *ps, int p, int axis)
{
    const int64_t nx = ps->dims[3 * p], ny = ps->dims[3 * p + 1];
    return axis == 0 ? 1 : (axis == 1 ? nx + 2 : (nx + 2) * (ny + 2));
}

// Layer `from` of patch ps along `axis` copied (times sign) into layer `to` of
// patch pd (tangential extents equal).
FaceOp face_op(const bs_patchset *ps, int pd, int to, int psrc, int from, int axis, double sign)
{
    const int t1 = axis == 0 ? 1 : 0, t2 = axis == 2 ? 1 : 2;
    FaceOp op{};
    int id[3] = {0, 0, 0}, is[3] = {0, 0, 0};
    id[axis] = to;
    is[axis] = from;
    op.d0 = ucell(ps, pd, id);
    op.s0 = ucell(ps, psrc, is);
    op.d1 = static_cast<int32_t>(ustride(ps, pd, t1));
    op.d2 = static_cast<int32_t>(ustride(ps, pd, t2));
    op.s1 = static_cast<int32_t>(ustride(ps, psrc, t1));
    op.s2 = static_cast<int32_t>(ustride(ps, psrc, t2));
    op.m1 = ps->dims[3 * pd + t1];
    op.m2 = ps->dims[3 * pd + t2];
    op.sign = sign;
    return op;
}

}  // namespace

bool ghost_active(const bs_patchset *ps) { return ps->nface_items > 0; }

bool bline_any(const bs_patchset *ps, int axis)
{
    int mask = 0;
    for (int a = 0; a < 3; ++a)
        if (a != axis) mask |= 3 << (2 * a);
    for (int p = 0; p < ps->npatch; ++p)
        if (ps->bc[p] & mask) return true;
    return false;
}

bool any_bc(const bs_patchset *ps)
{
    for (int p = 0; p < ps->npatch; ++p)
        if (ps->bc[p]) return true;
    return false;
}

// The face operations of one ghost update for the conditions bc and the links:
// the extrapolated faces (ghost = -adjacent interior), then both directions of
// every link.  Built aside; commit_face_ops swaps them in.
bs_status make_face_ops(const bs_patchset *ps, const std::vector<int32_t> &bc, const std::vector<int32_t> &links,
                        FaceOpsBuild &out)
{
    std::vector<FaceOp> ops;
    for (int p = 0; p < ps->npatch; ++p)
        for (int axis = 0; axis < 3; ++axis)
            for (int side = 0; side < 2; ++side) {
                if (!((bc[p] >> (2 * axis + side)) & 1)) continue;
                const int n = ps->dims[3 * p + axis];
                ops.push_back(face_op(ps, p, side ? n : -1, p, side ? n - 1 : 0, axis, -1.0));
            }
    const size_t nfill = ops.size();
    for (size_t t = 0; t < links.size() / 3; ++t) {
        const int a = links[3 * t], axis = links[3 * t + 1], b = links[3 * t + 2];
        const int na = ps->dims[3 * a + axis];
        ops.push_back(face_op(ps, a, na, b, 0, axis, 1.0));      // a's high ghosts <- b's first layer
        ops.push_back(face_op(ps, b, -1, a, na - 1, axis, 1.0)); // b's low ghosts <- a's last layer
    }
    std::vector<FaceItem> items;
    int nfill_items = 0;
    for (size_t o = 0; o < ops.size(); ++o) {
        const int64_t cells = static_cast<int64_t>(ops[o].m1) * ops[o].m2;
        for (int64_t c = 0; c < cells; c += kFaceItemCells)
            items.push_back(FaceItem{static_cast<int32_t>(o), static_cast<int32_t>(c),
                                     static_cast<int32_t>(std::min<int64_t>(kFaceItemCells, cells - c)), 0});
        if (o + 1 == nfill) nfill_items = static_cast<int>(items.size());
    }
    bs_status st = upload(out.ops, ops.data(), ops.size() * sizeof(FaceOp), "face operations");
    if (st != BS_OK) return st;
    if ((st = upload(out.items, items.data(), items.size() * sizeof(FaceItem), "face operations")) != BS_OK) return st;
    out.nfill = nfill_items;
    out.nitems = static_cast<int>(items.size());
    return BS_OK;
}

void commit_face_ops(bs_patchset *ps, FaceOpsBuild &b)
{
    clear_graphs(ps);
    ps->face_ops_d.swap(b.ops);
    ps->face_items_d.swap(b.items);
    ps->nfill_items = b.nfill;
    ps->nface_items = b.nitems;
}

// fill_only: the extrapolated faces alone (before the first sweep); else the
// whole update (after every sweep).
hipError_t ghost_update(const bs_patchset *ps, double *u, bool fill_only, hipStream_t s)
{
    const int n = fill_only ? ps->nfill_items : ps->nface_items;
    return launch_face_ops(u, static_cast<const FaceOp *>(ps->face_ops_d.p),
                           static_cast<const FaceItem *>(ps->face_items_d.p), n, s);
}

// The lines along `axis` next to extrapolated faces parallel to them, colour
// 0 first (colour = (p + q) mod 2, the two-colour rule of the line sweeps), and
// a scratch for their solves (shared by the axes: sized for the largest).
bs_status bline_prepare(bs_patchset *ps, int axis)
{
    if (ps->bline_ready[axis]) return BS_OK;
    const int b = axis == 0 ? 1 : 0, c = axis == 2 ? 1 : 2;
    std::vector<BLineItem> col[2];
    int maxlen = 0;
    for (int p = 0; p < ps->npatch; ++p) {
        const int bcm = ps->bc[p];
        const int nb = ps->dims[3 * p + b], nc = ps->dims[3 * p + c];
        if (!(bcm & ((3 << (2 * b)) | (3 << (2 * c))))) continue;
        for (int q = 0; q < nc; ++q)
            for (int pp = 0; pp < nb; ++pp)
                if (offline_extrap(bcm, b, pp, nb, c, q, nc)) {
                    col[(pp + q) & 1].push_back(BLineItem{p, pp, q, (pp + q) & 1});
                    maxlen = std::max(maxlen, ps->dims[3 * p + axis]);
                }
    }
    std::vector<BLineItem> all(col[0]);
    all.insert(all.end(), col[1].begin(), col[1].end());
    DevBuf d;
    bs_status st = upload(d, all.data(), all.size() * sizeof(BLineItem), "boundary lines");
    if (st != BS_OK) return st;
    const size_t need = 2 * static_cast<size_t>(maxlen) * all.size() * sizeof(double);
    if (need > ps->bline_scratch.bytes) {
        clear_graphs(ps);   // captured sequences may hold the old scratch
        if ((st = dev_alloc(ps->bline_scratch, need, "boundary line scratch")) != BS_OK) return st;
    }
    // the lines' LU factors depend on eps and the faces only: formed once here
    DevBuf fac;
    if ((st = dev_alloc(fac, std::max<size_t>(need, 8), "boundary line factors")) != BS_OK) return st;
    BLineArgs a{};
    a.pd = static_cast<const PatchDesc *>(ps->desc_d.p);
    a.items = static_cast<const BLineItem *>(d.p);
    a.fac = static_cast<double *>(fac.p);
    a.axis = axis;
    a.nlines = a.nitems = static_cast<int32_t>(all.size());
    hipError_t e = launch_bline_factors(a, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) return hip_fail(e, "boundary line factors");
    clear_graphs(ps);   // captured sequences may hold the old buffers
    ps->bline_d[axis].swap(d);
    ps->bline_fac[axis].swap(fac);
    ps->bline_count[axis][0] = static_cast<int>(col[0].size());
    ps->bline_count[axis][1] = static_cast<int>(col[1].size());
    ps->bline_maxlen[axis] = maxlen;
    ps->bline_ready[axis] = true;
    return BS_OK;
}

// colour -1: every boundary line (Jacobi); 0 / 1: that colour (in place).
bs_status bline_pass(bs_patchset *ps, int axis, int colour, const double *src, double *dst, const double *f,
                     double omega, hipStream_t s)
{
    const int n0 = ps->bline_count[axis][0], n1 = ps->bline_count[axis][1];
    BLineArgs a{};
    a.src = src;
    a.dst = dst;
    a.f = f;
    a.pd = static_cast<const PatchDesc *>(ps->desc_d.p);
    a.items = static_cast<const BLineItem *>(ps->bline_d[axis].p);
    a.scratch = static_cast<double *>(ps->bline_scratch.p);
    a.fac = static_cast<double *>(ps->bline_fac[axis].p);
    a.axis = axis;
    a.nlines = n0 + n1;
    a.first = colour == 1 ? n0 : 0;
    a.nitems = colour < 0 ? n0 + n1 : (colour == 0 ? n0 : n1);
    a.omega = omega;
    hipError_t e = launch_bline(a, ps->bline_maxlen[axis], s);
    return e == hipSuccess ? BS_OK : hip_fail(e, "boundary line kernel");
}

void reset_bc_state(bs_patchset *ps)
{
    for (int a = 0; a < 3; ++a) {
        ps->bline_ready[a] = false;
        ps->bline_count[a][0] = ps->bline_count[a][1] = 0;
    }
}

}  // namespace bs

using namespace bs;

extern "C" {

bs_status bs_set_links(bs_patchset *ps, int32_t nlinks, const int32_t *links_host)
{
    if (!ps) return fail(BS_ERR_INVALID, "bs_set_links: null patch set");
    if (nlinks < 0 || (nlinks > 0 && !links_host)) return fail(BS_ERR_INVALID, "bs_set_links: bad link list");
    std::set<std::tuple<int, int, int>> used;   // (patch, axis, side) of every linked face
    for (int t = 0; t < nlinks; ++t) {
        const int a = links_host[3 * t], axis = links_host[3 * t + 1], b = links_host[3 * t + 2];
        if (a < 0 || a >= ps->npatch || b < 0 || b >= ps->npatch || a == b || axis < 0 || axis > 2)
            return fail(BS_ERR_INVALID, "bs_set_links: link %d (%d, %d, %d) out of range", t, a, axis, b);
        for (int o = 0; o < 3; ++o)
            if (o != axis && ps->dims[3 * a + o] != ps->dims[3 * b + o])
                return fail(BS_ERR_INVALID, "bs_set_links: link %d joins faces of different extents", t);
        if (!used.insert(std::make_tuple(a, axis, 1)).second || !used.insert(std::make_tuple(b, axis, 0)).second)
            return fail(BS_ERR_INVALID, "bs_set_links: link %d uses a face that is already linked", t);
        if (((ps->bc[a] >> (2 * axis + 1)) & 1) || ((ps->bc[b] >> (2 * axis)) & 1))
            return fail(BS_ERR_INVALID, "bs_set_links: link %d joins an extrapolated face", t);
    }
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    std::vector<int32_t> nl(links_host, links_host + 3 * static_cast<size_t>(nlinks));
    FaceOpsBuild fb;
    bs_status st = make_face_ops(ps, ps->bc, nl, fb);
    if (st != BS_OK) return st;   // nothing changed
    ps->links.swap(nl);
    commit_face_ops(ps, fb);
    return BS_OK;
}

bs_status bs_exchange_ghosts(const bs_patchset *ps, double *u, hipStream_t stream)
{
    if (!ps || !u) return fail(BS_ERR_INVALID, "bs_exchange_ghosts: null patch set or u");
    hipError_t e = ghost_update(ps, u, false, stream);
    return e == hipSuccess ? BS_OK : hip_fail(e, "ghost update kernel");
}

}  // extern "C"
