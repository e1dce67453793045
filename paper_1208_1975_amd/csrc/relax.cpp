// Line sweep drivers: launch configurations, work lists, the sweep sequences
// of the three schemes (section 2: Jacobi through a second vector with a
// pointer swap; chaotic block Gauss-Seidel in place, Algorithm 1; plus
// two-colour GS), graph capture of whole sequences, the autotuner and the
// backward entry points' argument checks.
#include <algorithm>
#include <cmath>
#include <cstring>
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

// Tiles of one patch for a line kernel (kind 0 strided y/z lines, 1 x-line
// row blocks, 2 z-marching x-line items: tx = planes per item, nw = waves).
int tiles_of(const bs_patchset *ps, int p, int kind, int axis, int tx, int colour_mode, int nw = 0)
{
    const int nx = ps->dims[3 * p], ny = ps->dims[3 * p + 1], nz = ps->dims[3 * p + 2];
    if (kind == 2) {
        const int R = xz_item_rows(nx, nw);
        return ((ny + R - 1) / R) * ((nz + tx - 1) / tx);
    }
    if (kind == 3) return ((nx + 127) / 128) * (axis == 2 ? ny : nz);   // 128 x-cells by one row
    if (kind == 1) {
        const int64_t rows = static_cast<int64_t>(colour_mode == 1 ? (ny + 1) / 2 : ny) * nz;
        return static_cast<int>((rows + 63) / 64);
    }
    const int no = axis == 2 ? ny : nz;
    const int span = colour_mode == 1 ? (nx + 1) / 2 : nx;
    const int nti = (span + tx - 1) / tx;
    const int nto = (no + 64 / tx - 1) / (64 / tx);
    return nti * nto;
}

// Tile rows (along the other free axis) of one patch's strided tiles.
int tiles_per_row(const bs_patchset *ps, int p, int tx)
{
    return (ps->dims[3 * p] + tx - 1) / tx;
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

// Dispatch order for a patch set: whole patches go to one XCD each (greedy,
// larger patches first, balancing line cells), each patch's items stay
// consecutive in its XCD's sequence (neighbouring tiles then share that XCD's
// L2), and the sequences are interleaved so that workgroup j*8 + x runs the
// j-th item of XCD x; shorter sequences are padded with empty items.
std::vector<WorkItem> xcd_group(const std::vector<WorkItem> &run, const std::vector<int> &order,
                                const std::vector<int> &first, const std::vector<int> &count,
                                const std::vector<int64_t> &weight)
{
    std::vector<std::vector<WorkItem>> lists(8);
    int64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int p : order) {
        if (count[p] == 0) continue;
        int x = 0;
        for (int k = 1; k < 8; ++k)
            if (load[k] < load[x]) x = k;
        for (int t = 0; t < count[p]; ++t) lists[x].push_back(run[first[p] + t]);
        load[x] += weight[p];
    }
    size_t len = 0;
    for (const auto &l : lists) len = std::max(len, l.size());
    std::vector<WorkItem> out(8 * len, WorkItem{-1, 0, 0, 0});
    for (int x = 0; x < 8; ++x)
        for (size_t j = 0; j < lists[x].size(); ++j) out[j * 8 + x] = lists[x][j];
    return out;
}

// Dispatch order of the in-tile two-colour (chaotic) runs: each XCD takes
// contiguous tiles (one patch: an eighth of its tiles; a patch set: whole
// patches, balanced), its sequence is cut into chunks of about kChaoticChunk
// tiles, and each chunk runs its even tile rows before its odd ones.  The odd
// tiles then find their neighbours' new values, still in that XCD's L2; only
// chunk borders see older values (the asynchronous part of the scheme).  The
// eight sequences are interleaved as in xcd_group.
std::vector<WorkItem> chaotic_order(const bs_patchset *ps, const std::vector<WorkItem> run[2],
                                    const std::vector<int> &order, const std::vector<int> pfirst[2],
                                    const std::vector<int> pcount[2], int axis, int kChaoticChunk)
{
    // per XCD: the sequence of units, a unit = (run-0 items, run-1 items) of one patch or one slice
    struct Unit {
        std::vector<WorkItem> it[2];
    };
    std::vector<std::vector<Unit>> xl(8);
    if (ps->npatch == 1) {
        // spatial order: tiles in increasing index, split into 8 contiguous blocks
        std::vector<WorkItem> sp(run[0].begin(), run[0].end());
        sp.insert(sp.end(), run[1].begin(), run[1].end());
        std::sort(sp.begin(), sp.end(), [](const WorkItem &a, const WorkItem &b) { return a.tile < b.tile; });
        const size_t n = sp.size();
        for (int x = 0; x < 8; ++x) {
            Unit u;
            for (size_t j = n * x / 8; j < n * (x + 1) / 8; ++j) u.it[sp[j].colour].push_back(sp[j]);
            xl[x].push_back(u);
        }
    } else {
        int64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int p : order) {
            if (pcount[0][p] + pcount[1][p] == 0) continue;
            int x = 0;
            for (int k = 1; k < 8; ++k)
                if (load[k] < load[x]) x = k;
            Unit u;
            for (int c = 0; c < 2; ++c)
                for (int t = 0; t < pcount[c][p]; ++t) u.it[c].push_back(run[c][pfirst[c][p] + t]);
            load[x] += static_cast<int64_t>(pcount[0][p] + pcount[1][p]) * ps->dims[3 * p + axis];
            xl[x].push_back(u);
        }
    }
    std::vector<std::vector<WorkItem>> lists(8);
    for (int x = 0; x < 8; ++x) {
        // chunks of consecutive tiles: even tiles of the chunk, then its odd tiles
        std::vector<WorkItem> ev, od;
        auto flush = [&]() {
            lists[x].insert(lists[x].end(), ev.begin(), ev.end());
            lists[x].insert(lists[x].end(), od.begin(), od.end());
            ev.clear();
            od.clear();
        };
        for (const Unit &u : xl[x]) {
            // a single large unit is cut into chunks in its own spatial order
            std::vector<WorkItem> merged(u.it[0].begin(), u.it[0].end());
            merged.insert(merged.end(), u.it[1].begin(), u.it[1].end());
            std::sort(merged.begin(), merged.end(), [](const WorkItem &a, const WorkItem &b) { return a.tile < b.tile; });
            for (const WorkItem &w : merged) {
                (w.colour == 0 ? ev : od).push_back(w);
                if (static_cast<int>(ev.size() + od.size()) >= kChaoticChunk) flush();
            }
        }
        flush();
    }
    size_t len = 0;
    for (const auto &l : lists) len = std::max(len, l.size());
    std::vector<WorkItem> out(8 * len, WorkItem{-1, 0, 0, 0});
    for (int x = 0; x < 8; ++x)
        for (size_t j = 0; j < lists[x].size(); ++j) out[j * 8 + x] = lists[x][j];
    return out;
}

int device_cus()
{
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

}  // namespace

void clear_graphs(bs_patchset *ps)
{
    ++ps->gen;   // sequences captured elsewhere (multigrid cycles) hold the same pointers
    for (auto &kv : ps->graphs) (void)hipGraphExecDestroy(kv.second);
    ps->graphs.clear();
}

bs_status get_worklist(bs_patchset *ps, int kind, int axis, int popt, int tx, int colour_mode, WorkList **out,
                       int chunk)
{
    if (colour_mode != 2 || kind == 2) chunk = 0;
    if (colour_mode == 2 && chunk <= 0) chunk = ps->npatch == 1 ? 64 : 512;
    const WorkKey key{kind, axis, popt, tx, colour_mode, chunk};
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
    std::vector<WorkItem> all, plain;
    std::vector<WorkItem> runs[2];
    // z-marching x-line items: one run in every colour mode (chaotic GS orders
    // its lines inside each item)
    const int ncol = (colour_mode && kind != 2) ? 2 : 1;
    for (int c = 0; c < ncol; ++c) {
        std::vector<WorkItem> &run = runs[c];
        wl->pfirst[c].assign(ps->npatch, 0);
        wl->pcount[c].assign(ps->npatch, 0);
        for (int p : order) {
            const int nt = tiles_of(ps, p, kind, axis, tx, colour_mode, popt);
            wl->pfirst[c][p] = static_cast<int>(run.size());
            if (colour_mode == 2 && kind != 2) {
                // in-tile two-colour: all tiles, tile rows of parity c in run c
                // (x lines: a tile is a block of rows, alternate tiles)
                const int nti = kind == 1 ? 1 : tiles_per_row(ps, p, tx);
                for (int t = 0; t < nt; ++t)
                    if ((t / nti) % 2 == c) run.push_back(WorkItem{p, t, c, 0});
            } else {
                for (int t = 0; t < nt; ++t) run.push_back(WorkItem{p, t, c, 0});
            }
            wl->pcount[c][p] = static_cast<int>(run.size()) - wl->pfirst[c][p];
        }
        wl->pp_off[c] = static_cast<int>(plain.size());
        plain.insert(plain.end(), run.begin(), run.end());
    }
    if (colour_mode == 2 && kind != 2) {
        // one launch runs both groups: local even-then-odd chunks per XCD
        const std::vector<WorkItem> d = chaotic_order(ps, runs, order, wl->pfirst, wl->pcount, axis, chunk);
        wl->count[0] = static_cast<int>(d.size());
        wl->count[1] = 0;
        all.insert(all.end(), d.begin(), d.end());
    } else {
        for (int c = 0; c < ncol; ++c) {
            std::vector<WorkItem> run = runs[c];
            if (ps->npatch == 1) {
                xcd_order(run);
            } else {
                std::vector<int64_t> weight(ps->npatch);
                for (int p = 0; p < ps->npatch; ++p)
                    weight[p] = static_cast<int64_t>(wl->pcount[c][p]) * ps->dims[3 * p + axis];
                run = xcd_group(run, order, wl->pfirst[c], wl->pcount[c], weight);
            }
            wl->count[c] = static_cast<int>(run.size());
            all.insert(all.end(), run.begin(), run.end());
        }
    }
    for (int c = 0; c < ncol; ++c) wl->pp_off[c] += static_cast<int>(all.size());
    all.insert(all.end(), plain.begin(), plain.end());
    bs_status st = upload(wl->buf, all.data(), all.size() * sizeof(WorkItem), "work list");
    if (st != BS_OK) return st;
    *out = wl.get();
    ps->lists.emplace(key, std::move(wl));
    return BS_OK;
}

// Planes per z-marching x-line item: whole patches along z unless the set
// would have fewer than eight items per compute unit, then halved (down to 4).
int xz_planes(const bs_patchset *ps, int nwaves, int min_planes = 4)
{
    int zc = ps->max_n[2];
    auto items = [&](int z) {
        int64_t n = 0;
        for (int p = 0; p < ps->npatch; ++p) n += tiles_of(ps, p, 2, 0, z, 0, nwaves);
        return n;
    };
    while (zc > min_planes && items(zc) < 8 * static_cast<int64_t>(device_cus())) zc = (zc + 1) / 2;
    return std::max(zc, 1);
}

LineCfg default_line_cfg(const bs_patchset *ps, int axis, int colour_mode, bool direct)
{
    LineCfg c;
    c.deflt = 1;
    const int nmax = ps->max_n[axis];
    // the fewest chunks whose length stays <= 16 (about 126 VGPRs at 1024
    // threads); longer lines take 32-cell chunks.  On lines of 129..256
    // cells FP64 Jacobi in the direct form takes four chunks of up to 64 cells
    // (two 4-wave workgroups per CU; 256^3 z-lines: 97 us per sweep against
    // 102 us with eight chunks of 32 and 104 us with sixteen of 16), and the
    // two-cells-per-lane chaotic kernel eight of up to 32 (107-109 against
    // 111-112 us)
    const bool yz = axis != 0 && direct && nmax > 128 && nmax <= 256;
    const int lr_cap = (yz && colour_mode == 0 && ps->line_direct) ? 64
                       : (yz && colour_mode == 2 && ps->use_pair) ? 32 : 16;
    for (int o = 0; o < kNumPOpt; ++o) {
        const int Lr = (nmax + kPOpts[o] - 1) / kPOpts[o];
        if (Lr <= lr_cap || o == kNumPOpt - 1) {
            c.popt = o;
            break;
        }
    }
    int lr_max = 0;
    for (int p = 0; p < ps->npatch; ++p) lr_max = std::max(lr_max, ps->desc[p].line[axis][c.popt].Lr);
    c.Lmax = lmax_for(lr_max);
    c.nwaves = kPOpts[c.popt];
    if (axis != 0) {
        const int span = colour_mode == 1 ? (ps->max_n[0] + 1) / 2 : ps->max_n[0];
        c.tx = std::min(64, pow2_ceil(std::max(1, span)));
    } else {
        c.tx = 64;
    }
    c.grid = 0;
    if (axis == 0 && nmax <= kXregMaxN) {
        // x-lines of up to 64 cells: across the lanes of a 16-lane row, four
        // cells per lane, one line table (the line's own LU factors).  Plain
        // Jacobi sweeps march one-wavefront items along z, down to one plane
        // per item (single patches of 16^3..64^3: 1.2-2.1x faster than the
        // 4-wave register form; the result does not depend on the items);
        // chaotic GS keeps the register form's in-tile two-colour order unless
        // configured or tuned otherwise, and the solve-only and field
        // right-hand-side modes run on the register form
        c.popt = 0;
        c.Lmax = 4;
        if (direct && colour_mode == 0) {
            c.form = 2;
            c.nwaves = 1;
            c.zc = xz_planes(ps, 1, 1);
        } else {
            c.form = 1;
            c.nwaves = 4;
        }
    }
    return c;
}

size_t line_lds_bytes(const bs_patchset *ps, int axis, const LineCfg &c)
{
    if (c.form == 1 || c.form == 2) return 0;
    int tsz = 0, sd = 1;
    for (int p = 0; p < ps->npatch; ++p) {
        const LineTabRef &r = ps->desc[p].line[axis][c.popt];
        tsz = std::max(tsz, line_table_size(r.Lr, r.P));
        sd = std::max(sd, ps->dims[3 * p] | 1);
    }
    // y/z lines: the chunk values of u and two buffers of chunk ends (the
    // table is read through the scalar cache); x lines: table, chunk ends, the
    // tile's rows, row offsets
    if (axis != 0) {
        // the update form's copy of u (16-cell chunks, or 32-cell chunks on at
        // most eight wavefronts: the kernels' uc_in_lds rule)
        const bool ucl = c.Lmax <= 16 || (c.Lmax == 32 && c.nwaves <= 8);
        return static_cast<size_t>((ucl ? c.Lmax : 0) + 4) * 64 * static_cast<size_t>(c.nwaves) * sizeof(double);
    }
    size_t n = static_cast<size_t>((tsz + 1) & ~1) + 2 * 64 * static_cast<size_t>(c.nwaves);
    n += 64 * static_cast<size_t>(sd) + 128;
    return n * sizeof(double);
}

bs_status check_line_cfg(const bs_patchset *ps, int axis, const LineCfg &c)
{
    if (c.form == 1) {
        if (axis != 0 || ps->max_n[0] > kXregMaxN)
            return fail(BS_ERR_UNSUPPORTED, "line config: register x-lines need axis 0 and nx <= %d", kXregMaxN);
        if (c.popt != 0 || c.Lmax != 4) return fail(BS_ERR_INVALID, "line config: bad register x-line form");
        if (c.nwaves != 1 && c.nwaves != 2 && c.nwaves != 4)
            return fail(BS_ERR_INVALID, "line config: register x-lines take 1, 2 or 4 wavefronts");
        if (c.grid < 0) return fail(BS_ERR_INVALID, "line config: negative grid");
        for (int p = 0; p < ps->npatch; ++p)
            if (ps->desc[p].line[0][0].off < 0)
                return fail(BS_ERR_UNSUPPORTED, "line config: patch %d has no x-line factor table", p);
        return BS_OK;
    }
    if (c.form == 2) {
        if (axis != 0 || ps->max_n[0] > kXregMaxN)
            return fail(BS_ERR_UNSUPPORTED, "line config: z-marching x-lines need axis 0 and nx <= %d", kXregMaxN);
        if (c.popt != 0 || c.Lmax != 4) return fail(BS_ERR_INVALID, "line config: bad z-marching x-line form");
        if (c.nwaves < 1 || c.nwaves > 4) return fail(BS_ERR_INVALID, "line config: z-marching x-lines take 1 to 4 wavefronts");
        if (c.zc < 1) return fail(BS_ERR_INVALID, "line config: z-marching x-lines need planes per item >= 1");
        if (c.grid < 0) return fail(BS_ERR_INVALID, "line config: negative grid");
        for (int p = 0; p < ps->npatch; ++p)
            if (ps->desc[p].line[0][0].off < 0)
                return fail(BS_ERR_UNSUPPORTED, "line config: patch %d has no x-line factor table", p);
        return BS_OK;
    }
    if (c.form != 0) return fail(BS_ERR_INVALID, "line config: unknown kernel form");
    if (c.popt < 0 || c.popt >= kNumPOpt) return fail(BS_ERR_INVALID, "line config: bad chunk option");
    if (c.nwaves != kPOpts[c.popt]) return fail(BS_ERR_INVALID, "line config: waves != chunk count");
    if (c.tx < 1 || c.tx > 64 || (c.tx & (c.tx - 1))) return fail(BS_ERR_INVALID, "line config: bad tile width");
    if (c.Lmax != 8 && c.Lmax != 16 && c.Lmax != 32 && c.Lmax != 64)
        return fail(BS_ERR_INVALID, "line config: bad register chunk");
    if (c.grid < 0) return fail(BS_ERR_INVALID, "line config: negative grid");
    for (int p = 0; p < ps->npatch; ++p) {
        const LineTabRef &r = ps->desc[p].line[axis][c.popt];
        if (r.off < 0 || r.Lr > c.Lmax)
            return fail(BS_ERR_UNSUPPORTED, "line config: patch %d axis %d has no chunk table for %d chunks", p, axis,
                        kPOpts[c.popt]);
    }
    if (line_lds_bytes(ps, axis, c) > 160 * 1024) return fail(BS_ERR_UNSUPPORTED, "line config: LDS exceeds 160 KiB");
    return BS_OK;
}

// One pass over the lines of `axis`: colour_mode 0 = all lines (one run);
// colour_mode 1 with run = 0 / 1 = that colour only, run = 2 = both colours in
// one launch, colour 0 dispatched first (chaotic).  patch >= 0 restricts the
// pass to one patch's items (one launch per patch and run).
bool pair_for(const bs_patchset *ps, int axis, const LineCfg &c, double omega, int f32)
{
    return axis != 0 && ps->use_pair && omega == 1.0 && !f32 && c.form == 0 && c.Lmax <= 32 && !bline_any(ps, axis) &&
           (c.Lmax <= 16 || c.nwaves <= 8) && pair_lds_bytes(c.Lmax, c.nwaves) <= 160 * 1024;
}

bs_status line_pass(bs_patchset *ps, int axis, const LineCfg &c, int colour_mode, int run, const double *src,
                    double *dst, const double *f, double omega, hipStream_t stream, int patch, int rhs_mode,
                    int out_mode, int f32, double *dst2)
{
    if (out_mode == 2 && (axis == 0 || colour_mode != 0 || rhs_mode || f32 || !dst2 || c.form != 0))
        return fail(BS_ERR_INVALID, "line pass: the two-output mode needs FP64 Jacobi on y/z lines");
    if (c.form == 2 && (rhs_mode || out_mode))
        return fail(BS_ERR_INVALID, "line pass: z-marching x-lines run plain sweeps only");
    // chaotic GS on y/z lines with omega = 1: two cells per lane (kind 3)
    const bool pair = colour_mode == 2 && !rhs_mode && !out_mode && pair_for(ps, axis, c, omega, f32);
    const int kind = pair ? 3 : (axis == 0 ? (c.form == 2 ? 2 : 1) : 0);
    if (kind == 2 && colour_mode == 1)
        return fail(BS_ERR_INVALID, "line pass: z-marching x-lines run Jacobi or chaotic GS only");
    WorkList *wl = nullptr;
    bs_status st = get_worklist(ps, kind, axis, kind == 2 ? c.nwaves : c.popt,
                                kind == 2 ? c.zc : (kind == 3 ? 128 : c.tx), colour_mode, &wl,
                                (colour_mode == 2 && kind != 2) ? chaotic_chunk_for(ps, axis, c) : 0);
    if (st != BS_OK) return st;
    LineArgs a{};
    a.src = src;
    a.dst = dst;
    a.f = f;
    a.pd = static_cast<const PatchDesc *>(ps->desc_d.p);
    a.tab = static_cast<const double *>(ps->tab_d.p);
    a.tab32 = static_cast<const float *>(ps->tab32_d.p);
    a.f32 = f32;
    // Jacobi on u, v and f that together exceed the Infinity Cache: f is
    // streamed past it so that u and v stay cached from sweep to sweep
    a.f_stream = (colour_mode == 0 && (2 * ps->u_numel + ps->f_numel) * static_cast<int64_t>(sizeof(double)) >
                                         kMallBytes) ? 1 : 0;
    a.axis = axis;
    a.popt = c.popt;
    a.tx = kind == 2 ? c.zc : c.tx;
    a.colour_mode = colour_mode;
    a.rhs_mode = rhs_mode;
    a.out_mode = out_mode;
    a.dst2 = dst2;
    a.omega = omega;
    a.direct = (kind == 0 && c.form == 0 && colour_mode == 0 && !rhs_mode && !out_mode && !f32 && ps->line_direct) ? 1 : 0;
    // the direct form keeps no chunk values of u: the two buffers of chunk ends only
    const size_t lds = a.direct ? 4 * 64 * static_cast<size_t>(c.nwaves) * sizeof(double) : line_lds_bytes(ps, axis, c);
    const WorkItem *base = static_cast<const WorkItem *>(wl->buf.p);
    auto launch = [&](int first, int count) -> bs_status {
        if (count <= 0) return BS_OK;
        a.items = base + first;
        a.nitems = count;
        const int grid = c.grid > 0 ? std::min(count, c.grid) : count;
        hipError_t e = pair         ? launch_line_pair(a, grid, c.Lmax, c.nwaves, stream)
                       : c.form == 2  ? launch_line_xz(a, grid, c.nwaves, stream)
                       : c.form == 1  ? launch_line_xr(a, grid, c.nwaves, stream)
                       : axis == 0  ? launch_line_x(a, grid, c.Lmax, c.nwaves, lds, stream)
                                    : launch_line_strided(a, grid, c.Lmax, c.nwaves, lds, stream);
        return e == hipSuccess ? BS_OK : hip_fail(e, "line sweep kernel");
    };
    if (colour_mode == 2) run = 2;   // in-tile two-colour: both tile-row groups in one pass
    if (kind == 2) {                 // one run in every mode
        if (patch >= 0) return launch(wl->pp_off[0] + wl->pfirst[0][patch], wl->pcount[0][patch]);
        return launch(0, wl->count[0]);
    }
    if (patch >= 0) {
        const int runs = colour_mode ? (run == 2 ? 2 : 1) : 1;
        for (int k = 0; k < runs; ++k) {
            const int cr = colour_mode ? (run == 2 ? k : run) : 0;
            if ((st = launch(wl->pp_off[cr] + wl->pfirst[cr][patch], wl->pcount[cr][patch])) != BS_OK) return st;
        }
        return BS_OK;
    }
    if (!colour_mode) return launch(0, wl->count[0]);
    if (run == 0) return launch(0, wl->count[0]);
    if (run == 1) return launch(wl->count[0], wl->count[1]);
    return launch(0, wl->count[0] + wl->count[1]);
}

const LineCfg &line_cfg(bs_patchset *ps, int axis, int colour_mode)
{
    auto key = std::make_pair(axis, colour_mode);
    auto itr = ps->line_cfg.find(key);
    if (itr == ps->line_cfg.end()) itr = ps->line_cfg.emplace(key, default_line_cfg(ps, axis, colour_mode)).first;
    return itr->second;
}

// Kernel mode of a scheme: Jacobi 0 (all lines, ping-pong); two-colour GS 1
// (one colour per launch); chaotic GS 2 (contiguous tiles, the two colours in
// turn inside each tile, even tile rows -- alternate row blocks for x lines --
// dispatched first).
int scheme_mode(int axis, bs_scheme scheme)
{
    (void)axis;
    if (scheme == BS_JACOBI) return 0;
    if (scheme == BS_CHAOTIC_GS) return 2;
    return 1;
}

// The launch sequence of nsweeps line sweeps.  per_patch: one launch per
// patch and colour run instead of one per run (the comparison baseline).
bs_status enqueue_line_sweeps(bs_patchset *ps, int axis, bs_scheme scheme, const LineCfg &c, double omega,
                              int nsweeps, double *u, const double *f, double *work, hipStream_t stream,
                              bool per_patch, int f32)
{
    const PatchDesc *pdd = static_cast<const PatchDesc *>(ps->desc_d.p);
    bs_status st;
    // lines next to extrapolated faces parallel to them (their own kernel), and
    // the ghost update after every sweep (links and extrapolated faces)
    const bool bl = bline_any(ps, axis);
    const bool gh = ghost_active(ps);
    auto pass = [&](int cm, int run, const double *src, double *dst) -> bs_status {
        if (!per_patch) return line_pass(ps, axis, c, cm, run, src, dst, f, omega, stream, -1, 0, 0, f32);
        for (int p = 0; p < ps->npatch; ++p) {
            bs_status s2 = line_pass(ps, axis, c, cm, run, src, dst, f, omega, stream, p, 0, 0, f32);
            if (s2 != BS_OK) return s2;
        }
        return BS_OK;
    };
    auto ghosts = [&](double *v, bool fill_only) -> bs_status {
        if (!gh) return BS_OK;
        hipError_t e = ghost_update(ps, v, fill_only, stream);
        return e == hipSuccess ? BS_OK : hip_fail(e, "ghost update");
    };
    if ((st = ghosts(u, true)) != BS_OK) return st;
    if (scheme == BS_JACOBI) {
        hipError_t e = launch_ghost_copy(u, work, pdd, ps->npatch, stream);
        if (e != hipSuccess) return hip_fail(e, "ghost copy");
        for (int s = 0; s < nsweeps; ++s) {
            const double *src = (s & 1) ? work : u;
            double *dst = (s & 1) ? u : work;
            if ((st = pass(0, 0, src, dst)) != BS_OK) return st;
            if (bl && (st = bline_pass(ps, axis, -1, src, dst, f, omega, stream)) != BS_OK) return st;
            if ((st = ghosts(dst, false)) != BS_OK) return st;
        }
        if (nsweeps & 1) {
            e = launch_interior_copy(work, u, pdd, ps->npatch, stream);
            if (e != hipSuccess) return hip_fail(e, "interior copy");
            if ((st = ghosts(u, false)) != BS_OK) return st;
        }
        return BS_OK;
    }
    const int cm = scheme_mode(axis, scheme);
    if (scheme == BS_CHAOTIC_GS && chaotic_colour_major(ps, axis, c)) {
        // every tile would run at once (or boundary lines have their own
        // kernel): colour-major in two launches (all colour-0 lines, then all
        // colour-1 lines), the two-colour sweep
        const LineCfg c1 = line_cfg(ps, axis, 1);
        for (int s = 0; s < nsweeps; ++s) {
            for (int run = 0; run < 2; ++run) {
                if (!per_patch) {
                    st = line_pass(ps, axis, c1, 1, run, u, u, f, omega, stream, -1, 0, 0, f32);
                } else {
                    st = BS_OK;
                    for (int p = 0; p < ps->npatch && st == BS_OK; ++p)
                        st = line_pass(ps, axis, c1, 1, run, u, u, f, omega, stream, p, 0, 0, f32);
                }
                if (st != BS_OK) return st;
                if (bl && (st = bline_pass(ps, axis, run, u, u, f, omega, stream)) != BS_OK) return st;
            }
            if ((st = ghosts(u, false)) != BS_OK) return st;
        }
        return BS_OK;
    }
    for (int s = 0; s < nsweeps; ++s) {
        if (scheme == BS_COLORED_GS) {
            if ((st = pass(cm, 0, u, u)) != BS_OK) return st;
            if (bl && (st = bline_pass(ps, axis, 0, u, u, f, omega, stream)) != BS_OK) return st;
            if ((st = pass(cm, 1, u, u)) != BS_OK) return st;
            if (bl && (st = bline_pass(ps, axis, 1, u, u, f, omega, stream)) != BS_OK) return st;
        } else {
            if ((st = pass(cm, 2, u, u)) != BS_OK) return st;
        }
        if ((st = ghosts(u, false)) != BS_OK) return st;
    }
    return BS_OK;
}

// Chaotic GS in one launch orders each XCD's tiles in chunks, even tile rows
// before odd ones, so that a chunk's odd tiles read their even neighbours' new
// values; that holds only if the odd tiles start after the even ones have
// finished, i.e. if a chunk is at least twice the workgroups an XCD holds at
// once.  The chunk is therefore sized from the configuration's occupancy.
int chaotic_chunk_for(bs_patchset *ps, int axis, const LineCfg &c)
{
    if (ps->chaotic_chunk > 0) return ps->chaotic_chunk;
    const std::vector<int> key{axis, c.form, c.popt, c.Lmax, c.nwaves, c.tx, c.grid};
    auto itr = ps->chaotic_chunks.find(key);
    if (itr != ps->chaotic_chunks.end()) return itr->second;
    const int occ = c.form == 1 ? line_xr_occupancy(c.nwaves, 0)
                                : line_occupancy(axis, c.Lmax, c.nwaves, line_lds_bytes(ps, axis, c), 2, 0);
    int64_t resident = static_cast<int64_t>(occ) * device_cus();
    if (c.grid > 0) resident = std::min<int64_t>(resident, c.grid);
    const int per_xcd = static_cast<int>(std::max<int64_t>(1, (resident + 7) / 8));
    const int chunk = std::max(ps->npatch == 1 ? 64 : 512, 2 * per_xcd);
    ps->chaotic_chunks.emplace(key, chunk);
    return chunk;
}

// With fewer tiles than one chunk per XCD, every tile runs at once and the
// one-launch order cannot act (the sweep would converge like block Jacobi
// across tile borders); such sweeps are dispatched colour-major instead.
bool chaotic_colour_major(bs_patchset *ps, int axis, const LineCfg &c)
{
    // lines next to extrapolated faces are solved by their own kernel, which
    // the in-tile two-colour form cannot interleave with
    if (bline_any(ps, axis)) return true;
    if (c.form == 2) return false;   // z-marching items order their own lines
    const int kind = axis == 0 ? 1 : 0;
    int64_t tiles = 0;
    for (int p = 0; p < ps->npatch; ++p) tiles += tiles_of(ps, p, kind, axis, c.tx, 2);
    return tiles < 8 * static_cast<int64_t>(chaotic_chunk_for(ps, axis, c));
}

// Build every work list a sequence needs before any capture begins.
bs_status prepare_lists(bs_patchset *ps, int axis, const LineCfg &c, int colour_mode)
{
    WorkList *wl;
    if (colour_mode == 2 && chaotic_colour_major(ps, axis, c)) {
        const LineCfg &c1 = line_cfg(ps, axis, 1);
        bs_status st = check_line_cfg(ps, axis, c1);
        if (st != BS_OK) return st;
        return get_worklist(ps, axis == 0 ? 1 : 0, axis, c1.popt, c1.tx, 1, &wl);
    }
    if (c.form == 2) return get_worklist(ps, 2, axis, c.nwaves, c.zc, colour_mode, &wl, 0);
    return get_worklist(ps, axis == 0 ? 1 : 0, axis, c.popt, c.tx, colour_mode, &wl,
                        colour_mode == 2 ? chaotic_chunk_for(ps, axis, c) : 0);
}

}  // namespace bs

bs_patchset::~bs_patchset()
{
    bs::clear_graphs(this);
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
}

using namespace bs;

namespace {

bs_status check_line_args(int32_t axis, bs_scheme scheme, double omega, int32_t nsweeps, bs_precision prec,
                          const char *fn)
{
    if (axis < 0 || axis > 2) return fail(BS_ERR_INVALID, "%s: axis must be 0, 1 or 2", fn);
    if (scheme != BS_JACOBI && scheme != BS_CHAOTIC_GS && scheme != BS_COLORED_GS)
        return fail(BS_ERR_INVALID, "%s: unknown scheme", fn);
    if (!(omega > 0.0 && omega < 2.0)) return fail(BS_ERR_INVALID, "%s: omega must be in (0, 2)", fn);
    if (nsweeps < 0) return fail(BS_ERR_INVALID, "%s: nsweeps < 0", fn);
    if (prec != BS_FP64 && prec != BS_MIXED_FP32 && prec != BS_MIXED_BF16)
        return fail(BS_ERR_INVALID, "%s: unknown precision", fn);
    if (prec == BS_MIXED_BF16) return fail(BS_ERR_UNSUPPORTED, "%s: BF16 is offered for planes only", fn);
    return BS_OK;
}

bs_status check_line_ps(const bs_patchset *ps, int32_t axis, const char *fn)
{
    if (ps->max_n[axis] > 16 * kMaxChunkLen)
        return fail(BS_ERR_UNSUPPORTED, "%s: lines longer than %d cells", fn, 16 * kMaxChunkLen);
    if (axis == 0 && ps->max_n[0] > 256) return fail(BS_ERR_UNSUPPORTED, "%s: x-lines longer than 256 cells", fn);
    return BS_OK;
}

}  // namespace

namespace bs {
bs_status check_line_ps_ext(const bs_patchset *ps, int32_t axis, const char *fn) { return check_line_ps(ps, axis, fn); }
}  // namespace bs

extern "C" {

bs_status bs_line_relax(bs_patchset *ps, int32_t axis, bs_scheme scheme, double omega, int32_t nsweeps,
                        bs_precision prec, double *u, const double *f, double *work, hipStream_t stream)
{
    return line_relax_impl(ps, axis, scheme, omega, nsweeps, prec, u, f, work, stream, true);
}

}  // extern "C"

namespace bs {

bs_status line_relax_impl(bs_patchset *ps, int32_t axis, bs_scheme scheme, double omega, int32_t nsweeps,
                          bs_precision prec, double *u, const double *f, double *work, hipStream_t stream,
                          bool allow_graph)
{
    bs_status st = check_line_args(axis, scheme, omega, nsweeps, prec, "bs_line_relax");
    if (st != BS_OK) return st;
    if (!ps || !u || !f) return fail(BS_ERR_INVALID, "bs_line_relax: null patch set, u or f");
    if (scheme == BS_JACOBI && !work) return fail(BS_ERR_INVALID, "bs_line_relax: Jacobi needs a work buffer");
    if ((st = check_line_ps(ps, axis, "bs_line_relax")) != BS_OK) return st;
    if (nsweeps == 0) return BS_OK;
    const int cm = scheme_mode(axis, scheme);
    const int f32 = prec == BS_MIXED_FP32 ? 1 : 0;
    // the default configuration is chosen for the direct-form Jacobi and the
    // two-cells-per-lane chaotic kernels; FP32 solves and chaotic GS with
    // omega != 1 (the update form) take their own
    LineCfg c = line_cfg(ps, axis, cm);
    if (c.deflt && (f32 || (cm == 2 && omega != 1.0))) c = default_line_cfg(ps, axis, cm, false);
    if ((st = check_line_cfg(ps, axis, c)) != BS_OK) return st;
    if ((st = prepare_lists(ps, axis, c, cm)) != BS_OK) return st;
    if (bline_any(ps, axis) && (st = bline_prepare(ps, axis)) != BS_OK) return st;
    hipError_t e = prepare_line_kernels();
    if (e != hipSuccess) return hip_fail(e, "line kernel attributes");
    if (cm == 2 && !chaotic_colour_major(ps, axis, c) && pair_for(ps, axis, c, omega, f32)) {
        WorkList *wl;
        if ((st = get_worklist(ps, 3, axis, c.popt, 128, 2, &wl, chaotic_chunk_for(ps, axis, c))) != BS_OK) return st;
        if ((e = prepare_pair_kernels()) != hipSuccess) return hip_fail(e, "line kernel attributes");
    }
    if (!allow_graph || !ps->use_graphs || nsweeps < 2)
        return enqueue_line_sweeps(ps, axis, scheme, c, omega, nsweeps, u, f, work, stream, false, f32);

    // replay a captured graph of the whole sequence (captured on first use)
    int64_t obits;
    std::memcpy(&obits, &omega, sizeof obits);
    const std::vector<int64_t> key{0, axis, scheme, obits, nsweeps, reinterpret_cast<int64_t>(u),
                                   reinterpret_cast<int64_t>(f), reinterpret_cast<int64_t>(work), c.popt, c.tx,
                                   c.grid, c.Lmax, f32};
    auto itr = ps->graphs.find(key);
    if (itr == ps->graphs.end()) {
        if (ps->graphs.size() >= 64) clear_graphs(ps);
        if (!ps->capture_stream &&
            (e = hipStreamCreateWithFlags(&ps->capture_stream, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "capture stream");
        hipGraph_t graph = nullptr;
        if ((e = hipStreamBeginCapture(ps->capture_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(e, "hipStreamBeginCapture");
        st = enqueue_line_sweeps(ps, axis, scheme, c, omega, nsweeps, u, f, work, ps->capture_stream, false, f32);
        e = hipStreamEndCapture(ps->capture_stream, &graph);
        if (st != BS_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        itr = ps->graphs.emplace(key, exec).first;
    }
    if ((e = hipGraphLaunch(itr->second, stream)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return BS_OK;
}

}  // namespace bs

extern "C" {

bs_status bs_autotune_line(bs_patchset *ps, int32_t axis, bs_scheme scheme, const double *u, const double *f,
                           hipStream_t stream)
{
    bs_status st = check_line_args(axis, scheme, 1.0, 1, BS_FP64, "bs_autotune_line");
    if (st != BS_OK) return st;
    if (!ps || !u || !f) return fail(BS_ERR_INVALID, "bs_autotune_line: null patch set, u or f");
    if ((st = check_line_ps(ps, axis, "bs_autotune_line")) != BS_OK) return st;
    hipError_t e = prepare_line_kernels();
    if (e != hipSuccess) return hip_fail(e, "line kernel attributes");
    if (bline_any(ps, axis) && (st = bline_prepare(ps, axis)) != BS_OK) return st;
    const int cm = scheme_mode(axis, scheme);
    DevBuf su, sw;
    const size_t bytes = static_cast<size_t>(ps->u_numel) * sizeof(double);
    if ((st = dev_alloc(su, bytes, "autotune scratch")) != BS_OK) return st;
    if ((st = dev_alloc(sw, bytes, "autotune scratch")) != BS_OK) return st;
    if ((e = hipMemcpyAsync(su.p, u, bytes, hipMemcpyDeviceToDevice, stream)) != hipSuccess) return hip_fail(e, "copy");
    if ((e = hipMemcpyAsync(sw.p, u, bytes, hipMemcpyDeviceToDevice, stream)) != hipSuccess) return hip_fail(e, "copy");
    std::vector<LineCfg> cands;
    const int cus = device_cus();
    for (int o = 0; o < kNumPOpt; ++o) {
        int lr_max = 0;
        bool ok = true;
        for (int p = 0; p < ps->npatch; ++p) {
            const LineTabRef &r = ps->desc[p].line[axis][o];
            if (r.off < 0) ok = false;
            lr_max = std::max(lr_max, r.Lr);
        }
        if (!ok) continue;
        const int Lmax = lmax_for(lr_max);
        // shapes that would spill registers on gfx950 are not candidates
        if ((Lmax == 32 && kPOpts[o] > 8) || (Lmax == 64 && kPOpts[o] > 4)) continue;
        for (int tx : {64, 32, 16, 8}) {
            if (axis == 0 && tx != 64) continue;
            for (int grid : {0, 4 * cus, 8 * cus}) {
                LineCfg c;
                c.popt = o;
                c.nwaves = kPOpts[o];
                c.Lmax = Lmax;
                c.tx = tx;
                c.grid = grid;
                if (check_line_cfg(ps, axis, c) == BS_OK) cands.push_back(c);
            }
        }
    }
    if (axis == 0 && ps->max_n[0] <= kXregMaxN && cm != 1) {
        // x-lines marched along z (Jacobi and chaotic GS)
        for (int nw : {2, 4}) {
            const int zc0 = xz_planes(ps, nw);
            for (int zc : {zc0, std::max(1, zc0 / 4)}) {
                LineCfg c;
                c.form = 2;
                c.popt = 0;
                c.Lmax = 4;
                c.nwaves = nw;
                c.zc = zc;
                c.tx = 64;
                c.grid = 0;
                if (check_line_cfg(ps, axis, c) == BS_OK) cands.push_back(c);
                if (zc0 <= 4) break;
            }
        }
    }
    if (axis == 0 && ps->max_n[0] <= kXregMaxN) {
        for (int nw : {1, 2, 4}) {
            LineCfg c;
            c.form = 1;
            c.popt = 0;
            c.Lmax = 4;
            c.nwaves = nw;
            c.tx = 64;
            c.grid = 0;
            if (check_line_cfg(ps, axis, c) == BS_OK) cands.push_back(c);
        }
    }
    if (cands.empty()) return fail(BS_ERR_UNSUPPORTED, "bs_autotune_line: no valid configuration");
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "event");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "event");
    }
    double best_ms = 1e30;
    LineCfg best = cands[0];
    double *pu = static_cast<double *>(su.p), *pw = static_cast<double *>(sw.p);
    for (const LineCfg &c : cands) {
        if ((st = prepare_lists(ps, axis, c, cm)) != BS_OK) break;
        double tmin = 1e30;
        for (int rep = 0; rep < 4 && st == BS_OK; ++rep) {
            (void)hipEventRecord(e0, stream);
            st = enqueue_line_sweeps(ps, axis, scheme, c, scheme == BS_JACOBI ? 0.8 : 1.0, 2, pu, f, pw, stream,
                                     false);
            (void)hipEventRecord(e1, stream);
            if ((e = hipEventSynchronize(e1)) != hipSuccess) {
                st = hip_fail(e, "autotune timing");
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) tmin = std::min(tmin, static_cast<double>(ms));
        }
        if (st != BS_OK) break;
        if (tmin < best_ms) {
            best_ms = tmin;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != BS_OK) return st;
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "autotune");
    best.tuned = 1;
    ps->line_cfg[std::make_pair(static_cast<int>(axis), cm)] = best;
    clear_graphs(ps);
    return BS_OK;
}

bs_status bs_line_config(const bs_patchset *ps, int32_t axis, bs_scheme scheme, int32_t cfg_host[6])
{
    if (!ps || !cfg_host) return fail(BS_ERR_INVALID, "bs_line_config: null argument");
    if (axis < 0 || axis > 2) return fail(BS_ERR_INVALID, "bs_line_config: axis must be 0, 1 or 2");
    const int cm = scheme_mode(axis, scheme);
    auto itr = ps->line_cfg.find(std::make_pair(static_cast<int>(axis), cm));
    const bool set = itr != ps->line_cfg.end();
    const LineCfg c = set ? itr->second : default_line_cfg(ps, axis, cm);
    cfg_host[0] = c.form != 0 ? c.nwaves : kPOpts[c.popt];
    cfg_host[1] = c.Lmax;
    cfg_host[2] = c.form == 2 ? c.zc : c.tx;
    cfg_host[3] = c.grid;
    cfg_host[4] = c.tuned;
    cfg_host[5] = c.form;
    return BS_OK;
}

// Host-side hooks (not part of the public header).

// Set the launch configuration of line sweeps along `axis` for one scheme:
// popt indexes the chunk counts {1,2,4,8,16}; tx is the strided kernel's lanes
// per row; grid is the persistent grid size (0: one workgroup per work item).
int bsi_set_line_cfg(bs_patchset *ps, int axis, int scheme, int popt, int tx, int grid)
{
    if (!ps || axis < 0 || axis > 2 || scheme < 0 || scheme > 2) return BS_ERR_INVALID;
    const int colour_mode = scheme_mode(axis, static_cast<bs_scheme>(scheme));
    if (popt < 0 || popt >= kNumPOpt) return BS_ERR_INVALID;
    LineCfg c;
    c.popt = popt;
    c.nwaves = kPOpts[popt];
    c.tx = tx;
    c.grid = grid;
    int lr_max = 0;
    for (int p = 0; p < ps->npatch; ++p) {
        if (ps->desc[p].line[axis][popt].off < 0) return BS_ERR_UNSUPPORTED;
        lr_max = std::max(lr_max, ps->desc[p].line[axis][popt].Lr);
    }
    c.Lmax = lmax_for(lr_max);
    bs_status st = check_line_cfg(ps, axis, c);
    if (st != BS_OK) return st;
    ps->line_cfg[std::make_pair(axis, colour_mode)] = c;
    clear_graphs(ps);
    return BS_OK;
}

// Select the register x-line kernel (lines across the lanes of a 16-lane row)
// for `scheme`, with nwaves wavefronts per workgroup and a persistent grid
// (0: one workgroup per work item).
int bsi_set_xline_cfg(bs_patchset *ps, int scheme, int nwaves, int grid)
{
    if (!ps || scheme < 0 || scheme > 2) return BS_ERR_INVALID;
    const int colour_mode = scheme_mode(0, static_cast<bs_scheme>(scheme));
    LineCfg c;
    c.form = 1;
    c.popt = 0;
    c.Lmax = 4;
    c.nwaves = nwaves;
    c.tx = 64;
    c.grid = grid;
    bs_status st = check_line_cfg(ps, 0, c);
    if (st != BS_OK) return st;
    ps->line_cfg[std::make_pair(0, colour_mode)] = c;
    clear_graphs(ps);
    return BS_OK;
}

// Select the z-marching x-line kernel for `scheme` (Jacobi or chaotic GS):
// nwaves wavefronts per workgroup, zc planes per item (0: the default),
// persistent grid size (0: one workgroup per item).
int bsi_set_xz_cfg(bs_patchset *ps, int scheme, int nwaves, int zc, int grid)
{
    if (!ps || (scheme != BS_JACOBI && scheme != BS_CHAOTIC_GS) || zc < 0) return BS_ERR_INVALID;
    const int colour_mode = scheme_mode(0, static_cast<bs_scheme>(scheme));
    LineCfg c;
    c.form = 2;
    c.popt = 0;
    c.Lmax = 4;
    c.nwaves = nwaves;
    c.zc = zc > 0 ? zc : (nwaves >= 1 && nwaves <= 4 ? xz_planes(ps, nwaves) : 1);
    c.tx = 64;
    c.grid = grid;
    bs_status st = check_line_cfg(ps, 0, c);
    if (st != BS_OK) return st;
    ps->line_cfg[std::make_pair(0, colour_mode)] = c;
    clear_graphs(ps);
    return BS_OK;
}

// Tiles per even/odd chunk of the chaotic dispatch order (0: default).
int bsi_set_chaotic_chunk(bs_patchset *ps, int tiles)
{
    if (!ps || tiles < 0) return BS_ERR_INVALID;
    ps->chaotic_chunk = tiles;
    ps->chaotic_chunks.clear();
    ps->lists.clear();
    clear_graphs(ps);
    return BS_OK;
}

// Enable (1) or disable (0) the two-cells-per-lane chaotic kernel for y/z
// lines with omega 1 (disabled: the one-line-per-lane in-tile two-colour form).
int bsi_set_pair(bs_patchset *ps, int enable)
{
    if (!ps) return BS_ERR_INVALID;
    ps->use_pair = enable != 0;
    // default configurations depend on the kernel: chosen again on next use
    for (auto it = ps->line_cfg.begin(); it != ps->line_cfg.end();) {
        if (it->second.deflt)
            it = ps->line_cfg.erase(it);
        else
            ++it;
    }
    clear_graphs(ps);
    return BS_OK;
}

// Enable (1, the default) or disable (0) the direct form of Jacobi on y/z lines
// (dst = M^{-1}(omega b + (1 - omega) M src)); disabled, the kernel keeps u for
// the update dst = src + omega M^{-1} r.
int bsi_set_line_direct(bs_patchset *ps, int enable)
{
    if (!ps) return BS_ERR_INVALID;
    ps->line_direct = enable != 0;
    // default configurations depend on the form: chosen again on next use
    for (auto it = ps->line_cfg.begin(); it != ps->line_cfg.end();) {
        if (it->second.deflt)
            it = ps->line_cfg.erase(it);
        else
            ++it;
    }
    clear_graphs(ps);
    return BS_OK;
}

// Enable (1) or disable (0) graph capture of sweep sequences.
int bsi_set_graphs(bs_patchset *ps, int enable)
{
    if (!ps) return BS_ERR_INVALID;
    ps->use_graphs = enable != 0;
    return BS_OK;
}

// The same sweeps as bs_line_relax with one launch per patch and colour run
// (no graph): the per-patch baseline that one batched launch replaces.
int bsi_line_relax_per_patch(bs_patchset *ps, int32_t axis, bs_scheme scheme, double omega, int32_t nsweeps,
                             double *u, const double *f, double *work, hipStream_t stream)
{
    bs_status st = check_line_args(axis, scheme, omega, nsweeps, BS_FP64, "bsi_line_relax_per_patch");
    if (st != BS_OK) return st;
    if (!ps || !u || !f || (scheme == BS_JACOBI && !work)) return BS_ERR_INVALID;
    if ((st = check_line_ps(ps, axis, "bsi_line_relax_per_patch")) != BS_OK) return st;
    const int cm = scheme_mode(axis, scheme);
    const LineCfg c = line_cfg(ps, axis, cm);
    if ((st = check_line_cfg(ps, axis, c)) != BS_OK) return st;
    if ((st = prepare_lists(ps, axis, c, cm)) != BS_OK) return st;
    if (bline_any(ps, axis) && (st = bline_prepare(ps, axis)) != BS_OK) return st;
    if (prepare_line_kernels() != hipSuccess) return BS_ERR_HIP;
    if (prepare_pair_kernels() != hipSuccess) return BS_ERR_HIP;
    return enqueue_line_sweeps(ps, axis, scheme, c, omega, nsweeps, u, f, work, stream, true);
}

}  // extern "C"
