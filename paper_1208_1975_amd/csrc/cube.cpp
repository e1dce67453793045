// Geometric cube blocks: the paper's own block kind (section 2: geometric
// blocks of bx x by x bz cells in lexicographic order; the block Jacobi
// algorithm on GPUs; the block-inversion section).  Each block's correction is
// the precomputed dense inverse of its block matrix applied to its residual:
//   step 1  R[block][cell] = h^2 f - A u          (k_cube_resid)
//   step 2  DU = R Ainv^T                          (FP64 matrix cores)
//   step 3  u' = u + omega DU                      (the product's epilogue)
// for blocks of more than 256 cells, or all three in one kernel, one launch
// per operand size for every patch class and shape of the set: k_cube_small
// for blocks of up to 64 cells (inverse in LDS), k_cube_big for 65 to 256
// (residuals in LDS, inverse read from memory).  For 512-cell blocks the
// fused form measured slower than the two kernels (0.58 against 0.52 ms per
// sweep of 64 x 64^3): its 32 x 512 FP64 accumulators per workgroup leave one
// workgroup per compute unit, with nothing to hide its loads behind.
// fused_max (a test hook) can lower the size limit of the fused kernels.
// The blocks of a patch of equal shape share one inverse (constant
// coefficients), so step 2 is one dense product per shape: the blocks are the
// rows, which is what makes it a matrix-core contraction rather than the
// paper's one matrix-vector product per thread block.
//
// Where an edge of the patch is not a multiple of the block edge, the last
// block along that axis is shorter and has its own inverse (the block-inversion
// section's option of precomputing every inverse; at most 8 shapes a patch).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <tuple>
#include <vector>

#include "patchset.h"
#include "plane.h"
#include "relax.h"
#include "tables.h"

namespace bs {

namespace {

constexpr int kCubeMaxCells = 512;                      // cells per block (8^3, the paper's largest)
constexpr int64_t kCubeMaxInvBytes = int64_t(1) << 30;  // all inverses of one block size

// Orthonormal eigenbasis V[i][p] of the 1D block operator tridiag(-1, 2, -1)
// of order n, with its first / last diagonal entry raised by one where the
// block touches an extrapolated face at that end (lo / hi), and its
// eigenvalues: the DST-I basis with neither, DST-II with both, the one-sided
// sine basis with one (closed forms in tables.cpp).
void block_basis(int n, int lo, int hi, std::vector<double> &V, std::vector<double> &sig)
{
    V = bc_sine_basis(n, lo, hi);
    const std::vector<long double> s = bc_sine_eigenvalues(n, 1.0, lo, hi);
    sig.assign(s.begin(), s.end());
}

// Dense inverse of the block matrix of an ni x nj x nk block,
//   A_b = ex (I (x) I (x) T_ni) + ey (I (x) T_nj (x) I) + ez (T_nk (x) I (x) I),
// (the stencil restricted to the block; T_n = tridiag(-1, 2, -1), with an end
// diagonal raised by one where the block touches an extrapolated face: bits of
// `raise`, 2a low / 2a+1 high end of axis a), from its eigen-decomposition:
// A_b^{-1} = S diag(1/lambda) S^T with S = S_k (x) S_j (x) S_i orthonormal and
// lambda_pqr = ex sig_p + ey sig_q + ez sig_r.  Column c' is
// S (lambda^{-1} .* S^T e_c'), S^T e_c' being the product of one row of each
// basis; the outer S is applied one axis at a time.  Cells are numbered x
// fastest.
void block_inverse(int ni, int nj, int nk, double ex, double ey, double ez, int raise, double *out)
{
    std::vector<double> Si, Sj, Sk, si, sj, sk;
    block_basis(ni, raise & 1, (raise >> 1) & 1, Si, si);
    block_basis(nj, (raise >> 2) & 1, (raise >> 3) & 1, Sj, sj);
    block_basis(nk, (raise >> 4) & 1, (raise >> 5) & 1, Sk, sk);
    const int nb = ni * nj * nk;
    std::vector<double> w(nb), t1(nb), t2(nb);
    for (int ck2 = 0; ck2 < nk; ++ck2)
        for (int cj2 = 0; cj2 < nj; ++cj2)
            for (int ci2 = 0; ci2 < ni; ++ci2) {
                const int col = (ck2 * nj + cj2) * ni + ci2;
                for (int r = 0; r < nk; ++r)
                    for (int q = 0; q < nj; ++q)
                        for (int p = 0; p < ni; ++p)
                            w[(r * nj + q) * ni + p] = Si[size_t(ci2) * ni + p] * Sj[size_t(cj2) * nj + q] *
                                                       Sk[size_t(ck2) * nk + r] /
                                                       (ex * si[p] + ey * sj[q] + ez * sk[r]);
                for (int r = 0; r < nk; ++r)   // along x
                    for (int q = 0; q < nj; ++q)
                        for (int ci = 0; ci < ni; ++ci) {
                            double acc = 0.0;
                            for (int p = 0; p < ni; ++p) acc += Si[size_t(ci) * ni + p] * w[(r * nj + q) * ni + p];
                            t1[(r * nj + q) * ni + ci] = acc;
                        }
                for (int r = 0; r < nk; ++r)   // along y
                    for (int cj = 0; cj < nj; ++cj)
                        for (int ci = 0; ci < ni; ++ci) {
                            double acc = 0.0;
                            for (int q = 0; q < nj; ++q) acc += Sj[size_t(cj) * nj + q] * t1[(r * nj + q) * ni + ci];
                            t2[(r * nj + cj) * ni + ci] = acc;
                        }
                for (int ck = 0; ck < nk; ++ck)   // along z
                    for (int cj = 0; cj < nj; ++cj)
                        for (int ci = 0; ci < ni; ++ci) {
                            double acc = 0.0;
                            for (int r = 0; r < nk; ++r) acc += Sk[size_t(ck) * nk + r] * t2[(r * nj + cj) * ni + ci];
                            out[size_t((ck * nj + cj) * ni + ci) * nb + col] = acc;
                        }
            }
}

// Host image of a plan's device buffer: 256-byte aligned pieces.
struct HostImage {
    std::vector<char> bytes;
    int64_t put(const void *src, size_t n)
    {
        const int64_t off = int64_t((bytes.size() + 255) & ~size_t(255));
        bytes.resize(size_t(off) + n);
        if (n) std::memcpy(bytes.data() + off, src, n);
        return off;
    }
};

bs_status build_plan(const bs_patchset *ps, int bx, int by, int bz, CubePlan &plan)
{
    // classes of patches with equal dims, eps, h and extrapolated faces share
    // inverses and offsets
    using ClassKey = std::tuple<int, int, int, double, double, double, double, int>;
    std::vector<std::pair<ClassKey, std::vector<int>>> classes;
    for (int p = 0; p < ps->npatch; ++p) {
        const ClassKey k{ps->dims[3 * p], ps->dims[3 * p + 1], ps->dims[3 * p + 2], ps->eps[3 * p],
                         ps->eps[3 * p + 1], ps->eps[3 * p + 2], ps->h[p], ps->bc[p]};
        auto it = std::find_if(classes.begin(), classes.end(), [&](const auto &c) { return c.first == k; });
        if (it == classes.end()) classes.push_back({k, {p}});
        else it->second.push_back(p);
    }
    HostImage img;
    int64_t rmax = 0, inv_bytes = 0;
    plan.groups.clear();
    for (const auto &cl : classes) {
        const int nx = std::get<0>(cl.first), ny = std::get<1>(cl.first), nz = std::get<2>(cl.first);
        const double ex = std::get<3>(cl.first), ey = std::get<4>(cl.first), ez = std::get<5>(cl.first);
        const double h = std::get<6>(cl.first);
        const int bcm = std::get<7>(cl.first);
        const int cb[3] = {std::min(bx, nx), std::min(by, ny), std::min(bz, nz)};
        const int n[3] = {nx, ny, nz};
        const int64_t SY = nx + 2, SZ = int64_t(nx + 2) * (ny + 2);
        // per axis, the blocks' origins grouped by (edge, touches an
        // extrapolated low face, touches an extrapolated high face): the full
        // edge and, if the axis is not a multiple of it, the remainder
        struct Seg {
            int size, lo, hi;
            std::vector<int> origins;
        };
        std::vector<Seg> segs[3];
        for (int a = 0; a < 3; ++a)
            for (int o = 0; o < n[a]; o += cb[a]) {
                const int size = std::min(cb[a], n[a] - o);
                const int lo = (o == 0 && ((bcm >> (2 * a)) & 1)) ? 1 : 0;
                const int hi = (o + size == n[a] && ((bcm >> (2 * a + 1)) & 1)) ? 1 : 0;
                auto it = std::find_if(segs[a].begin(), segs[a].end(),
                                       [&](const Seg &sg) { return sg.size == size && sg.lo == lo && sg.hi == hi; });
                if (it == segs[a].end()) segs[a].push_back(Seg{size, lo, hi, {o}});
                else it->origins.push_back(o);
            }
        for (const Seg &gx : segs[0])
            for (const Seg &gy : segs[1])
                for (const Seg &gz : segs[2]) {
                    const int sx = gx.size, sy = gy.size, sz = gz.size;
                    const int raise = gx.lo | (gx.hi << 1) | (gy.lo << 2) | (gy.hi << 3) | (gz.lo << 4) | (gz.hi << 5);
                    const int nb = sx * sy * sz;
                    inv_bytes += int64_t(nb) * nb * 8;
                    if (inv_bytes > kCubeMaxInvBytes)
                        return fail(BS_ERR_UNSUPPORTED,
                                    "bs_cube_prepare: the block inverses of this patch set exceed %lld bytes",
                                    (long long)kCubeMaxInvBytes);
                    CubeGroup g;
                    g.nb = nb;
                    g.ex = ex;
                    g.ey = ey;
                    g.ez = ez;
                    g.h2 = h * h;
                    g.sy = SY;
                    g.sz = SZ;
                    std::vector<double> inv(size_t(nb) * nb);
                    block_inverse(sx, sy, sz, ex, ey, ez, raise, inv.data());
                    g.o_ainv = img.put(inv.data(), inv.size() * 8);
                    std::vector<int32_t> uo(nb), fo(nb);
                    for (int ck = 0; ck < sz; ++ck)
                        for (int cj = 0; cj < sy; ++cj)
                            for (int ci = 0; ci < sx; ++ci) {
                                const int c = (ck * sy + cj) * sx + ci;
                                uo[c] = int32_t(ck * SZ + cj * SY + ci);
                                fo[c] = int32_t((int64_t(ck) * ny + cj) * nx + ci);
                            }
                    g.o_uoff = img.put(uo.data(), uo.size() * 4);
                    g.o_foff = img.put(fo.data(), fo.size() * 4);
                    const std::vector<int> &oi = gx.origins, &oj = gy.origins, &ok = gz.origins;
                    // Block lists in dispatch order: x fastest, then y within a band of
                    // G block rows, then z, then the next band, so that a run of 64
                    // blocks (one workgroup of the fused kernel) is a slab one block
                    // thick in z and the next run is its z-neighbour: the face both
                    // read is fetched once into the XCD's L2.  `want`: the colour to
                    // list (-1: every block, the Jacobi list).
                    std::vector<int64_t> ub, fb;
                    auto emit = [&](int want) {
                        const int per_row = want < 0 ? int(oi.size()) : int(oi.size() + 1) / 2;
                        const int G = std::max(1, 64 / std::max(1, per_row));
                        for (int p : cl.second)
                            for (size_t jg = 0; jg < oj.size(); jg += G)
                                for (int k0 : ok)
                                    for (size_t jj = jg; jj < std::min(oj.size(), jg + G); ++jj)
                                        for (int i0 : oi) {
                                            const int j0 = oj[jj];
                                            const int col = (i0 / cb[0] + j0 / cb[1] + k0 / cb[2]) & 1;
                                            if (want >= 0 && col != want) continue;
                                            ub.push_back(ps->uoff[p] + (k0 + 1) * SZ + (j0 + 1) * SY + (i0 + 1));
                                            fb.push_back(ps->foff[p] + (int64_t(k0) * ny + j0) * nx + i0);
                                        }
                    };
                    emit(-1);
                    g.nblk = int(ub.size());
                    g.o_jbase = img.put(ub.data(), ub.size() * 8);
                    g.o_jfbase = img.put(fb.data(), fb.size() * 8);
                    ub.clear();
                    fb.clear();
                    emit(0);
                    g.ncol0 = int(ub.size());
                    emit(1);
                    g.o_ubase = img.put(ub.data(), ub.size() * 8);
                    g.o_fbase = img.put(fb.data(), fb.size() * 8);
                    if (nb > ps->cube_fused_max) rmax = std::max(rmax, int64_t(g.nblk) * nb);
                    plan.groups.push_back(g);
                }
    }
    bs_status st = upload(plan.buf, img.bytes.data(), img.bytes.size(), "cube tables");
    if (st != BS_OK) return st;
    // every group in one launch per operand size and list (chunks of 64
    // blocks for the small-block kernel, 32 for the large-block one)
    const char *base = static_cast<const char *>(plan.buf.p);
    std::vector<CubeGroupDev> gd;
    std::vector<CubeChunk> lists[5][3];
    for (const CubeGroup &g : plan.groups) {
        const int gi = int(gd.size());
        CubeGroupDev d{};
        d.ainv = reinterpret_cast<const double *>(base + g.o_ainv);
        d.uoff = reinterpret_cast<const int32_t *>(base + g.o_uoff);
        d.foff = reinterpret_cast<const int32_t *>(base + g.o_foff);
        d.ubase[0] = reinterpret_cast<const int64_t *>(base + g.o_ubase);
        d.fbase[0] = reinterpret_cast<const int64_t *>(base + g.o_fbase);
        d.ubase[1] = reinterpret_cast<const int64_t *>(base + g.o_jbase);
        d.fbase[1] = reinterpret_cast<const int64_t *>(base + g.o_jfbase);
        d.nb = g.nb;
        d.sy = g.sy;
        d.sz = g.sz;
        d.ex = g.ex;
        d.ey = g.ey;
        d.ez = g.ez;
        d.h2 = g.h2;
        gd.push_back(d);
        if (g.nb > ps->cube_fused_max) continue;   // residual matrix and product (cube_pass)
        const int npc = g.nb <= 16 ? 0 : g.nb <= 32 ? 1 : g.nb <= 64 ? 2 : g.nb <= 128 ? 3 : 4;
        const int per = npc < 3 ? 64 : kCubeBigChunk;
        auto cut = [&](std::vector<CubeChunk> &v, int lo, int hi) {
            for (int b = lo; b < hi; b += per) v.push_back(CubeChunk{gi, b, std::min(b + per, hi), 0});
        };
        cut(lists[npc][0], 0, g.nblk);        // Jacobi: the colour-free list
        cut(lists[npc][1], 0, g.ncol0);       // colour 0 of the colour-major list
        cut(lists[npc][2], g.ncol0, g.nblk);  // colour 1
    }
    std::vector<CubeChunk> all;
    for (int p = 0; p < 5; ++p)
        for (int k = 0; k < 3; ++k) {
            plan.chunk_off[p][k] = int(all.size());
            plan.chunk_cnt[p][k] = int(lists[p][k].size());
            all.insert(all.end(), lists[p][k].begin(), lists[p][k].end());
        }
    if ((st = upload(plan.gdesc, gd.data(), gd.size() * sizeof(CubeGroupDev), "cube group descriptors")) != BS_OK)
        return st;
    if ((st = upload(plan.chunks, all.data(), all.size() * sizeof(CubeChunk), "cube chunk lists")) != BS_OK)
        return st;
    plan.inv_bytes = inv_bytes;
    plan.fused_max = ps->cube_fused_max;
    if (plan.rbuf.bytes < size_t(rmax) * 8 &&
        (st = dev_alloc(plan.rbuf, size_t(rmax) * 8, "cube residual scratch")) != BS_OK)
        return st;
    return BS_OK;
}

// Steps 1-3 for blocks [lo, lo + n) of a group of blocks over fused_max cells:
// src -> dst, in two kernels.
bs_status cube_pass(const CubePlan &plan, const CubeGroup &g, bool jacobi, int lo, int n, const double *src,
                    double *dst, const double *f, double omega, hipStream_t stream)
{
    if (n <= 0) return BS_OK;
    const char *base = static_cast<const char *>(plan.buf.p);
    const int64_t *ub = reinterpret_cast<const int64_t *>(base + (jacobi ? g.o_jbase : g.o_ubase)) + lo;
    const int64_t *fb = reinterpret_cast<const int64_t *>(base + (jacobi ? g.o_jfbase : g.o_fbase)) + lo;
    const int32_t *uo = reinterpret_cast<const int32_t *>(base + g.o_uoff);
    // blocks of over 64 cells: residual gather, then the product
    CubeArgs a{};
    a.u = src;
    a.f = f;
    a.R = static_cast<double *>(plan.rbuf.p);
    a.ubase = ub;
    a.fbase = fb;
    a.uoff = uo;
    a.foff = reinterpret_cast<const int32_t *>(base + g.o_foff);
    a.nb = g.nb;
    a.nblk = n;
    a.per = g.nb >= 256 ? 1 : 256 / g.nb;
    a.sy = g.sy;
    a.sz = g.sz;
    a.ex = g.ex;
    a.ey = g.ey;
    a.ez = g.ez;
    a.h2 = g.h2;
    hipError_t e = launch_cube_resid(a, stream);
    if (e != hipSuccess) return hip_fail(e, "cube residual");
    GemmArgs m{};
    m.A = a.R;
    m.lda = g.nb;
    m.B = reinterpret_cast<const double *>(base + g.o_ainv);
    m.ldb = g.nb;
    m.M = n;
    m.N = g.nb;
    m.K = g.nb;
    m.batch = 1;
    m.b_trans = 1;
    m.usrc = src;
    m.udst = dst;
    m.omega = omega;
    m.ebase = ub;
    m.eoff = uo;
    e = launch_gemm_f64(m, kEpiGather, stream);
    if (e != hipSuccess) return hip_fail(e, "cube block product");
    return BS_OK;
}

// Blocks of every group, list k (0 Jacobi, 1 colour 0, 2 colour 1): one
// fused launch per operand size (big: the sizes over 64 cells, else those up
// to 64).
bs_status small_pass(const CubePlan &plan, int k, const double *src, double *dst, const double *f, double omega,
                     hipStream_t stream, bool big = false)
{
    for (int p = big ? 3 : 0; p < (big ? 5 : 3); ++p) {
        if (!plan.chunk_cnt[p][k]) continue;
        CubeBatchArgs a{};
        a.u = src;
        a.dst = dst;
        a.f = f;
        a.groups = static_cast<const CubeGroupDev *>(plan.gdesc.p);
        a.chunks = static_cast<const CubeChunk *>(plan.chunks.p) + plan.chunk_off[p][k];
        a.list = k == 0 ? 1 : 0;
        a.omega = omega;
        hipError_t e = p < 3 ? launch_cube_small(a, plan.chunk_cnt[p][k], 16 << p, stream)
                             : launch_cube_big(a, plan.chunk_cnt[p][k], 16 << p, stream);
        if (e != hipSuccess) return hip_fail(e, "cube blocks (fused)");
    }
    return BS_OK;
}

bs_status enqueue_cube_sweeps(bs_patchset *ps, const CubePlan &plan, bs_scheme scheme, double omega, int nsweeps,
                              double *u, const double *f, double *work, hipStream_t stream)
{
    const PatchDesc *pdd = static_cast<const PatchDesc *>(ps->desc_d.p);
    bs_status st;
    // ghosts of linked faces are exchanged after every sweep (section 2)
    auto ghosts = [&](double *v) -> bs_status {
        if (!ghost_active(ps)) return BS_OK;
        hipError_t e = ghost_update(ps, v, false, stream);
        return e == hipSuccess ? BS_OK : hip_fail(e, "ghost update");
    };
    // extrapolated faces: their ghosts hold the negated adjacent values before
    // the first sweep (each is read only by its own cell's block)
    if (ghost_active(ps)) {
        hipError_t e = ghost_update(ps, u, true, stream);
        if (e != hipSuccess) return hip_fail(e, "ghost update");
    }
    if (scheme == BS_JACOBI) {
        hipError_t e = launch_ghost_copy(u, work, pdd, ps->npatch, stream);
        if (e != hipSuccess) return hip_fail(e, "ghost copy");
        for (int s = 0; s < nsweeps; ++s) {
            const double *src = (s & 1) ? work : u;
            double *dst = (s & 1) ? u : work;
            if ((st = small_pass(plan, 0, src, dst, f, omega, stream)) != BS_OK) return st;
            if ((st = small_pass(plan, 0, src, dst, f, omega, stream, true)) != BS_OK) return st;
            for (const CubeGroup &g : plan.groups)
                if (g.nb > plan.fused_max &&
                    (st = cube_pass(plan, g, true, 0, g.nblk, src, dst, f, omega, stream)) != BS_OK)
                    return st;
            if ((st = ghosts(dst)) != BS_OK) return st;
        }
        if (nsweeps & 1) {
            e = launch_interior_copy(work, u, pdd, ps->npatch, stream);
            if (e != hipSuccess) return hip_fail(e, "interior copy");
            if ((st = ghosts(u)) != BS_OK) return st;
        }
        return BS_OK;
    }
    // coloured (and chaotic) block GS: colour-0 blocks of every group, then colour 1, in place
    for (int s = 0; s < nsweeps; ++s) {
        for (int col = 0; col < 2; ++col) {
            if ((st = small_pass(plan, 1 + col, u, u, f, omega, stream)) != BS_OK) return st;
            if ((st = small_pass(plan, 1 + col, u, u, f, omega, stream, true)) != BS_OK) return st;
            for (const CubeGroup &g : plan.groups) {
                if (g.nb <= plan.fused_max) continue;
                const int lo = col ? g.ncol0 : 0, n = col ? g.nblk - g.ncol0 : g.ncol0;
                if ((st = cube_pass(plan, g, false, lo, n, u, u, f, omega, stream)) != BS_OK) return st;
            }
        }
        if ((st = ghosts(u)) != BS_OK) return st;
    }
    return BS_OK;
}

bs_status check_block(const bs_patchset *ps, int32_t bx, int32_t by, int32_t bz, const char *fn)
{
    if (!ps) return fail(BS_ERR_INVALID, "%s: null patch set", fn);
    if (bx < 1 || by < 1 || bz < 1) return fail(BS_ERR_INVALID, "%s: block edges must be >= 1", fn);
    if (int64_t(std::min(bx, ps->max_n[0])) * std::min(by, ps->max_n[1]) * std::min(bz, ps->max_n[2]) >
        kCubeMaxCells)
        return fail(BS_ERR_UNSUPPORTED, "%s: blocks of more than %d cells", fn, kCubeMaxCells);
    return BS_OK;
}

}  // namespace

bs_status cube_rebuild_all(bs_patchset *ps)
{
    // each plan is rebuilt aside and swapped in whole.  When a rebuild fails,
    // that size and every size not rebuilt yet are dropped (they hold inverses
    // of the old eps and must be prepared again); sizes rebuilt before it keep
    // their new plans
    for (auto it = ps->cube.begin(); it != ps->cube.end(); ++it) {
        std::unique_ptr<CubePlan> fresh(new CubePlan);
        bs_status st = build_plan(ps, std::get<0>(it->first), std::get<1>(it->first), std::get<2>(it->first), *fresh);
        if (st != BS_OK) {
            ps->cube.erase(it, ps->cube.end());
            return st;
        }
        it->second.swap(fresh);
    }
    return BS_OK;
}

}  // namespace bs

using namespace bs;

extern "C" {

bs_status bs_cube_prepare(bs_patchset *ps, int32_t bx, int32_t by, int32_t bz)
{
    bs_status st = check_block(ps, bx, by, bz, "bs_cube_prepare");
    if (st != BS_OK) return st;
    const auto key = std::make_tuple(int(bx), int(by), int(bz));
    if (ps->cube.count(key)) return BS_OK;
    hipError_t e = hipSetDevice(ps->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    std::unique_ptr<CubePlan> plan(new CubePlan);
    if ((st = build_plan(ps, bx, by, bz, *plan)) != BS_OK) return st;
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    ps->cube.emplace(key, std::move(plan));
    return BS_OK;
}

bs_status bs_cube_relax(bs_patchset *ps, int32_t bx, int32_t by, int32_t bz, bs_scheme scheme, double omega,
                        int32_t nsweeps, bs_precision prec, double *u, const double *f, double *work,
                        hipStream_t stream)
{
    bs_status st = check_block(ps, bx, by, bz, "bs_cube_relax");
    if (st != BS_OK) return st;
    if (scheme != BS_JACOBI && scheme != BS_CHAOTIC_GS && scheme != BS_COLORED_GS)
        return fail(BS_ERR_INVALID, "bs_cube_relax: unknown scheme");
    if (!(omega > 0.0 && omega < 2.0)) return fail(BS_ERR_INVALID, "bs_cube_relax: omega must be in (0, 2)");
    if (nsweeps < 0) return fail(BS_ERR_INVALID, "bs_cube_relax: nsweeps < 0");
    if (prec != BS_FP64 && prec != BS_MIXED_FP32 && prec != BS_MIXED_BF16)
        return fail(BS_ERR_INVALID, "bs_cube_relax: unknown precision");
    if (prec != BS_FP64) return fail(BS_ERR_UNSUPPORTED, "bs_cube_relax: cube blocks run in FP64 only");
    if (!u || !f) return fail(BS_ERR_INVALID, "bs_cube_relax: null u or f");
    if (scheme == BS_JACOBI && !work) return fail(BS_ERR_INVALID, "bs_cube_relax: Jacobi needs a work buffer");
    auto it = ps->cube.find(std::make_tuple(int(bx), int(by), int(bz)));
    if (it == ps->cube.end())
        return fail(BS_ERR_INVALID, "bs_cube_relax: block size %dx%dx%d not prepared (bs_cube_prepare)", bx, by, bz);
    if (nsweeps == 0) return BS_OK;
    const CubePlan &plan = *it->second;
    if (!ps->use_graphs || nsweeps < 2) return enqueue_cube_sweeps(ps, plan, scheme, omega, nsweeps, u, f, work, stream);

    // replay a captured graph of the whole sequence (captured on first use)
    int64_t obits;
    std::memcpy(&obits, &omega, sizeof obits);
    const std::vector<int64_t> key{2, bx, by, bz, scheme, obits, nsweeps, reinterpret_cast<int64_t>(u),
                                   reinterpret_cast<int64_t>(f), reinterpret_cast<int64_t>(work)};
    auto itr = ps->graphs.find(key);
    hipError_t e;
    if (itr == ps->graphs.end()) {
        if (ps->graphs.size() >= 64) clear_graphs(ps);
        if (!ps->capture_stream &&
            (e = hipStreamCreateWithFlags(&ps->capture_stream, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "capture stream");
        hipGraph_t graph = nullptr;
        if ((e = hipStreamBeginCapture(ps->capture_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(e, "hipStreamBeginCapture");
        st = enqueue_cube_sweeps(ps, plan, scheme, omega, nsweeps, u, f, work, ps->capture_stream);
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

// Largest cube block (cells, 64..256) on the fused kernels; larger blocks take
// the residual matrix and a separate product.  Drops the prepared sizes.
int bsi_set_cube_fused_max(bs_patchset *ps, int cells)
{
    if (!ps || cells < 64 || cells > 256) return BS_ERR_INVALID;
    ps->cube_fused_max = cells;
    clear_graphs(ps);
    ps->cube.clear();
    return BS_OK;
}

}  // extern "C"
