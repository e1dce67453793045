// Plane-block relaxation driver: tables, scratch and the four-product chain
// of fast diagonalisation for each plane orientation.
#include <algorithm>
#include <cmath>

#include "patchset.h"
#include "plane.h"
#include "relax.h"
#include "tables.h"

namespace bs {

namespace {

constexpr int kMaxPlaneEdge = 1024;

// Bases S_x, S_y, S_z of every patch and the inverse eigenvalue grid of every
// (patch, normal):  normal z: [q_y][p_x] = 1/(sigma_y,q + sigma_x,p + 2 eps_z);
// normal y: [q_z][p_x]; normal x: [q_z][q_y].
bs_status build_plane_tables(bs_patchset *ps)
{
    std::vector<double> tab;
    ps->basis_off.assign(3 * static_cast<size_t>(ps->npatch), -1);
    ps->lam_off.assign(3 * static_cast<size_t>(ps->npatch), -1);
    for (int p = 0; p < ps->npatch; ++p) {
        const int n[3] = {ps->dims[3 * p], ps->dims[3 * p + 1], ps->dims[3 * p + 2]};
        const double *e = &ps->eps[3 * static_cast<size_t>(p)];
        std::vector<long double> sg[3];
        for (int a = 0; a < 3; ++a) {
            ps->basis_off[3 * p + a] = static_cast<int64_t>(tab.size());
            const std::vector<double> S = sine_basis(n[a]);
            tab.insert(tab.end(), S.begin(), S.end());
            while (tab.size() % 4) tab.push_back(0.0);
            sg[a] = sine_eigenvalues(n[a], e[a]);
        }
        for (int c = 0; c < 3; ++c) {
            // rows (slow index) and columns (fast index) of the grid
            const int ar = c == 0 ? 2 : (c == 1 ? 2 : 1);
            const int ac = c == 0 ? 1 : 0;
            ps->lam_off[3 * p + c] = static_cast<int64_t>(tab.size());
            for (int q = 0; q < n[ar]; ++q)
                for (int r = 0; r < n[ac]; ++r)
                    tab.push_back(static_cast<double>(1.0L / (sg[ar][q] + sg[ac][r] + 2.0L * e[c])));
            while (tab.size() % 4) tab.push_back(0.0);
        }
    }
    bs_status st = upload(ps->plane_tab_d, tab.data(), tab.size() * sizeof(double), "plane tables");
    if (st != BS_OK) return st;
    if (!ps->plane_r_d.p) {
        if ((st = dev_alloc(ps->plane_r_d, static_cast<size_t>(ps->f_numel) * 8, "plane scratch")) != BS_OK) return st;
        if ((st = dev_alloc(ps->plane_t_d, static_cast<size_t>(ps->f_numel) * 8, "plane scratch")) != BS_OK) return st;
    }
    ps->plane_ready = true;
    return BS_OK;
}

GemmArgs gemm(const double *A, int64_t lda, int64_t sA, const double *B, int64_t ldb, int64_t sB, double *C,
              int64_t ldc, int64_t sC, int M, int N, int K, int batch)
{
    GemmArgs g{};
    g.A = A; g.lda = lda; g.sA = sA;
    g.B = B; g.ldb = ldb; g.sB = sB;
    g.C = C; g.ldc = ldc; g.sC = sC;
    g.M = M; g.N = N; g.K = K; g.batch = batch;
    g.ncolour = -1;
    return g;
}

// One pass of plane solves with normal c over the planes of `colour` (-1: all)
// of every patch: R = residual(src) must already be in plane_r; writes dst.
bs_status plane_chain(bs_patchset *ps, int c, int colour, const double *src, double *dst, double omega,
                      hipStream_t s)
{
    const double *tab = static_cast<const double *>(ps->plane_tab_d.p);
    double *Rall = static_cast<double *>(ps->plane_r_d.p);
    double *Tall = static_cast<double *>(ps->plane_t_d.p);
    for (int p = 0; p < ps->npatch; ++p) {
        const int nx = ps->dims[3 * p], ny = ps->dims[3 * p + 1], nz = ps->dims[3 * p + 2];
        const int64_t sx = nx + 2, sy = sx * (ny + 2), pl = static_cast<int64_t>(nx) * ny;
        const int64_t uo = ps->uoff[p];
        double *R = Rall + ps->foff[p];
        double *T = Tall + ps->foff[p];
        const double *Sx = tab + ps->basis_off[3 * p + 0];
        const double *Sy = tab + ps->basis_off[3 * p + 1];
        const double *Sz = tab + ps->basis_off[3 * p + 2];
        const double *lam = tab + ps->lam_off[3 * p + c];
        const int first = colour < 0 ? 0 : colour, step = colour < 0 ? 1 : 2;
        GemmArgs g1, g2, g3, g4;
        if (c == 2) {          // planes k: (ny x nx); x by right product, y by left product
            const int nb = (nz - first + step - 1) / step;
            if (nb <= 0) continue;
            const int64_t o = first * pl, sb = step * pl;
            g1 = gemm(R + o, nx, sb, Sx, nx, 0, T + o, nx, sb, ny, nx, nx, nb);
            g2 = gemm(Sy, ny, 0, T + o, nx, sb, R + o, nx, sb, ny, nx, ny, nb);
            g2.scale = lam; g2.sc_b = 0; g2.sc_m = nx; g2.sc_n = 1;
            g3 = gemm(Sy, ny, 0, R + o, nx, sb, T + o, nx, sb, ny, nx, ny, nb);
            g4 = gemm(T + o, nx, sb, Sx, nx, 0, nullptr, 0, 0, ny, nx, nx, nb);
            g4.u0 = uo + (first + 1) * sy + sx + 1; g4.u_b = step * sy; g4.u_m = sx; g4.u_n = 1;
        } else if (c == 1) {   // planes j: (nz x nx) with row stride nx*ny
            const int nb = (ny - first + step - 1) / step;
            if (nb <= 0) continue;
            const int64_t o = static_cast<int64_t>(first) * nx, sb = static_cast<int64_t>(step) * nx;
            g1 = gemm(R + o, pl, sb, Sx, nx, 0, T + o, pl, sb, nz, nx, nx, nb);
            g2 = gemm(Sz, nz, 0, T + o, pl, sb, R + o, pl, sb, nz, nx, nz, nb);
            g2.scale = lam; g2.sc_b = 0; g2.sc_m = nx; g2.sc_n = 1;
            g3 = gemm(Sz, nz, 0, R + o, pl, sb, T + o, pl, sb, nz, nx, nz, nb);
            g4 = gemm(T + o, pl, sb, Sx, nx, 0, nullptr, 0, 0, nz, nx, nx, nb);
            g4.u0 = uo + sy + (first + 1) * sx + 1; g4.u_b = step * sx; g4.u_m = sy; g4.u_n = 1;
        } else {               // planes i: z by left product per j, y by left product per k
            g1 = gemm(Sz, nz, 0, R, pl, nx, T, pl, nx, nz, nx, nz, ny);
            g2 = gemm(Sy, ny, 0, T, nx, pl, R, nx, pl, ny, nx, ny, nz);
            g2.scale = lam; g2.sc_b = ny; g2.sc_m = 1; g2.sc_n = 0;
            g3 = gemm(Sy, ny, 0, R, nx, pl, T, nx, pl, ny, nx, ny, nz);
            g4 = gemm(Sz, nz, 0, T, pl, nx, nullptr, 0, 0, nz, nx, nz, ny);
            g4.u0 = uo + sy + sx + 1; g4.u_b = sx; g4.u_m = sy; g4.u_n = 1;
            g4.ncolour = colour; g4.colour_shift = 0;
        }
        g4.usrc = src;
        g4.udst = dst;
        g4.omega = omega;
        hipError_t e;
        if ((e = launch_gemm_f64(g1, kEpiStore, s)) != hipSuccess) return hip_fail(e, "plane transform 1");
        if ((e = launch_gemm_f64(g2, kEpiScale, s)) != hipSuccess) return hip_fail(e, "plane transform 2");
        if ((e = launch_gemm_f64(g3, kEpiStore, s)) != hipSuccess) return hip_fail(e, "plane transform 3");
        if ((e = launch_gemm_f64(g4, kEpiUpdate, s)) != hipSuccess) return hip_fail(e, "plane transform 4");
    }
    return BS_OK;
}

bs_status residual_into_scratch(bs_patchset *ps, const double *u, const double *f, hipStream_t s)
{
    ResidArgs a{};
    a.u = u;
    a.f = f;
    a.r = static_cast<double *>(ps->plane_r_d.p);
    a.partial = nullptr;
    a.pd = static_cast<const PatchDesc *>(ps->desc_d.p);
    a.block_patch = static_cast<const int32_t *>(ps->rblock_patch_d.p);
    a.block_first = static_cast<const int32_t *>(ps->rblock_first_d.p);
    hipError_t e = launch_residual(a, ps->nrblocks, s);
    if (e != hipSuccess) return hip_fail(e, "plane residual");
    return BS_OK;
}

}  // namespace

}  // namespace bs

using namespace bs;

extern "C" bs_status bs_plane_relax(bs_patchset *ps, int32_t normal_axis, bs_scheme scheme, double omega,
                                    int32_t nsweeps, bs_precision prec, int32_t refine, double *u,
                                    const double *f, double *work, hipStream_t stream)
{
    if (normal_axis < 0 || normal_axis > 2) return fail(BS_ERR_INVALID, "bs_plane_relax: axis must be 0, 1 or 2");
    if (scheme != BS_JACOBI && scheme != BS_CHAOTIC_GS && scheme != BS_COLORED_GS)
        return fail(BS_ERR_INVALID, "bs_plane_relax: unknown scheme");
    if (!(omega > 0.0 && omega < 2.0)) return fail(BS_ERR_INVALID, "bs_plane_relax: omega must be in (0, 2)");
    if (nsweeps < 0) return fail(BS_ERR_INVALID, "bs_plane_relax: nsweeps < 0");
    if (refine < 0) return fail(BS_ERR_INVALID, "bs_plane_relax: refine < 0");
    if (prec != BS_FP64 && prec != BS_MIXED_FP32 && prec != BS_MIXED_BF16)
        return fail(BS_ERR_INVALID, "bs_plane_relax: unknown precision");
    if (!ps || !u || !f) return fail(BS_ERR_INVALID, "bs_plane_relax: null patch set, u or f");
    if (scheme == BS_JACOBI && !work) return fail(BS_ERR_INVALID, "bs_plane_relax: Jacobi needs a work buffer");
    for (int a = 0; a < 3; ++a)
        if (a != normal_axis && ps->max_n[a] > kMaxPlaneEdge)
            return fail(BS_ERR_UNSUPPORTED, "bs_plane_relax: an in-plane edge exceeds %d", kMaxPlaneEdge);
    if (prec != BS_FP64) return fail(BS_ERR_UNSUPPORTED, "bs_plane_relax: mixed precision is not built yet");
    if (nsweeps == 0) return BS_OK;
    bs_status st;
    if (!ps->plane_ready && (st = build_plane_tables(ps)) != BS_OK) return st;
    const PatchDesc *pdd = static_cast<const PatchDesc *>(ps->desc_d.p);
    if (scheme == BS_JACOBI) {
        hipError_t e = launch_ghost_copy(u, work, pdd, ps->npatch, stream);
        if (e != hipSuccess) return hip_fail(e, "ghost copy");
        for (int sw = 0; sw < nsweeps; ++sw) {
            const double *src = (sw & 1) ? work : u;
            double *dst = (sw & 1) ? u : work;
            if ((st = residual_into_scratch(ps, src, f, stream)) != BS_OK) return st;
            if ((st = plane_chain(ps, normal_axis, -1, src, dst, omega, stream)) != BS_OK) return st;
        }
        if (nsweeps & 1) {
            e = launch_interior_copy(work, u, pdd, ps->npatch, stream);
            if (e != hipSuccess) return hip_fail(e, "interior copy");
        }
        return BS_OK;
    }
    // Gauss-Seidel: planes of colour 0, then colour 1 (the chaotic scheme runs
    // the same colour-major order), in place
    for (int sw = 0; sw < nsweeps; ++sw)
        for (int colour = 0; colour < 2; ++colour) {
            if ((st = residual_into_scratch(ps, u, f, stream)) != BS_OK) return st;
            if ((st = plane_chain(ps, normal_axis, colour, u, u, omega, stream)) != BS_OK) return st;
        }
    return BS_OK;
}

// Host-side test hook (not part of the public header): one batched product
// C_b = A_b B_b with the plane kernel's store epilogue (epi 0) or scale
// epilogue (epi 1, scale indexed [b*sc_b + m*sc_m + n*sc_n]).  Device pointers.
extern "C" int bsi_gemm_f64(const double *A, int64_t lda, int64_t sA, const double *B, int64_t ldb, int64_t sB,
                            double *C, int64_t ldc, int64_t sC, int M, int N, int K, int batch, int epi,
                            const double *scale, int64_t sc_b, int64_t sc_m, int64_t sc_n, hipStream_t s)
{
    if (epi != bs::kEpiStore && epi != bs::kEpiScale) return BS_ERR_INVALID;
    bs::GemmArgs g = bs::gemm(A, lda, sA, B, ldb, sB, C, ldc, sC, M, N, K, batch);
    g.scale = scale;
    g.sc_b = sc_b;
    g.sc_m = sc_m;
    g.sc_n = sc_n;
    return bs::launch_gemm_f64(g, epi, s) == hipSuccess ? BS_OK : BS_ERR_HIP;
}
