// Plane-block relaxation driver: tables, scratch and the four-product chain
// of fast diagonalisation for each plane orientation, in FP64 or mixed
// precision (FP32 / BF16 products, FP64 residual, defect and update).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "patchset.h"
#include "plane.h"
#include "relax.h"
#include "tables.h"

namespace bs {

namespace {

constexpr int kMaxPlaneEdge = 1024;

// FP64 -> BF16 bit pattern, rounded to nearest even through FP32 (finite
// inputs; the tables hold O(1) values).
uint16_t bf16_bits(double v)
{
    const float f = static_cast<float>(v);
    uint32_t u;
    std::memcpy(&u, &f, sizeof u);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return static_cast<uint16_t>(u >> 16);
}

// Bases of every patch and axis and the inverse eigenvalue grid of every
// (patch, normal):  normal z: [q_y][p_x] = 1/(sigma_y,q + sigma_x,p + 2 eps_z);
// normal y: [q_z][p_x]; normal x: [q_z][q_y].  An axis with extrapolated faces
// takes the eigenbasis of its raised line block (stored as V^T for the forward
// and V for the inverse transforms), and a plane next to an extrapolated face
// normal to the planes adds eps_c per such face to its grid.  FP32 copies
// share the offsets.
bs_status build_plane_tables(bs_patchset *ps)
{
    std::vector<double> tab;
    const size_t n3 = 3 * static_cast<size_t>(ps->npatch);
    ps->basis_off.assign(n3, -1);
    ps->basis_inv_off.assign(n3, -1);
    ps->basis_kind.assign(n3, 0);
    ps->lam_off.assign(n3, -1);
    ps->lam_lo_off.assign(n3, -1);
    ps->lam_hi_off.assign(n3, -1);
    for (int p = 0; p < ps->npatch; ++p) {
        const int n[3] = {ps->dims[3 * p], ps->dims[3 * p + 1], ps->dims[3 * p + 2]};
        const double *e = &ps->eps[3 * static_cast<size_t>(p)];
        const int bcm = ps->bc[p];
        std::vector<long double> sg[3];
        for (int a = 0; a < 3; ++a) {
            const int lo = (bcm >> (2 * a)) & 1, hi = (bcm >> (2 * a + 1)) & 1;
            const std::vector<double> V = bc_sine_basis(n[a], lo, hi);
            ps->basis_kind[3 * p + a] = static_cast<int8_t>(lo && hi ? 1 : (lo || hi ? 2 : 0));
            ps->basis_inv_off[3 * p + a] = static_cast<int64_t>(tab.size());
            tab.insert(tab.end(), V.begin(), V.end());
            while (tab.size() % 8) tab.push_back(0.0);   // 16-byte aligned BF16 copies
            if (lo || hi) {
                ps->basis_off[3 * p + a] = static_cast<int64_t>(tab.size());
                for (int i = 0; i < n[a]; ++i)
                    for (int k = 0; k < n[a]; ++k) tab.push_back(V[static_cast<size_t>(k) * n[a] + i]);
                while (tab.size() % 8) tab.push_back(0.0);
            } else {
                ps->basis_off[3 * p + a] = ps->basis_inv_off[3 * p + a];   // symmetric
            }
            sg[a] = bc_sine_eigenvalues(n[a], e[a], lo, hi);
        }
        for (int c = 0; c < 3; ++c) {
            const int ar = c == 0 ? 2 : (c == 1 ? 2 : 1);   // grid rows (slow index)
            const int ac = c == 0 ? 1 : 0;                   // grid columns
            const int lo = (bcm >> (2 * c)) & 1, hi = (bcm >> (2 * c + 1)) & 1;
            auto grid = [&](long double shift) {
                const int64_t off = static_cast<int64_t>(tab.size());
                for (int q = 0; q < n[ar]; ++q)
                    for (int r = 0; r < n[ac]; ++r)
                        tab.push_back(static_cast<double>(1.0L / (sg[ar][q] + sg[ac][r] + 2.0L * e[c] + shift)));
                while (tab.size() % 8) tab.push_back(0.0);
                return off;
            };
            ps->lam_off[3 * p + c] = grid(0.0L);
            // one plane along the normal takes both shifts
            if (n[c] == 1 && (lo || hi)) {
                ps->lam_lo_off[3 * p + c] = grid(static_cast<long double>(e[c]) * (lo + hi));
            } else {
                if (lo) ps->lam_lo_off[3 * p + c] = grid(e[c]);
                if (hi) ps->lam_hi_off[3 * p + c] = grid(e[c]);
            }
        }
    }
    bs_status st = upload(ps->plane_tab_d, tab.data(), tab.size() * sizeof(double), "plane tables");
    if (st != BS_OK) return st;
    std::vector<float> tab32(tab.begin(), tab.end());
    if ((st = upload(ps->plane_tab32_d, tab32.data(), tab32.size() * sizeof(float), "plane tables")) != BS_OK) return st;
    // BF16 copy (round to nearest even from FP64) for the BF16 products
    std::vector<uint16_t> tab16(tab.size());
    for (size_t t = 0; t < tab.size(); ++t) tab16[t] = bf16_bits(tab[t]);
    if ((st = upload(ps->plane_tab16_d, tab16.data(), tab16.size() * sizeof(uint16_t), "plane tables")) != BS_OK)
        return st;
    if (!ps->plane_r_d.p) {
        if ((st = dev_alloc(ps->plane_r_d, static_cast<size_t>(ps->f_numel) * 8, "plane scratch")) != BS_OK) return st;
        if ((st = dev_alloc(ps->plane_t_d, static_cast<size_t>(ps->f_numel) * 8, "plane scratch")) != BS_OK) return st;
    }
    ps->plane_ready = true;
    ++ps->gen;
    return BS_OK;
}

bs_status ensure_mixed_scratch(bs_patchset *ps)
{
    bs_status st = BS_OK;
    if (!ps->plane_f1_d.p) {
        if ((st = dev_alloc(ps->plane_f1_d, static_cast<size_t>(ps->f_numel) * 4, "plane scratch")) != BS_OK) return st;
        if ((st = dev_alloc(ps->plane_f2_d, static_cast<size_t>(ps->f_numel) * 4, "plane scratch")) != BS_OK) return st;
    }
    return st;
}

// Geometry of one product of the chain: C_b = A_b B_b, with A, B, C given as
// (buffer id, offset, leading dimension, batch stride).  Buffer ids:
// kX = input field, kY = the other scratch field, bases/grid from the tables.
enum Buf { kIn = 0, kOut = 1, kSx = 2, kSy = 3, kSz = 4, kLam = 5 };
struct Operand {
    int buf;
    int64_t off, ld, sb;
};
struct Product {
    Operand A, B, C;
    int M, N, K, batch;
    int64_t sc_b = 0, sc_m = 0, sc_n = 0;   // grid strides (second product)
};
struct Chain {
    Product g[4];
    int64_t u0, u_b, u_m, u_n;   // update mapping of the last product
    int filter_n = 0;            // last product filters columns by colour (normal x)
    int colour_shift = 0;        // column n of the last product is plane n + colour_shift
    bool empty = false;
};

// The four products M_P^{-1} R = S_b[(S_b R S_a)./Lambda]S_a for every plane
// of one patch with normal c and the given colour (-1: all).  Fields live in
// the patch's f layout; the chain alternates between the input field (kIn)
// and the scratch field (kOut), ending with the update.  Normals y and z:
// by default the right (x) products come first and last; lr: the left ones,
// so that the last product -- whose even / odd halves write every other row
// or column of u -- writes whole x-rows (the transforms along the two axes
// commute; the FP32 chain takes this order).
Chain plane_chain_geometry(const bs_patchset *ps, int p, int c, int colour, int k0 = 0, int k1 = -1,
                           bool lr = false)
{
    Chain ch;
    const int nx = ps->dims[3 * p], ny = ps->dims[3 * p + 1], nz = ps->dims[3 * p + 2];
    const int64_t sx = nx + 2, sy = sx * (ny + 2), pl = static_cast<int64_t>(nx) * ny;
    const int64_t uo = ps->uoff[p];
    // planes [k0, k1) along the normal (all by default)
    if (k1 < 0) k1 = ps->dims[3 * p + c];
    const int first = colour < 0 ? k0 : k0 + ((colour - k0) & 1), step = colour < 0 ? 1 : 2;
    if (first >= k1) {
        ch.empty = true;
        return ch;
    }
    auto prod = [](Operand A, Operand B, Operand C, int M, int N, int K, int batch) {
        Product q;
        q.A = A; q.B = B; q.C = C; q.M = M; q.N = N; q.K = K; q.batch = batch;
        return q;
    };
    if (c == 2) {   // planes k: (ny x nx); x by right product, y by left product
        const int nb = (k1 - first + step - 1) / step;
        if (nb <= 0) { ch.empty = true; return ch; }
        const int64_t o = first * pl, sb = step * pl;
        if (lr) {
            ch.g[0] = prod({kSy, 0, ny, 0}, {kIn, o, nx, sb}, {kOut, o, nx, sb}, ny, nx, ny, nb);
            ch.g[1] = prod({kOut, o, nx, sb}, {kSx, 0, nx, 0}, {kIn, o, nx, sb}, ny, nx, nx, nb);
            ch.g[2] = prod({kIn, o, nx, sb}, {kSx, 0, nx, 0}, {kOut, o, nx, sb}, ny, nx, nx, nb);
            ch.g[3] = prod({kSy, 0, ny, 0}, {kOut, o, nx, sb}, {kIn, o, nx, sb}, ny, nx, ny, nb);
        } else {
            ch.g[0] = prod({kIn, o, nx, sb}, {kSx, 0, nx, 0}, {kOut, o, nx, sb}, ny, nx, nx, nb);
            ch.g[1] = prod({kSy, 0, ny, 0}, {kOut, o, nx, sb}, {kIn, o, nx, sb}, ny, nx, ny, nb);
            ch.g[2] = prod({kSy, 0, ny, 0}, {kIn, o, nx, sb}, {kOut, o, nx, sb}, ny, nx, ny, nb);
            ch.g[3] = prod({kOut, o, nx, sb}, {kSx, 0, nx, 0}, {kIn, o, nx, sb}, ny, nx, nx, nb);
        }
        ch.g[1].sc_m = nx; ch.g[1].sc_n = 1;
        ch.u0 = uo + (first + 1) * sy + sx + 1; ch.u_b = step * sy; ch.u_m = sx; ch.u_n = 1;
    } else if (c == 1) {   // planes j: (nz x nx) with row stride nx*ny
        const int nb = (k1 - first + step - 1) / step;
        if (nb <= 0) { ch.empty = true; return ch; }
        const int64_t o = static_cast<int64_t>(first) * nx, sb = static_cast<int64_t>(step) * nx;
        if (lr) {
            ch.g[0] = prod({kSz, 0, nz, 0}, {kIn, o, pl, sb}, {kOut, o, pl, sb}, nz, nx, nz, nb);
            ch.g[1] = prod({kOut, o, pl, sb}, {kSx, 0, nx, 0}, {kIn, o, pl, sb}, nz, nx, nx, nb);
            ch.g[2] = prod({kIn, o, pl, sb}, {kSx, 0, nx, 0}, {kOut, o, pl, sb}, nz, nx, nx, nb);
            ch.g[3] = prod({kSz, 0, nz, 0}, {kOut, o, pl, sb}, {kIn, o, pl, sb}, nz, nx, nz, nb);
        } else {
            ch.g[0] = prod({kIn, o, pl, sb}, {kSx, 0, nx, 0}, {kOut, o, pl, sb}, nz, nx, nx, nb);
            ch.g[1] = prod({kSz, 0, nz, 0}, {kOut, o, pl, sb}, {kIn, o, pl, sb}, nz, nx, nz, nb);
            ch.g[2] = prod({kSz, 0, nz, 0}, {kIn, o, pl, sb}, {kOut, o, pl, sb}, nz, nx, nz, nb);
            ch.g[3] = prod({kOut, o, pl, sb}, {kSx, 0, nx, 0}, {kIn, o, pl, sb}, nz, nx, nx, nb);
        }
        ch.g[1].sc_m = nx; ch.g[1].sc_n = 1;
        ch.u0 = uo + sy + (first + 1) * sx + 1; ch.u_b = step * sx; ch.u_m = sy; ch.u_n = 1;
    } else {   // planes i (columns [k0, k1)): z by left product per j, y by left product per k;
               // colour filters columns
        const int w = k1 - k0;
        ch.g[0] = prod({kSz, 0, nz, 0}, {kIn, k0, pl, nx}, {kOut, k0, pl, nx}, nz, w, nz, ny);
        ch.g[1] = prod({kSy, 0, ny, 0}, {kOut, k0, nx, pl}, {kIn, k0, nx, pl}, ny, w, ny, nz);
        ch.g[1].sc_b = ny; ch.g[1].sc_m = 1; ch.g[1].sc_n = 0;
        ch.g[2] = prod({kSy, 0, ny, 0}, {kIn, k0, nx, pl}, {kOut, k0, nx, pl}, ny, w, ny, nz);
        ch.g[3] = prod({kSz, 0, nz, 0}, {kOut, k0, pl, nx}, {kIn, k0, pl, nx}, nz, w, nz, ny);
        ch.u0 = uo + sy + sx + 1 + k0; ch.u_b = sx; ch.u_m = sy; ch.u_n = 1;
        ch.filter_n = 1;
        ch.colour_shift = k0;
    }
    return ch;
}

// inv: the inverse transforms (the last two products) read V, the forward ones
// V^T (the same entries for the symmetric DST-I basis).
template <typename T>
const T *operand_ptr(const bs_patchset *ps, int p, int c, const Operand &o, const T *in, const T *out, const T *tab,
                     bool inv = false)
{
    const std::vector<int64_t> &bo = inv ? ps->basis_inv_off : ps->basis_off;
    switch (o.buf) {
    case kIn: return in + o.off;
    case kOut: return out + o.off;
    case kSx: return tab + bo[3 * p + 0];
    case kSy: return tab + bo[3 * p + 1];
    case kSz: return tab + bo[3 * p + 2];
    default: return tab + ps->lam_off[3 * p + c];
    }
}

// FP64 chain for one patch: R (residual, f layout) is consumed as scratch.
// Every product has a sine basis on one side.  The DST-I basis obeys
// S[n-1-i][j] = (-1)^j S[i][j] and is symmetric, so each product splits into
// its even and its odd output rows (left products) or columns (right
// products), each a product over half the contraction with the field folded
// about its middle (x[k] + x[n-1-k] for even, x[k] - x[n-1-k] for odd
// outputs): half the flops.  The basis of an axis with both faces
// extrapolated keeps the mirror property in its rows only, so only the
// forward transforms fold; an axis with one extrapolated face has no mirror
// property and its products run unfolded.  Planes next to an extrapolated
// face normal to them are solved by chains of their own (their eigenvalue
// grid is shifted).
bs_status chain_range(bs_patchset *ps, int p, int c, int colour, int k0, int k1, int64_t lam, const double *src,
                      double *dst, double omega, hipStream_t s)
{
    const Chain ch = plane_chain_geometry(ps, p, c, colour, k0, k1);
    if (ch.empty) return BS_OK;
    const double *tab = static_cast<const double *>(ps->plane_tab_d.p);
    double *R = static_cast<double *>(ps->plane_r_d.p) + ps->foff[p];
    double *T = static_cast<double *>(ps->plane_t_d.p) + ps->foff[p];
    for (int q = 0; q < 4; ++q) {
        const Product &pr = ch.g[q];
        const bool right = pr.B.buf == kSx || pr.B.buf == kSy || pr.B.buf == kSz;   // C = A S, else C = S B
        const int baxis = (right ? pr.B.buf : pr.A.buf) - kSx;
        const int kind = ps->basis_kind[3 * p + baxis];
        const bool inv = q >= 2;
        const bool fold = kind == 0 || (kind == 1 && !inv);
        for (int par = 0; par < (fold ? 2 : 1); ++par) {
            GemmArgs g{};
            g.A = operand_ptr<double>(ps, p, c, pr.A, R, T, tab, inv);
            g.lda = pr.A.ld; g.sA = pr.A.sb;
            g.B = operand_ptr<double>(ps, p, c, pr.B, R, T, tab, inv);
            g.ldb = pr.B.ld; g.sB = pr.B.sb;
            g.C = const_cast<double *>(operand_ptr<double>(ps, p, c, pr.C, R, T, tab, inv));
            g.ldc = pr.C.ld; g.sC = pr.C.sb;
            g.M = pr.M; g.N = pr.N; g.batch = pr.batch;
            g.Kfull = pr.K;
            g.K = pr.K;
            g.row_s = 1; g.col_s = 1;
            if (right) g.b_trans = 1;   // B(k, n) at n*ldb + k: V^T / V stored row-major
            if (fold) {
                g.K = par == 0 ? (pr.K + 1) / 2 : pr.K / 2;
                g.fsign = par == 0 ? 1 : -1;
                if (right) {   // columns n = 2n' + par; B' = rows 2n' + par of the stored basis
                    g.fold = 1;
                    g.B += static_cast<int64_t>(par) * pr.B.ld;
                    g.ldb = 2 * pr.B.ld;
                    g.N = (pr.N + 1 - par) / 2;
                    g.col_s = 2; g.col_o = par;
                } else {       // rows m = 2m' + par; A' = rows 2m' + par of the basis
                    g.fold = 2;
                    g.A += static_cast<int64_t>(par) * pr.A.ld;
                    g.lda = 2 * pr.A.ld;
                    g.M = (pr.M + 1 - par) / 2;
                    g.row_s = 2; g.row_o = par;
                }
            }
            if (g.K <= 0 || g.M <= 0 || g.N <= 0) continue;
            g.ncolour = -1;
            int epi = kEpiStore;
            if (q == 1) {
                epi = kEpiScale;
                g.scale = tab + lam;
                g.sc_b = pr.sc_b; g.sc_m = pr.sc_m; g.sc_n = pr.sc_n;
            } else if (q == 3) {
                epi = kEpiUpdate;
                g.usrc = src; g.udst = dst; g.omega = omega;
                g.u0 = ch.u0; g.u_b = ch.u_b; g.u_m = ch.u_m; g.u_n = ch.u_n;
                if (ch.filter_n) { g.ncolour = colour; g.colour_shift = ch.colour_shift; }
            }
            hipError_t e = launch_gemm_f64(g, epi, s);
            if (e != hipSuccess) return hip_fail(e, "plane transform");
        }
    }
    return BS_OK;
}

bs_status chain_f64(bs_patchset *ps, int p, int c, int colour, const double *src, double *dst, double omega,
                    hipStream_t s)
{
    const int nc = ps->dims[3 * p + c];
    const int64_t lo = ps->lam_lo_off[3 * p + c], hi = ps->lam_hi_off[3 * p + c];
    if (lo < 0 && hi < 0) return chain_range(ps, p, c, colour, 0, nc, ps->lam_off[3 * p + c], src, dst, omega, s);
    if (nc == 1) return chain_range(ps, p, c, colour, 0, 1, lo, src, dst, omega, s);
    int k0 = 0, k1 = nc;
    bs_status st;
    if (lo >= 0) {
        if ((st = chain_range(ps, p, c, colour, 0, 1, lo, src, dst, omega, s)) != BS_OK) return st;
        k0 = 1;
    }
    if (hi >= 0) {
        if ((st = chain_range(ps, p, c, colour, nc - 1, nc, hi, src, dst, omega, s)) != BS_OK) return st;
        k1 = nc - 1;
    }
    if (k1 > k0) return chain_range(ps, p, c, colour, k0, k1, ps->lam_off[3 * p + c], src, dst, omega, s);
    return BS_OK;
}

// Low-precision chain M~^{-1} E for one patch: E (float, f layout) in F1,
// scratch F2; the last product either updates u (final) or stores / adds
// into D (FP64).  The mixed forms run on DST-I bases only (no extrapolated
// faces), so every product splits into its even and odd halves as the FP64
// chain's do (half the flops each; the field operand folded about its
// middle).
bs_status chain_lowp(bs_patchset *ps, int p, int c, int colour, int prec, int last_epi, int accumulate,
                     const double *src, double *dst, double omega, hipStream_t s)
{
    const Chain ch = plane_chain_geometry(ps, p, c, colour, 0, -1, ps->plane_lr);
    if (ch.empty) return BS_OK;
    const float *tab = static_cast<const float *>(ps->plane_tab32_d.p);
    float *F1 = static_cast<float *>(ps->plane_f1_d.p) + ps->foff[p];
    float *F2 = static_cast<float *>(ps->plane_f2_d.p) + ps->foff[p];
    double *D = static_cast<double *>(ps->plane_t_d.p) + ps->foff[p];
    for (int q = 0; q < 4; ++q)
    for (int par = 0; par < 2; ++par) {
        const Product &pr = ch.g[q];
        const bool right = pr.B.buf == kSx || pr.B.buf == kSy || pr.B.buf == kSz;   // C = A S, else C = S B
        GemmMixedArgs g{};
        g.A = operand_ptr<float>(ps, p, c, pr.A, F1, F2, tab);
        g.lda = pr.A.ld; g.sA = pr.A.sb;
        g.B = operand_ptr<float>(ps, p, c, pr.B, F1, F2, tab);
        g.ldb = pr.B.ld; g.sB = pr.B.sb;
        g.C = const_cast<float *>(operand_ptr<float>(ps, p, c, pr.C, F1, F2, tab));
        g.ldc = pr.C.ld; g.sC = pr.C.sb;
        g.M = pr.M; g.N = pr.N; g.batch = pr.batch;
        g.Kfull = pr.K;
        g.K = par == 0 ? (pr.K + 1) / 2 : pr.K / 2;
        g.fsign = par == 0 ? 1 : -1;
        g.row_s = 1; g.col_s = 1;
        if (right) {   // columns n = 2n' + par; B' = rows 2n' + par of the (symmetric) basis, as [n][k]
            g.fold = 1;
            g.b_trans = 1;
            g.B += static_cast<int64_t>(par) * pr.B.ld;
            g.ldb = 2 * pr.B.ld;
            g.N = (pr.N + 1 - par) / 2;
            g.col_s = 2; g.col_o = par;
        } else {       // rows m = 2m' + par; A' = rows 2m' + par of the basis
            g.fold = 2;
            g.A += static_cast<int64_t>(par) * pr.A.ld;
            g.lda = 2 * pr.A.ld;
            g.M = (pr.M + 1 - par) / 2;
            g.row_s = 2; g.row_o = par;
        }
        if (g.K <= 0 || g.M <= 0 || g.N <= 0) continue;
        g.ncolour = -1;
        g.dlayout = ps->mixed_dlayout;
        int epi = kEpiStore;
        if (q == 1) {
            epi = kEpiScale;
            g.scale = tab + ps->lam_off[3 * p + c];
            g.sc_b = pr.sc_b; g.sc_m = pr.sc_m; g.sc_n = pr.sc_n;
        } else if (q == 3) {
            epi = last_epi;
            if (epi == kEpiUpdate || epi == kEpiUpdateAcc) {
                g.usrc = src; g.udst = dst; g.omega = omega;
                g.u0 = ch.u0; g.u_b = ch.u_b; g.u_m = ch.u_m; g.u_n = ch.u_n;
                if (ch.filter_n) { g.ncolour = colour; g.colour_shift = ch.colour_shift; }
            }
            if (epi == kEpiD64 || epi == kEpiUpdateAcc) {
                // D shares the f-layout indexing of the chain's final field (kIn = F1)
                g.D = D + (g.C - F1);
                g.accumulate = accumulate;
            }
        }
        hipError_t e = launch_gemm_mixed(g, prec, epi, s);
        if (e != hipSuccess) return hip_fail(e, "plane transform (mixed)");
    }
    return BS_OK;
}

// BF16 chain M~^{-1} E: E (BF16, f layout) in F1, scratch F2 (both BF16);
// the bases are symmetric, so a basis B operand is passed as [n][k].
bs_status chain_bf16(bs_patchset *ps, int p, int c, int colour, int last_epi, int accumulate, const double *src,
                     double *dst, double omega, hipStream_t s)
{
    const Chain ch = plane_chain_geometry(ps, p, c, colour);
    if (ch.empty) return BS_OK;
    const uint16_t *tab = static_cast<const uint16_t *>(ps->plane_tab16_d.p);
    const float *tab32 = static_cast<const float *>(ps->plane_tab32_d.p);
    uint16_t *F1 = static_cast<uint16_t *>(ps->plane_f1_d.p) + ps->foff[p];
    uint16_t *F2 = static_cast<uint16_t *>(ps->plane_f2_d.p) + ps->foff[p];
    float *D = static_cast<float *>(ps->plane_t_d.p) + ps->foff[p];   // FP32 correction
    // Planes with x in-plane (normals y and z): the first two products store
    // their result transposed in a compact per-plane layout (plane b at
    // b*M*N, element (m, n) at n*M + m), so the second and third products
    // read that field k-contiguous (no transposition through LDS).
    const bool tr = c != 0;
    const int64_t MN = static_cast<int64_t>(ch.g[0].M) * ch.g[0].N;
    for (int q = 0; q < 4; ++q) {
        const Product &pr = ch.g[q];
        GemmBf16Args g{};
        g.A = operand_ptr<uint16_t>(ps, p, c, pr.A, F1, F2, tab);
        g.lda = pr.A.ld; g.sA = pr.A.sb;
        g.B = operand_ptr<uint16_t>(ps, p, c, pr.B, F1, F2, tab);
        g.ldb = pr.B.ld; g.sB = pr.B.sb;
        int b_trans = (pr.B.buf == kSx || pr.B.buf == kSy || pr.B.buf == kSz) ? 1 : 0;
        g.C = const_cast<uint16_t *>(operand_ptr<uint16_t>(ps, p, c, pr.C, F1, F2, tab));
        g.ldc = pr.C.ld; g.sC = pr.C.sb;
        if (tr && (q == 1 || q == 2)) {   // B: the previous product's compact C^T, [n][k]
            g.B = pr.B.buf == kIn ? F1 : F2;
            g.ldb = pr.M; g.sB = MN;
            b_trans = 1;
        }
        if (tr && (q == 0 || q == 1)) {   // C^T into the compact layout
            g.C = pr.C.buf == kIn ? F1 : F2;
            g.ldc = pr.M; g.sC = MN;
            g.c_trans = 1;
        }
        g.M = pr.M; g.N = pr.N; g.K = pr.K; g.batch = pr.batch;
        g.ncolour = -1;
        int epi = kEpiStore;
        if (q == 1) {
            epi = kEpiScale;
            g.scale = tab32 + ps->lam_off[3 * p + c];
            g.sc_b = pr.sc_b; g.sc_m = pr.sc_m; g.sc_n = pr.sc_n;
        } else if (q == 3) {
            epi = last_epi;
            if (epi == kEpiUpdate || epi == kEpiUpdateAcc) {
                g.usrc = src; g.udst = dst; g.omega = omega;
                g.u0 = ch.u0; g.u_b = ch.u_b; g.u_m = ch.u_m; g.u_n = ch.u_n;
                if (ch.filter_n) { g.ncolour = colour; g.colour_shift = ch.colour_shift; }
            }
            if (epi == kEpiD64 || epi == kEpiUpdateAcc) {
                g.D = D + (g.C - F1);
                g.accumulate = accumulate;
            }
        }
        hipError_t e = launch_gemm_bf16(g, b_trans, epi, s);
        if (e != hipSuccess) return hip_fail(e, "plane transform (BF16)");
    }
    return BS_OK;
}

// One plane pass (normal c, colour or -1) on every patch.  R = residual of
// src must be in plane_r.  Mixed: D_0 = M~^{-1} R, refine defect corrections,
// then dst = src + omega D.
bs_status plane_pass(bs_patchset *ps, int c, int colour, int prec, int refine, const double *src, double *dst,
                     double omega, hipStream_t s)
{
    for (int p = 0; p < ps->npatch; ++p) {
        if (prec == BS_FP64) {
            bs_status st = chain_f64(ps, p, c, colour, src, dst, omega, s);
            if (st != BS_OK) return st;
            continue;
        }
        const int nx = ps->dims[3 * p], ny = ps->dims[3 * p + 1], nz = ps->dims[3 * p + 2];
        const double *R = static_cast<const double *>(ps->plane_r_d.p) + ps->foff[p];
        double *D = static_cast<double *>(ps->plane_t_d.p) + ps->foff[p];
        float *F1 = static_cast<float *>(ps->plane_f1_d.p) + ps->foff[p];
        // the BF16 chain keeps R and D in FP32 (their rounding, 2^-24
        // relative, is far below the BF16 solve's error after two defect steps)
        const float *R32 = static_cast<const float *>(ps->plane_r_d.p) + ps->foff[p];
        const float *D32 = static_cast<const float *>(ps->plane_t_d.p) + ps->foff[p];
        const double *eps = &ps->eps[3 * static_cast<size_t>(p)];
        const bool b16 = prec == BS_MIXED_BF16;
        uint16_t *E16 = static_cast<uint16_t *>(ps->plane_f1_d.p) + ps->foff[p];
        auto defect = [&]() {
            return b16 ? launch_plane_defect_bf16(R32, D32, E16, nx, ny, nz, c, eps, s)
                       : launch_plane_defect(R, D, F1, nx, ny, nz, c, eps, s);
        };
        auto chain = [&](int epi, int acc) {
            return b16 ? chain_bf16(ps, p, c, colour, epi, acc, src, dst, omega, s)
                       : chain_lowp(ps, p, c, colour, 1, epi, acc, src, dst, omega, s);
        };
        // E = low-precision R was written by the residual kernel
        bs_status st;
        if (refine == 0) {
            if ((st = chain(kEpiUpdate, 0)) != BS_OK) return st;
            continue;
        }
        if ((st = chain(kEpiD64, 0)) != BS_OK) return st;
        for (int j = 0; j < refine; ++j) {
            hipError_t e = defect();
            if (e != hipSuccess) return hip_fail(e, "plane defect");
            // the last defect step updates u straight from its product
            if ((st = chain(j + 1 < refine ? kEpiD64 : kEpiUpdateAcc, 1)) != BS_OK) return st;
        }
    }
    return BS_OK;
}

// R = residual (f layout) for the FP64 chain and for refined mixed solves
// (FP32 for the BF16 chain); the mixed solves also get E = low-precision R in
// F1 (R itself is skipped when nothing reads it).
bs_status residual_into_scratch(bs_patchset *ps, const double *u, const double *f, hipStream_t s, int prec,
                                int refine)
{
    ResidArgs a{};
    a.u = u;
    a.f = f;
    a.r = (prec == BS_FP64 || (prec == BS_MIXED_FP32 && refine > 0)) ? static_cast<double *>(ps->plane_r_d.p)
                                                                       : nullptr;
    if (prec == BS_MIXED_BF16 && refine > 0) a.r32 = static_cast<float *>(ps->plane_r_d.p);
    if (prec == BS_MIXED_FP32) a.e32 = static_cast<float *>(ps->plane_f1_d.p);
    if (prec == BS_MIXED_BF16) a.e16 = static_cast<uint16_t *>(ps->plane_f1_d.p);
    a.partial = nullptr;
    a.pd = static_cast<const PatchDesc *>(ps->desc_d.p);
    a.tiles = static_cast<const ResidTile *>(ps->rtile_d.p);
    hipError_t e = launch_residual(a, ps->nrtiles, s);
    if (e != hipSuccess) return hip_fail(e, "plane residual");
    return BS_OK;
}

}  // namespace

// One FP64 plane half-step for the adjoint's recomputation: dst = src + omega
// P M^{-1} r(src) on the planes of `colour` (-1: all; dst == src in place).
bs_status plane_step(bs_patchset *ps, int normal, int colour, const double *src, double *dst, const double *f,
                     double omega, hipStream_t s)
{
    bs_status st;
    if (!ps->plane_ready && (st = build_plane_tables(ps)) != BS_OK) return st;
    if ((st = residual_into_scratch(ps, src, f, s, BS_FP64, 0)) != BS_OK) return st;
    return plane_pass(ps, normal, colour, BS_FP64, 0, src, dst, omega, s);
}

// out += M^{-1} P rhs on the planes of `colour`, rhs = r(src) = h^2 f - A src
// (f given) or src's interior (f null); out (u layout) is zero where the
// result goes, so that it receives M^{-1} P rhs there.
bs_status plane_solve(bs_patchset *ps, int normal, int colour, const double *src, const double *f, double *out,
                      hipStream_t s)
{
    bs_status st;
    if (!ps->plane_ready && (st = build_plane_tables(ps)) != BS_OK) return st;
    if (f) {
        if ((st = residual_into_scratch(ps, src, f, s, BS_FP64, 0)) != BS_OK) return st;
    } else {
        hipError_t e = launch_u_to_f(src, static_cast<double *>(ps->plane_r_d.p),
                                     static_cast<const PatchDesc *>(ps->desc_d.p), ps->npatch, s);
        if (e != hipSuccess) return hip_fail(e, "field copy");
    }
    return plane_pass(ps, normal, colour, BS_FP64, 0, out, out, 1.0, s);
}

}  // namespace bs

using namespace bs;

extern "C" {

bs_status bs_plane_relax(bs_patchset *ps, int32_t normal_axis, bs_scheme scheme, double omega, int32_t nsweeps,
                         bs_precision prec, int32_t refine, double *u, const double *f, double *work,
                         hipStream_t stream)
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
    if (any_bc(ps) && prec != BS_FP64)
        return fail(BS_ERR_UNSUPPORTED, "bs_plane_relax: extrapolated faces with mixed precision");
    if (nsweeps == 0) return BS_OK;
    bs_status st;
    if (!ps->plane_ready && (st = build_plane_tables(ps)) != BS_OK) return st;
    if (prec != BS_FP64 && (st = ensure_mixed_scratch(ps)) != BS_OK) return st;
    const int rf = prec == BS_FP64 ? 0 : refine;
    const PatchDesc *pdd = static_cast<const PatchDesc *>(ps->desc_d.p);
    // ghosts of linked faces are exchanged after every sweep (section 2)
    auto ghosts = [&](double *v) -> bs_status {
        if (!ghost_active(ps)) return BS_OK;
        hipError_t e = ghost_update(ps, v, false, stream);
        return e == hipSuccess ? BS_OK : hip_fail(e, "ghost update");
    };
    if (scheme == BS_JACOBI) {
        hipError_t e = launch_ghost_copy(u, work, pdd, ps->npatch, stream);
        if (e != hipSuccess) return hip_fail(e, "ghost copy");
        for (int sw = 0; sw < nsweeps; ++sw) {
            const double *src = (sw & 1) ? work : u;
            double *dst = (sw & 1) ? u : work;
            if ((st = residual_into_scratch(ps, src, f, stream, prec, rf)) != BS_OK) return st;
            if ((st = plane_pass(ps, normal_axis, -1, prec, rf, src, dst, omega, stream)) != BS_OK) return st;
            if ((st = ghosts(dst)) != BS_OK) return st;
        }
        if (nsweeps & 1) {
            e = launch_interior_copy(work, u, pdd, ps->npatch, stream);
            if (e != hipSuccess) return hip_fail(e, "interior copy");
            if ((st = ghosts(u)) != BS_OK) return st;
        }
        return BS_OK;
    }
    // Gauss-Seidel: planes of colour 0, then colour 1 (the chaotic scheme runs
    // the same colour-major order), in place
    for (int sw = 0; sw < nsweeps; ++sw) {
        for (int colour = 0; colour < 2; ++colour) {
            if ((st = residual_into_scratch(ps, u, f, stream, prec, rf)) != BS_OK) return st;
            if ((st = plane_pass(ps, normal_axis, colour, prec, rf, u, u, omega, stream)) != BS_OK) return st;
        }
        if ((st = ghosts(u)) != BS_OK) return st;
    }
    return BS_OK;
}

// Host-side test hooks (not part of the public header).

// One batched product C_b = A_b B_b with the FP64 kernel's store (epi 0) or
// scale (epi 1, scale indexed [b*sc_b + m*sc_m + n*sc_n]) epilogue.
int bsi_gemm_f64(const double *A, int64_t lda, int64_t sA, const double *B, int64_t ldb, int64_t sB, double *C,
                 int64_t ldc, int64_t sC, int M, int N, int K, int batch, int epi, const double *scale, int64_t sc_b,
                 int64_t sc_m, int64_t sc_n, hipStream_t s)
{
    if (epi != kEpiStore && epi != kEpiScale) return BS_ERR_INVALID;
    GemmArgs g{};
    g.A = A; g.lda = lda; g.sA = sA;
    g.B = B; g.ldb = ldb; g.sB = sB;
    g.C = C; g.ldc = ldc; g.sC = sC;
    g.M = M; g.N = N; g.K = K; g.batch = batch;
    g.scale = scale; g.sc_b = sc_b; g.sc_m = sc_m; g.sc_n = sc_n;
    g.ncolour = -1;
    return launch_gemm_f64(g, epi, s) == hipSuccess ? BS_OK : BS_ERR_HIP;
}

// The same with FP32 operands (prec 1), store epilogue, dlayout as in
// GemmMixedArgs.
int bsi_gemm_mixed(const float *A, int64_t lda, int64_t sA, const float *B, int64_t ldb, int64_t sB, float *C,
                   int64_t ldc, int64_t sC, int M, int N, int K, int batch, int prec, int dlayout, hipStream_t s)
{
    if (prec != 1) return BS_ERR_INVALID;
    GemmMixedArgs g{};
    g.A = A; g.lda = lda; g.sA = sA;
    g.B = B; g.ldb = ldb; g.sB = sB;
    g.C = C; g.ldc = ldc; g.sC = sC;
    g.M = M; g.N = N; g.K = K; g.batch = batch;
    g.ncolour = -1;
    g.dlayout = dlayout;
    return launch_gemm_mixed(g, prec, kEpiStore, s) == hipSuccess ? BS_OK : BS_ERR_HIP;
}

// One batched BF16 product (operands and result as BF16 bit patterns): store
// (epi 0) or scale (epi 1) epilogue; b_trans as in launch_gemm_bf16.
int bsi_gemm_bf16(const uint16_t *A, int64_t lda, int64_t sA, const uint16_t *B, int64_t ldb, int64_t sB,
                  int b_trans, uint16_t *C, int64_t ldc, int64_t sC, int M, int N, int K, int batch, int epi,
                  const float *scale, int64_t sc_b, int64_t sc_m, int64_t sc_n, hipStream_t s)
{
    if (epi != kEpiStore && epi != kEpiScale) return BS_ERR_INVALID;
    GemmBf16Args g{};
    g.A = A; g.lda = lda; g.sA = sA;
    g.B = B; g.ldb = ldb; g.sB = sB;
    g.C = C; g.ldc = ldc; g.sC = sC;
    g.M = M; g.N = N; g.K = K; g.batch = batch;
    g.scale = scale; g.sc_b = sc_b; g.sc_m = sc_m; g.sc_n = sc_n;
    g.ncolour = -1;
    return launch_gemm_bf16(g, b_trans, epi, s) == hipSuccess ? BS_OK : BS_ERR_HIP;
}

// Operand staging of the BF16 products (process-wide): -1 default, 0 through
// registers, 1 direct to LDS where the shapes allow it.
int bsi_set_bf16_async(int mode)
{
    if (mode < -1 || mode > 1) return BS_ERR_INVALID;
    set_bf16_async(mode);
    return BS_OK;
}

// Order of the FP32 plane chain for normals y and z: 1 (default) left
// products first and last, 0 right products first and last (the FP64 chain's
// order: there the other order measured slower, 6.98 against 6.75 ms per
// 512^3 sweep; for FP32 it is faster, 4.25 against 4.79 ms).
int bsi_set_plane_lr(bs_patchset *ps, int lr)
{
    if (!ps || (lr != 0 && lr != 1)) return BS_ERR_INVALID;
    ps->plane_lr = lr != 0;
    clear_graphs(ps);
    return BS_OK;
}

// Register-to-row mapping used by the mixed products of this patch set.
int bsi_set_mixed_dlayout(bs_patchset *ps, int dlayout)
{
    if (!ps || (dlayout != 0 && dlayout != 1)) return BS_ERR_INVALID;
    ps->mixed_dlayout = dlayout;
    return BS_OK;
}

}  // extern "C"
