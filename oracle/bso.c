/*
 * bso.c -- the oracle: a plain, slow, FP64 CPU implementation of block
 * relaxation for the constant-coefficient 7-point stencil, written from the
 * paper (Birke, Philip, Wang, Berrill, "Block-Relaxation Methods for 3D
 * Constant-Coefficient Stencils on GPUs and Multicore CPUs").
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  The product path (the HIP
 * library) shares no code, header, table or helper with this file.
 *
 * Conventions (section 1.1 and the index-space discussion of section 2.1):
 *   - a patch has nx*ny*nz interior cells, x fastest;
 *   - u is stored WITH one ghost layer: (nz+2)(ny+2)(nx+2) doubles, interior
 *     cell (i,j,k) at ((k+1)(ny+2)+(j+1))(nx+2)+(i+1);
 *   - f is stored WITHOUT ghosts: nz*ny*nx doubles, cell (i,j,k) at
 *     (k*ny+j)*nx+i.
 *   - Ghosts are caller data and never change during a sweep; boundary cells
 *     use the same stencil as interior cells (section 1.1).  Zero Dirichlet
 *     means a zero ghost layer.
 *
 * Operator (eq. stencil3d7, with one weight per axis; at eps = (1,1,1) it is
 * exactly the paper's stencil):
 *   (A u)_c = sum_a eps_a (2 u_c - u_{c-e_a} - u_{c+e_a}),  b = h^2 f,
 *   r = b - A u  over interior cells.
 *
 * Iteration (eq. blockiteration2, residual-correction form):
 *   u_b <- u_b + omega * M_b^{-1} r_b
 * where M_b is the diagonal block of A for block b:
 *   - a line along axis a: tridiag(-eps_a, d, -eps_a), d = 2(eps_x+eps_y+eps_z);
 *   - a plane with normal c (in-plane axes a<b): d I - eps_a(shifts in a)
 *     - eps_b(shifts in b), truncated at the plane edge.
 * Schemes (section 2, Algorithm 1 and eq. sm:blockm):
 *   - Jacobi: every block from the same old u, written to a second vector;
 *   - lexicographic block Gauss-Seidel: blocks visited in lexicographic order
 *     of their free indices (lower axis fastest), each using the current u;
 *   - coloured block Gauss-Seidel: colour = (sum of the free indices) mod 2
 *     for lines, plane index mod 2 for planes; colour 0 first, then colour 1.
 *
 * Numerical choices:
 *   - line solves: the textbook Thomas algorithm, factorised on every call;
 *   - plane solves: partial diagonalisation -- an explicit sine transform
 *     along the lower in-plane axis (DST-I basis, integer-reduced argument),
 *     one Thomas solve per sine mode along the other axis, inverse transform;
 *   - sums of squares accumulate in long double in a fixed order.
 * Compile with -ffp-contract=off so no FMA contraction changes the rounding.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { BSO_JACOBI = 0, BSO_LEX_GS = 1, BSO_COLORED_GS = 2 };

typedef struct {
    int nx, ny, nz;
    double ex, ey, ez, h2;
    ptrdiff_t sx, sy;   /* u strides in y and z (padded) */
    int bc;             /* extrapolated-Dirichlet faces: bit 2a low, bit 2a+1 high face of axis a */
} grid_t;

static grid_t mkgrid(int nx, int ny, int nz, const double eps[3], double h)
{
    grid_t g;
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.ex = eps[0]; g.ey = eps[1]; g.ez = eps[2];
    g.h2 = h * h;
    g.sx = nx + 2;
    g.sy = (ptrdiff_t)(nx + 2) * (ny + 2);
    g.bc = 0;
    return g;
}

static inline ptrdiff_t uidx(const grid_t *g, int i, int j, int k)
{
    return (ptrdiff_t)(k + 1) * g->sy + (ptrdiff_t)(j + 1) * g->sx + (i + 1);
}

static inline ptrdiff_t fidx(const grid_t *g, int i, int j, int k)
{
    return ((ptrdiff_t)k * g->ny + j) * g->nx + i;
}

static int dim_of(const grid_t *g, int a) { return a == 0 ? g->nx : (a == 1 ? g->ny : g->nz); }
static double eps_of(const grid_t *g, int a) { return a == 0 ? g->ex : (a == 1 ? g->ey : g->ez); }
static ptrdiff_t ustride_of(const grid_t *g, int a) { return a == 0 ? 1 : (a == 1 ? g->sx : g->sy); }

/* Boundary reading (section 1.1: boundary conditions are extrapolated into the
 * ghost layer).  By default the ghosts are data (zero Dirichlet = a zero ghost
 * layer).  A face whose bit is set in bc instead takes the value that puts
 * zero on the face between the boundary cell and its ghost, ghost = -(the
 * adjacent interior value), so the stencil's ghost term folds into the
 * operator: the boundary cell's diagonal gains eps_a and the ghost is never
 * read.  Neighbour of cell c (index t along axis a, n_a cells) on side dir. */
static inline double nbr(const grid_t *g, const double *u, ptrdiff_t c, int a, int t, int dir)
{
    ptrdiff_t st = a == 0 ? 1 : (a == 1 ? g->sx : g->sy);
    int n = a == 0 ? g->nx : (a == 1 ? g->ny : g->nz);
    if (dir < 0 && t == 0 && (g->bc >> (2 * a) & 1)) return -u[c];
    if (dir > 0 && t == n - 1 && (g->bc >> (2 * a + 1) & 1)) return -u[c];
    return dir < 0 ? u[c - st] : u[c + st];
}

/* Residual of one interior cell: h^2 f - (A u) (eq. stencil3d7 with axis weights). */
static inline double cell_res(const grid_t *g, const double *u, const double *f, int i, int j, int k)
{
    ptrdiff_t c = uidx(g, i, j, k);
    if (g->bc) {
        double ax = g->ex * (2.0 * u[c] - nbr(g, u, c, 0, i, -1) - nbr(g, u, c, 0, i, 1));
        double ay = g->ey * (2.0 * u[c] - nbr(g, u, c, 1, j, -1) - nbr(g, u, c, 1, j, 1));
        double az = g->ez * (2.0 * u[c] - nbr(g, u, c, 2, k, -1) - nbr(g, u, c, 2, k, 1));
        return g->h2 * f[fidx(g, i, j, k)] - (ax + ay + az);
    }
    double ax = g->ex * (2.0 * u[c] - u[c - 1] - u[c + 1]);
    double ay = g->ey * (2.0 * u[c] - u[c - g->sx] - u[c + g->sx]);
    double az = g->ez * (2.0 * u[c] - u[c - g->sy] - u[c + g->sy]);
    return g->h2 * f[fidx(g, i, j, k)] - (ax + ay + az);
}

/* Diagonal of the operator at cell (i,j,k): sum_a eps_a (2 + the number of
 * extrapolated faces of axis a that the cell touches). */
static double diag_at(const grid_t *g, int i, int j, int k)
{
    const int t[3] = {i, j, k}, n[3] = {g->nx, g->ny, g->nz};
    const double e[3] = {g->ex, g->ey, g->ez};
    double d = 0.0;
    for (int a = 0; a < 3; ++a) {
        double m = 2.0;
        if (t[a] == 0 && (g->bc >> (2 * a) & 1)) m += 1.0;
        if (t[a] == n[a] - 1 && (g->bc >> (2 * a + 1) & 1)) m += 1.0;
        d += e[a] * m;
    }
    return d;
}

static int g_threads = 0;
void bso_set_threads(int n) { g_threads = n; }
int bso_get_threads(void)
{
#ifdef _OPENMP
    return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
    return 1;
#endif
}
#ifdef _OPENMP
#define NT bso_get_threads()
#endif

/* ------------------------------------------------------------------------- */
/* Residual and its norm (the quantity monitored in section 3).               */
/* ------------------------------------------------------------------------- */

/* r (unpadded, may be NULL) = h^2 f - A u; returns sum of r^2 over interior
 * cells, accumulated in long double in k,j,i order. */
double bso_residual_bc(int nx, int ny, int nz, const double eps[3], double h,
                       const double *u, const double *f, double *r, int bc)
{
    grid_t g = mkgrid(nx, ny, nz, eps, h);
    g.bc = bc;
    long double *part = (long double *)calloc((size_t)nz, sizeof(long double));
#ifdef _OPENMP
#pragma omp parallel for num_threads(NT) schedule(static)
#endif
    for (int k = 0; k < nz; ++k) {
        long double s = 0.0L;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double v = cell_res(&g, u, f, i, j, k);
                if (r) r[fidx(&g, i, j, k)] = v;
                s += (long double)v * (long double)v;
            }
        part[k] = s;
    }
    long double tot = 0.0L;
    for (int k = 0; k < nz; ++k) tot += part[k];
    free(part);
    return (double)tot;
}

double bso_residual(int nx, int ny, int nz, const double eps[3], double h,
                    const double *u, const double *f, double *r)
{
    return bso_residual_bc(nx, ny, nz, eps, h, u, f, r, 0);
}

/* ------------------------------------------------------------------------- */
/* Tridiagonal solve (textbook Thomas algorithm, Conte & de Boor form).       */
/* Solves tridiag(off, diag, off) x = rhs for a symmetric Toeplitz system,    */
/* factorising on every call.  cp is scratch of length n.  x may alias rhs.   */
/* ------------------------------------------------------------------------- */
static void thomas(int n, double off, double diag, const double *rhs, double *x, double *cp)
{
    /* forward elimination */
    double denom = diag;
    cp[0] = off / denom;
    x[0] = rhs[0] / denom;
    for (int i = 1; i < n; ++i) {
        denom = diag - off * cp[i - 1];
        cp[i] = off / denom;
        x[i] = (rhs[i] - off * x[i - 1]) / denom;
    }
    /* back substitution */
    for (int i = n - 2; i >= 0; --i)
        x[i] = x[i] - cp[i] * x[i + 1];
}

/* The same for tridiag(off, diag[t], off) with a diagonal that varies along the
 * line (extrapolated boundary faces). */
static void thomas_v(int n, double off, const double *diag, const double *rhs, double *x, double *cp)
{
    double denom = diag[0];
    cp[0] = off / denom;
    x[0] = rhs[0] / denom;
    for (int i = 1; i < n; ++i) {
        denom = diag[i] - off * cp[i - 1];
        cp[i] = off / denom;
        x[i] = (rhs[i] - off * x[i - 1]) / denom;
    }
    for (int i = n - 2; i >= 0; --i)
        x[i] = x[i] - cp[i] * x[i + 1];
}

/* Exposed for the test that pins the line solver against a banded LAPACK solve. */
void bso_tridiag_solve(int n, double off, double diag, const double *rhs, double *x)
{
    double *cp = (double *)malloc(sizeof(double) * (size_t)n);
    thomas(n, off, diag, rhs, x, cp);
    free(cp);
}

/* ------------------------------------------------------------------------- */
/* Line blocks.                                                               */
/* A line along axis a is named by its two free indices (p, q): p is the      */
/* lower remaining axis, q the higher one.                                    */
/* ------------------------------------------------------------------------- */
static void line_cell(int axis, int p, int q, int t, int *i, int *j, int *k)
{
    if (axis == 0) { *i = t; *j = p; *k = q; }
    else if (axis == 1) { *i = p; *j = t; *k = q; }
    else { *i = p; *j = q; *k = t; }
}

static void free_dims(const grid_t *g, int axis, int *np, int *nq)
{
    if (axis == 0) { *np = g->ny; *nq = g->nz; }
    else if (axis == 1) { *np = g->nx; *nq = g->nz; }
    else { *np = g->nx; *nq = g->ny; }
}

/* One block update of line (p,q): residual from usrc, exact tridiagonal
 * solve, udst = usrc + omega*du on the line's cells.  All residuals are formed
 * before any value is written, so usrc == udst (in place) is allowed.
 * buf must hold 3n doubles. */
static void line_update(const grid_t *g, int axis, int p, int q, const double *usrc,
                        double *udst, const double *f, double omega, double *buf)
{
    int n = dim_of(g, axis);
    double ea = eps_of(g, axis);
    double d = 2.0 * (g->ex + g->ey + g->ez);
    double *r = buf, *cp = buf + n;
    int i, j, k;
    for (int t = 0; t < n; ++t) {
        line_cell(axis, p, q, t, &i, &j, &k);
        r[t] = cell_res(g, usrc, f, i, j, k);
    }
    if (g->bc) {
        double *dg = buf + 2 * (size_t)n;
        for (int t = 0; t < n; ++t) {
            line_cell(axis, p, q, t, &i, &j, &k);
            dg[t] = diag_at(g, i, j, k);
        }
        thomas_v(n, -ea, dg, r, r, cp);
    } else {
        thomas(n, -ea, d, r, r, cp);
    }
    for (int t = 0; t < n; ++t) {
        line_cell(axis, p, q, t, &i, &j, &k);
        ptrdiff_t c = uidx(g, i, j, k);
        udst[c] = usrc[c] + omega * r[t];
    }
}

static void copy_padded(const grid_t *g, const double *src, double *dst)
{
    size_t n = (size_t)(g->nz + 2) * (size_t)g->sy;
    memcpy(dst, src, n * sizeof(double));
}

/* Line sweeps.  scheme: 0 Jacobi, 1 lexicographic GS, 2 coloured GS.
 * lex_form: 0 = the serial lexicographic loop (the definition);
 *           1 = the anti-diagonal form: lines (p,q) with equal p+q are
 *               mutually uncoupled and all their already-updated neighbours
 *               lie on the previous anti-diagonal, so processing diagonals in
 *               order gives bit-identical results, in parallel.
 * Returns 0 on success, nonzero on bad arguments. */
int bso_line_sweeps_bc(int nx, int ny, int nz, const double eps[3], double h, int axis,
                       int scheme, double omega, int nsweeps, int lex_form,
                       double *u, const double *f, int bc)
{
    if (nx < 1 || ny < 1 || nz < 1 || axis < 0 || axis > 2 || nsweeps < 0 || bc < 0 || bc > 63) return 1;
    grid_t g = mkgrid(nx, ny, nz, eps, h);
    g.bc = bc;
    int n = dim_of(&g, axis), np, nq;
    free_dims(&g, axis, &np, &nq);
    size_t tot = (size_t)(nz + 2) * (size_t)g.sy;
    double *v = NULL;
    if (scheme == BSO_JACOBI) {
        v = (double *)malloc(tot * sizeof(double));
        copy_padded(&g, u, v);   /* ghosts of the second vector = ghosts of u */
    }
    for (int s = 0; s < nsweeps; ++s) {
        if (scheme == BSO_JACOBI) {
#ifdef _OPENMP
#pragma omp parallel num_threads(NT)
#endif
            {
                double *buf = (double *)malloc(sizeof(double) * 3 * (size_t)n);
#ifdef _OPENMP
#pragma omp for collapse(2) schedule(static)
#endif
                for (int q = 0; q < nq; ++q)
                    for (int p = 0; p < np; ++p)
                        line_update(&g, axis, p, q, u, v, f, omega, buf);
                free(buf);
            }
            double *t = u; /* copy back (the oracle keeps the result in u) */
            copy_padded(&g, v, t);
        } else if (scheme == BSO_LEX_GS) {
            if (lex_form == 0) {
                double *buf = (double *)malloc(sizeof(double) * 3 * (size_t)n);
                for (int q = 0; q < nq; ++q)
                    for (int p = 0; p < np; ++p)
                        line_update(&g, axis, p, q, u, u, f, omega, buf);
                free(buf);
            } else {
#ifdef _OPENMP
#pragma omp parallel num_threads(NT)
#endif
                {
                    double *buf = (double *)malloc(sizeof(double) * 3 * (size_t)n);
                    for (int dg = 0; dg <= (np - 1) + (nq - 1); ++dg) {
                        int qlo = dg - (np - 1) > 0 ? dg - (np - 1) : 0;
                        int qhi = dg < nq - 1 ? dg : nq - 1;
                        /* the loop's implicit barrier ends each anti-diagonal */
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
                        for (int q = qlo; q <= qhi; ++q)
                            line_update(&g, axis, dg - q, q, u, u, f, omega, buf);
                    }
                    free(buf);
                }
            }
        } else if (scheme == BSO_COLORED_GS) {
            for (int colour = 0; colour < 2; ++colour) {
#ifdef _OPENMP
#pragma omp parallel num_threads(NT)
#endif
                {
                    double *buf = (double *)malloc(sizeof(double) * 3 * (size_t)n);
#ifdef _OPENMP
#pragma omp for collapse(2) schedule(static)
#endif
                    for (int q = 0; q < nq; ++q)
                        for (int p = 0; p < np; ++p)
                            if (((p + q) & 1) == colour)
                                line_update(&g, axis, p, q, u, u, f, omega, buf);
                    free(buf);
                }
            }
        } else {
            free(v);
            return 2;
        }
    }
    free(v);
    return 0;
}

int bso_line_sweeps(int nx, int ny, int nz, const double eps[3], double h, int axis,
                    int scheme, double omega, int nsweeps, int lex_form,
                    double *u, const double *f)
{
    return bso_line_sweeps_bc(nx, ny, nz, eps, h, axis, scheme, omega, nsweeps, lex_form, u, f, 0);
}

/* ------------------------------------------------------------------------- */
/* Plane blocks, solved by partial diagonalisation.                           */
/* Plane with normal c at index s; in-plane axes a < b.  The plane block is   */
/*   M = T_a (x) I + I (x) T'_b,  T_a = tridiag(-eps_a, 2eps_a, -eps_a),      */
/*   T'_b = tridiag(-eps_b, 2eps_b + 2eps_c, -eps_b).                          */
/* T_a = S diag(sigma) S with the orthonormal DST-I basis                      */
/*   S[i][p] = sqrt(2/(n+1)) sin(pi (i+1)(p+1)/(n+1)),                         */
/*   sigma_p = 4 eps_a sin^2((p+1) pi / (2(n+1))).                             */
/* Transforming along a leaves one tridiagonal system in b per mode p.         */
/* ------------------------------------------------------------------------- */
typedef struct {
    int na, nb;
    double *S;      /* na*na, S[i*na + p] */
    double *sigma;  /* na */
} sine_basis_t;

static sine_basis_t make_basis(int na, double ea)
{
    sine_basis_t B;
    B.na = na; B.nb = 0;
    B.S = (double *)malloc(sizeof(double) * (size_t)na * na);
    B.sigma = (double *)malloc(sizeof(double) * (size_t)na);
    const double scale = sqrt(2.0 / (double)(na + 1));
    const long period = 2L * (na + 1);
    for (int i = 0; i < na; ++i)
        for (int p = 0; p < na; ++p) {
            long m = ((long)(i + 1) * (long)(p + 1)) % period;   /* exact reduction */
            B.S[(size_t)i * na + p] = scale * sin(M_PI * (double)m / (double)(na + 1));
        }
    for (int p = 0; p < na; ++p) {
        double s = sin(M_PI * (double)(p + 1) / (2.0 * (double)(na + 1)));
        B.sigma[p] = 4.0 * ea * s * s;
    }
    return B;
}

/* Orthonormal eigenbasis of tridiag(-1, 2, -1) on n cells whose low / high end
 * is an extrapolated face (diagonal 3 there), and its eigenvalues times ea.
 * The eigenvectors are sines sampled at the cell centres:
 *   neither end: sin(theta (i+1)),      theta = (p+1) pi / (n+1)    (DST-I)
 *   both ends:   sin(theta (i+1/2)),    theta = (p+1) pi / n        (DST-II)
 *   low end:     sin(theta (i+1/2)),    theta = (p+1) pi / (n+1/2)
 *   high end:    sin(theta (n-i-1/2)),  the mirror image,
 * with eigenvalue 4 sin^2(theta/2) (the extrapolated ghost -v_0 and the zero
 * ghost v_n are what these sines take one cell beyond each end).  Sine
 * arguments are reduced in integers; columns are normalised by their sums of
 * squares. */
static sine_basis_t make_basis_bc(int na, double ea, int lo, int hi)
{
    if (!lo && !hi) return make_basis(na, ea);
    sine_basis_t B;
    B.na = na; B.nb = 0;
    B.S = (double *)malloc(sizeof(double) * (size_t)na * na);
    B.sigma = (double *)malloc(sizeof(double) * (size_t)na);
    /* theta (i + 1/2) = pi m / den with the integer m below */
    long den = (lo && hi) ? 2L * na : 2L * na + 1;
    for (int p = 0; p < na; ++p) {
        long double ss = 0.0L;
        for (int i = 0; i < na; ++i) {
            long ii = (lo ? i : na - 1 - i);
            long m = ((long)(p + 1) * (2 * ii + 1)) % (2 * den);
            double v = sin(M_PI * (double)m / (double)den);
            B.S[(size_t)i * na + p] = v;
            ss += (long double)v * v;
        }
        double sc = (double)(1.0L / sqrtl(ss));
        for (int i = 0; i < na; ++i) B.S[(size_t)i * na + p] *= sc;
        double s = sin(M_PI * (double)(p + 1) / (double)den);
        B.sigma[p] = 4.0 * ea * s * s;
    }
    return B;
}

static void free_basis(sine_basis_t *B) { free(B->S); free(B->sigma); }

static void plane_axes(int normal, int *a, int *b)
{
    if (normal == 0) { *a = 1; *b = 2; }
    else if (normal == 1) { *a = 0; *b = 2; }
    else { *a = 0; *b = 1; }
}

static void plane_cell(int normal, int s, int ia, int ib, int *i, int *j, int *k)
{
    if (normal == 0) { *i = s; *j = ia; *k = ib; }
    else if (normal == 1) { *i = ia; *j = s; *k = ib; }
    else { *i = ia; *j = ib; *k = s; }
}

/* buf must hold 3*na*nb + 2*nb doubles. */
static void plane_update(const grid_t *g, int normal, int s, const sine_basis_t *B,
                         const double *usrc, double *udst, const double *f, double omega,
                         double *buf)
{
    int a, b;
    plane_axes(normal, &a, &b);
    int na = dim_of(g, a), nb = dim_of(g, b);
    double eb = eps_of(g, b), ec = eps_of(g, normal);
    double *r = buf;                          /* r[ia*nb + ib] */
    double *rh = buf + (size_t)na * nb;       /* rh[p*nb + ib] */
    double *w = buf + 2 * (size_t)na * nb;    /* w[ia*nb + ib] */
    double *cp = buf + 3 * (size_t)na * nb;   /* nb */
    int i, j, k;
    for (int ia = 0; ia < na; ++ia)
        for (int ib = 0; ib < nb; ++ib) {
            plane_cell(normal, s, ia, ib, &i, &j, &k);
            r[(size_t)ia * nb + ib] = cell_res(g, usrc, f, i, j, k);
        }
    /* forward sine transform along a: rh[p][ib] = sum_ia S[ia][p] r[ia][ib] */
    for (int p = 0; p < na; ++p)
        for (int ib = 0; ib < nb; ++ib) {
            double acc = 0.0;
            for (int ia = 0; ia < na; ++ia)
                acc += B->S[(size_t)ia * na + p] * r[(size_t)ia * nb + ib];
            rh[(size_t)p * nb + ib] = acc;
        }
    /* one tridiagonal solve along b per mode (with extrapolated faces, the
     * ends along b and the planes at extrapolated faces of c have their
     * diagonal raised by the folded ghost terms) */
    if (g->bc) {
        double *dg = cp + nb;
        int sc = s;
        double cdiag = ec * (2.0 + ((sc == 0 && (g->bc >> (2 * normal) & 1)) ? 1.0 : 0.0) +
                             ((sc == dim_of(g, normal) - 1 && (g->bc >> (2 * normal + 1) & 1)) ? 1.0 : 0.0));
        for (int p = 0; p < na; ++p) {
            for (int ib = 0; ib < nb; ++ib) {
                double m = 2.0;
                if (ib == 0 && (g->bc >> (2 * b) & 1)) m += 1.0;
                if (ib == nb - 1 && (g->bc >> (2 * b + 1) & 1)) m += 1.0;
                dg[ib] = B->sigma[p] + eb * m + cdiag;
            }
            thomas_v(nb, -eb, dg, rh + (size_t)p * nb, rh + (size_t)p * nb, cp);
        }
    } else {
        for (int p = 0; p < na; ++p)
            thomas(nb, -eb, B->sigma[p] + 2.0 * eb + 2.0 * ec, rh + (size_t)p * nb,
                   rh + (size_t)p * nb, cp);
    }
    /* inverse transform: w[ia][ib] = sum_p S[ia][p] rh[p][ib] */
    for (int ia = 0; ia < na; ++ia)
        for (int ib = 0; ib < nb; ++ib) {
            double acc = 0.0;
            for (int p = 0; p < na; ++p)
                acc += B->S[(size_t)ia * na + p] * rh[(size_t)p * nb + ib];
            w[(size_t)ia * nb + ib] = acc;
        }
    for (int ia = 0; ia < na; ++ia)
        for (int ib = 0; ib < nb; ++ib) {
            plane_cell(normal, s, ia, ib, &i, &j, &k);
            ptrdiff_t c = uidx(g, i, j, k);
            udst[c] = usrc[c] + omega * w[(size_t)ia * nb + ib];
        }
}

/* Plane sweeps (normal axis 0/1/2).  scheme as for lines; lexicographic GS
 * visits planes s = 0..n_c-1 in order. */
int bso_plane_sweeps_bc(int nx, int ny, int nz, const double eps[3], double h, int normal,
                        int scheme, double omega, int nsweeps, double *u, const double *f, int bc)
{
    if (nx < 1 || ny < 1 || nz < 1 || normal < 0 || normal > 2 || nsweeps < 0 || bc < 0 || bc > 63) return 1;
    grid_t g = mkgrid(nx, ny, nz, eps, h);
    g.bc = bc;
    int a, b;
    plane_axes(normal, &a, &b);
    int na = dim_of(&g, a), nb = dim_of(&g, b), nc = dim_of(&g, normal);
    sine_basis_t B = make_basis_bc(na, eps_of(&g, a), bc >> (2 * a) & 1, bc >> (2 * a + 1) & 1);
    size_t tot = (size_t)(nz + 2) * (size_t)g.sy;
    size_t bufn = 3 * (size_t)na * nb + 2 * (size_t)nb;
    double *v = NULL;
    if (scheme == BSO_JACOBI) {
        v = (double *)malloc(tot * sizeof(double));
        copy_padded(&g, u, v);
    }
    for (int sw = 0; sw < nsweeps; ++sw) {
        if (scheme == BSO_JACOBI) {
#ifdef _OPENMP
#pragma omp parallel num_threads(NT)
#endif
            {
                double *buf = (double *)malloc(sizeof(double) * bufn);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
                for (int s = 0; s < nc; ++s)
                    plane_update(&g, normal, s, &B, u, v, f, omega, buf);
                free(buf);
            }
            copy_padded(&g, v, u);
        } else if (scheme == BSO_LEX_GS) {
            double *buf = (double *)malloc(sizeof(double) * bufn);
            for (int s = 0; s < nc; ++s)
                plane_update(&g, normal, s, &B, u, u, f, omega, buf);
            free(buf);
        } else if (scheme == BSO_COLORED_GS) {
            for (int colour = 0; colour < 2; ++colour) {
#ifdef _OPENMP
#pragma omp parallel num_threads(NT)
#endif
                {
                    double *buf = (double *)malloc(sizeof(double) * bufn);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
                    for (int s = 0; s < nc; ++s)
                        if ((s & 1) == colour)
                            plane_update(&g, normal, s, &B, u, u, f, omega, buf);
                    free(buf);
                }
            }
        } else {
            free(v);
            free_basis(&B);
            return 2;
        }
    }
    free(v);
    free_basis(&B);
    return 0;
}

int bso_plane_sweeps(int nx, int ny, int nz, const double eps[3], double h, int normal,
                     int scheme, double omega, int nsweeps, double *u, const double *f)
{
    return bso_plane_sweeps_bc(nx, ny, nz, eps, h, normal, scheme, omega, nsweeps, u, f, 0);
}

/* One Jacobi plane update restricted to a list of planes, reading usrc and
 * writing udst (padded).  Used to check single planes of a large sweep. */
int bso_plane_update_some(int nx, int ny, int nz, const double eps[3], double h, int normal,
                          double omega, int nplanes, const int *planes,
                          const double *usrc, double *udst, const double *f)
{
    if (nx < 1 || ny < 1 || nz < 1 || normal < 0 || normal > 2) return 1;
    grid_t g = mkgrid(nx, ny, nz, eps, h);
    int a, b;
    plane_axes(normal, &a, &b);
    int na = dim_of(&g, a), nb = dim_of(&g, b), nc = dim_of(&g, normal);
    sine_basis_t B = make_basis(na, eps_of(&g, a));
    size_t bufn = 3 * (size_t)na * nb + 2 * (size_t)nb;
    int bad = 0;
#ifdef _OPENMP
#pragma omp parallel num_threads(NT)
#endif
    {
        double *buf = (double *)malloc(sizeof(double) * bufn);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int t = 0; t < nplanes; ++t) {
            if (planes[t] < 0 || planes[t] >= nc) { bad = 1; continue; }
            plane_update(&g, normal, planes[t], &B, usrc, udst, f, omega, buf);
        }
        free(buf);
    }
    free_basis(&B);
    return bad;
}

/* One line update for a list of lines (p,q), reading usrc, writing udst. */
int bso_line_update_some(int nx, int ny, int nz, const double eps[3], double h, int axis,
                         double omega, int nlines, const int *pq,
                         const double *usrc, double *udst, const double *f)
{
    if (nx < 1 || ny < 1 || nz < 1 || axis < 0 || axis > 2) return 1;
    grid_t g = mkgrid(nx, ny, nz, eps, h);
    int n = dim_of(&g, axis), np, nq, bad = 0;
    free_dims(&g, axis, &np, &nq);
    double *buf = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    for (int t = 0; t < nlines; ++t) {
        int p = pq[2 * t], q = pq[2 * t + 1];
        if (p < 0 || p >= np || q < 0 || q >= nq) { bad = 1; continue; }
        line_update(&g, axis, p, q, usrc, udst, f, omega, buf);
    }
    free(buf);
    return bad;
}

/* ------------------------------------------------------------------------- */
/* Geometric cube blocks (section 2: lexicographically ordered geometric       */
/* blocks of bx*by*bz cells; Algorithm 1 and the GPU block Jacobi algorithm    */
/* with the block inverse).  Blocks tile the patch from its origin; along an   */
/* axis whose length is not a multiple of the block edge the last block is     */
/* shorter, with its own block matrix (the option of the block-inversion      */
/* section that precomputes every inverse instead of overlapping blocks).      */
/* Block (bi,bj,bk) covers cells i in [bi*bx, min((bi+1)bx, nx)), etc.; its    */
/* cells are numbered x fastest.  The block matrix A_b is A restricted to the  */
/* block's cells (coupling to cells outside the block goes to the residual);   */
/* it is symmetric positive definite, and each block system is solved by a    */
/* Cholesky factorisation formed on every call (the definition, not a fast    */
/* method).                                                                    */
/* Schemes: Jacobi; lexicographic block GS (bi fastest, then bj, then bk);     */
/* coloured block GS with colour (bi+bj+bk) mod 2, colour 0 first.             */
/* ------------------------------------------------------------------------- */

/* In-place Cholesky A = L L^T of an n x n SPD matrix (row-major; only the
 * lower triangle is read, and it is overwritten by L), then x = A^{-1} b by
 * two triangular solves.
 * x may alias b.  Returns nonzero if a pivot is not positive. */
static int chol_solve(int n, double *A, const double *b, double *x)
{
    for (int j = 0; j < n; ++j) {
        double s = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) s -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
        if (!(s > 0.0)) return 1;
        double ljj = sqrt(s);
        A[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double t = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
            A[(size_t)i * n + j] = t / ljj;
        }
    }
    for (int i = 0; i < n; ++i) {          /* L y = b */
        double t = b[i];
        for (int k = 0; k < i; ++k) t -= A[(size_t)i * n + k] * x[k];
        x[i] = t / A[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {     /* L^T x = y */
        double t = x[i];
        for (int k = i + 1; k < n; ++k) t -= A[(size_t)k * n + i] * x[k];
        x[i] = t / A[(size_t)i * n + i];
    }
    return 0;
}

/* One update of cube block (bi,bj,bk): residual of its cells from usrc, exact
 * block solve, udst = usrc + omega*du on its cells.  All residuals are formed
 * before any write, so usrc == udst is allowed.  buf: nb*nb + nb doubles,
 * nb = bx*by*bz. */
static int cube_update(const grid_t *g, int bx, int by, int bz, int bi, int bj, int bk,
                       const double *usrc, double *udst, const double *f, double omega, double *buf)
{
    int i0 = bi * bx, j0 = bj * by, k0 = bk * bz;
    int ni = g->nx - i0 < bx ? g->nx - i0 : bx;
    int nj = g->ny - j0 < by ? g->ny - j0 : by;
    int nk = g->nz - k0 < bz ? g->nz - k0 : bz;
    int nb = ni * nj * nk;
    double d = 2.0 * (g->ex + g->ey + g->ez);
    double *A = buf, *r = buf + (size_t)nb * nb;
    memset(A, 0, sizeof(double) * (size_t)nb * nb);
    for (int ck = 0; ck < nk; ++ck)
        for (int cj = 0; cj < nj; ++cj)
            for (int ci = 0; ci < ni; ++ci) {
                int c = (ck * nj + cj) * ni + ci;
                r[c] = cell_res(g, usrc, f, i0 + ci, j0 + cj, k0 + ck);
                A[(size_t)c * nb + c] = g->bc ? diag_at(g, i0 + ci, j0 + cj, k0 + ck) : d;
                if (ci > 0) A[(size_t)c * nb + c - 1] = -g->ex;
                if (ci + 1 < ni) A[(size_t)c * nb + c + 1] = -g->ex;
                if (cj > 0) A[(size_t)c * nb + c - ni] = -g->ey;
                if (cj + 1 < nj) A[(size_t)c * nb + c + ni] = -g->ey;
                if (ck > 0) A[(size_t)c * nb + c - ni * nj] = -g->ez;
                if (ck + 1 < nk) A[(size_t)c * nb + c + ni * nj] = -g->ez;
            }
    if (chol_solve(nb, A, r, r)) return 1;
    for (int ck = 0; ck < nk; ++ck)
        for (int cj = 0; cj < nj; ++cj)
            for (int ci = 0; ci < ni; ++ci) {
                ptrdiff_t c = uidx(g, i0 + ci, j0 + cj, k0 + ck);
                udst[c] = usrc[c] + omega * r[(ck * nj + cj) * ni + ci];
            }
    return 0;
}

/* Cube-block sweeps.  scheme: 0 Jacobi, 1 lexicographic GS, 2 coloured GS.
 * Returns 0 on success, nonzero on bad arguments. */
int bso_cube_sweeps_bc(int nx, int ny, int nz, const double eps[3], double h, int bx, int by, int bz,
                       int scheme, double omega, int nsweeps, double *u, const double *f, int bc)
{
    if (nx < 1 || ny < 1 || nz < 1 || bx < 1 || by < 1 || bz < 1 || nsweeps < 0 || bc < 0 || bc > 63) return 1;
    if (scheme < BSO_JACOBI || scheme > BSO_COLORED_GS) return 2;
    grid_t g = mkgrid(nx, ny, nz, eps, h);
    g.bc = bc;
    if (bx > nx) bx = nx;
    if (by > ny) by = ny;
    if (bz > nz) bz = nz;
    int mi = (nx + bx - 1) / bx, mj = (ny + by - 1) / by, mk = (nz + bz - 1) / bz;
    size_t nb = (size_t)bx * by * bz, bufn = nb * nb + nb;
    size_t tot = (size_t)(nz + 2) * (size_t)g.sy;
    double *v = NULL;
    int bad = 0;
    if (scheme == BSO_JACOBI) {
        v = (double *)malloc(tot * sizeof(double));
        copy_padded(&g, u, v);
    }
    for (int s = 0; s < nsweeps && !bad; ++s) {
        if (scheme == BSO_LEX_GS) {
            double *buf = (double *)malloc(sizeof(double) * bufn);
            for (int bk = 0; bk < mk; ++bk)
                for (int bj = 0; bj < mj; ++bj)
                    for (int bi = 0; bi < mi; ++bi)
                        bad |= cube_update(&g, bx, by, bz, bi, bj, bk, u, u, f, omega, buf);
            free(buf);
            continue;
        }
        /* Jacobi: one pass from u into v; coloured: two in-place passes */
        for (int colour = 0; colour < (scheme == BSO_JACOBI ? 1 : 2); ++colour) {
            double *dst = scheme == BSO_JACOBI ? v : u;
#ifdef _OPENMP
#pragma omp parallel num_threads(NT) reduction(| : bad)
#endif
            {
                double *buf = (double *)malloc(sizeof(double) * bufn);
#ifdef _OPENMP
#pragma omp for collapse(3) schedule(dynamic)
#endif
                for (int bk = 0; bk < mk; ++bk)
                    for (int bj = 0; bj < mj; ++bj)
                        for (int bi = 0; bi < mi; ++bi)
                            if (scheme == BSO_JACOBI || ((bi + bj + bk) & 1) == colour)
                                bad |= cube_update(&g, bx, by, bz, bi, bj, bk, u, dst, f, omega, buf);
                free(buf);
            }
        }
        if (scheme == BSO_JACOBI) copy_padded(&g, v, u);
    }
    free(v);
    return bad ? 3 : 0;
}

int bso_cube_sweeps(int nx, int ny, int nz, const double eps[3], double h, int bx, int by, int bz,
                    int scheme, double omega, int nsweeps, double *u, const double *f)
{
    return bso_cube_sweeps_bc(nx, ny, nz, eps, h, bx, by, bz, scheme, omega, nsweeps, u, f, 0);
}

/* ------------------------------------------------------------------------- */
/* Adjoint of K damped Jacobi line sweeps (reverse mode, every state stored). */
/*                                                                            */
/* Forward: x^{k+1} = x^k + omega M^{-1} r(x^k), r = h^2 F + B g - A_int x,   */
/* with interior unknowns x, fixed ghosts g (B g = ghost terms of the         */
/* stencil) and A_int the interior operator with zero ghosts.  M and A are    */
/* symmetric, so for a loss L with dL/dx^K = gbar:                            */
/*   lambda   = M^{-1} gbar                                                   */
/*   dL/dF   += omega h^2 lambda                                              */
/*   dL/dg   += omega B^T lambda          (face ghosts only)                  */
/*   dL/deps_a += -omega <lambda, D_a U^k + (dM/deps_a) w^k>,                 */
/*                 w^k = M^{-1} r(x^k),  D_a U = 2U - U_{-a} - U_{+a}         */
/*   gbar    <- gbar - omega A_int lambda                                     */
/* and finally dL/dx^0 = gbar.  For lines along a, dM/deps_a =                */
/* tridiag(-1,2,-1) on each line and dM/deps_other = 2 I.                     */
/* All gradient arrays are padded like u; gK's ghost entries are ignored.     */
/* g_u0 receives interior gradients and face-ghost gradients (edges and       */
/* corners are never read and get 0).                                         */
/* ------------------------------------------------------------------------- */

/* M^{-1} applied to every line of a padded field (interior), out may alias in. */
static void apply_minv_lines(const grid_t *g, int axis, const double *in, double *out)
{
    int n = dim_of(g, axis), np, nq;
    free_dims(g, axis, &np, &nq);
    double ea = eps_of(g, axis), d = 2.0 * (g->ex + g->ey + g->ez);
#ifdef _OPENMP
#pragma omp parallel num_threads(NT)
#endif
    {
        double *buf = (double *)malloc(sizeof(double) * 3 * (size_t)n);
        int i, j, k;
#ifdef _OPENMP
#pragma omp for collapse(2) schedule(static)
#endif
        for (int q = 0; q < nq; ++q)
            for (int p = 0; p < np; ++p) {
                for (int t = 0; t < n; ++t) {
                    line_cell(axis, p, q, t, &i, &j, &k);
                    buf[t] = in[uidx(g, i, j, k)];
                }
                thomas(n, -ea, d, buf, buf, buf + n);
                for (int t = 0; t < n; ++t) {
                    line_cell(axis, p, q, t, &i, &j, &k);
                    out[uidx(g, i, j, k)] = buf[t];
                }
            }
        free(buf);
    }
}

/* out = A_int x (x padded, its ghosts treated as zero), interior written. */
static void apply_a_int(const grid_t *g, const double *x, double *out)
{
#ifdef _OPENMP
#pragma omp parallel for num_threads(NT) schedule(static)
#endif
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                ptrdiff_t c = uidx(g, i, j, k);
                double xm = i > 0 ? x[c - 1] : 0.0, xp = i < g->nx - 1 ? x[c + 1] : 0.0;
                double ym = j > 0 ? x[c - g->sx] : 0.0, yp = j < g->ny - 1 ? x[c + g->sx] : 0.0;
                double zm = k > 0 ? x[c - g->sy] : 0.0, zp = k < g->nz - 1 ? x[c + g->sy] : 0.0;
                out[c] = g->ex * (2.0 * x[c] - xm - xp) + g->ey * (2.0 * x[c] - ym - yp)
                       + g->ez * (2.0 * x[c] - zm - zp);
            }
}

/* D_a U (ghosts included) at interior cell c. */
static inline double d_axis(const grid_t *g, const double *u, ptrdiff_t c, int a)
{
    ptrdiff_t s = ustride_of(g, a);
    return 2.0 * u[c] - u[c - s] - u[c + s];
}

/* (dM/deps_b) w at interior cell for lines along `axis`. */
static inline double dm_apply(const grid_t *g, int axis, int b, const double *w, int i, int j, int k)
{
    ptrdiff_t c = uidx(g, i, j, k);
    if (b != axis) return 2.0 * w[c];
    int t = axis == 0 ? i : (axis == 1 ? j : k);
    int n = dim_of(g, axis);
    ptrdiff_t s = ustride_of(g, axis);
    double lo = t > 0 ? w[c - s] : 0.0, hi = t < n - 1 ? w[c + s] : 0.0;
    return 2.0 * w[c] - lo - hi;
}

static void jacobi_line_step(const grid_t *g, int axis, double omega, const double *x,
                             double *xn, const double *f, double *w)
{
    /* w = M^{-1} r(x); xn = x + omega w (ghosts of xn = ghosts of x) */
    size_t tot = (size_t)(g->nz + 2) * (size_t)g->sy;
    memcpy(xn, x, tot * sizeof(double));
    memset(w, 0, tot * sizeof(double));
#ifdef _OPENMP
#pragma omp parallel for num_threads(NT) schedule(static)
#endif
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i)
                w[uidx(g, i, j, k)] = cell_res(g, x, f, i, j, k);
    apply_minv_lines(g, axis, w, w);
#ifdef _OPENMP
#pragma omp parallel for num_threads(NT) schedule(static)
#endif
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                ptrdiff_t c = uidx(g, i, j, k);
                xn[c] = x[c] + omega * w[c];
            }
}

/* Forward K Jacobi line sweeps that keep every state: states[(k)*tot ...]. */
int bso_line_jacobi_adjoint(int nx, int ny, int nz, const double eps[3], double h, int axis,
                            double omega, int K, const double *u0, const double *f,
                            const double *gK, double *g_u0, double *g_f, double g_eps[3])
{
    if (nx < 1 || ny < 1 || nz < 1 || axis < 0 || axis > 2 || K < 0) return 1;
    grid_t g = mkgrid(nx, ny, nz, eps, h);
    size_t tot = (size_t)(nz + 2) * (size_t)g.sy;
    double *states = (double *)malloc(sizeof(double) * tot * (size_t)(K + 1));
    double *ws = (double *)malloc(sizeof(double) * tot * (size_t)(K > 0 ? K : 1));
    memcpy(states, u0, tot * sizeof(double));
    for (int k = 0; k < K; ++k)
        jacobi_line_step(&g, axis, omega, states + (size_t)k * tot, states + (size_t)(k + 1) * tot,
                         f, ws + (size_t)k * tot);

    double *gb = (double *)calloc(tot, sizeof(double));
    double *lam = (double *)calloc(tot, sizeof(double));
    double *alam = (double *)calloc(tot, sizeof(double));
    double *gghost = (double *)calloc(tot, sizeof(double));
    long double geps[3] = {0.0L, 0.0L, 0.0L};
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                ptrdiff_t c = uidx(&g, i, j, k);
                gb[c] = gK[c];
            }
    if (g_f) memset(g_f, 0, sizeof(double) * (size_t)nx * ny * nz);
    double ev[3] = {g.ex, g.ey, g.ez};
    for (int k = K - 1; k >= 0; --k) {
        const double *U = states + (size_t)k * tot;
        const double *W = ws + (size_t)k * tot;
        apply_minv_lines(&g, axis, gb, lam);                 /* lambda = M^{-1} gbar */
        for (int b = 0; b < 3; ++b) {                          /* eps partials, fixed order */
            long double s = 0.0L;
            for (int kk = 0; kk < nz; ++kk)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        ptrdiff_t c = uidx(&g, i, j, kk);
                        double t = d_axis(&g, U, c, b) + dm_apply(&g, axis, b, W, i, j, kk);
                        s += (long double)lam[c] * (long double)t;
                    }
            geps[b] += -(long double)omega * s;
        }
        if (g_f)
            for (int kk = 0; kk < nz; ++kk)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i)
                        g_f[fidx(&g, i, j, kk)] += omega * g.h2 * lam[uidx(&g, i, j, kk)];
        /* ghost gradient: B^T lambda -- face ghost next to interior cell c gets eps_a lambda_c */
        for (int kk = 0; kk < nz; ++kk)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    ptrdiff_t c = uidx(&g, i, j, kk);
                    double l = omega * lam[c];
                    if (i == 0) gghost[c - 1] += ev[0] * l;
                    if (i == nx - 1) gghost[c + 1] += ev[0] * l;
                    if (j == 0) gghost[c - g.sx] += ev[1] * l;
                    if (j == ny - 1) gghost[c + g.sx] += ev[1] * l;
                    if (kk == 0) gghost[c - g.sy] += ev[2] * l;
                    if (kk == nz - 1) gghost[c + g.sy] += ev[2] * l;
                }
        apply_a_int(&g, lam, alam);
        for (int kk = 0; kk < nz; ++kk)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    ptrdiff_t c = uidx(&g, i, j, kk);
                    gb[c] = gb[c] - omega * alam[c];
                }
    }
    if (g_u0) {
        for (size_t t = 0; t < tot; ++t) g_u0[t] = gghost[t];
        for (int kk = 0; kk < nz; ++kk)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    ptrdiff_t c = uidx(&g, i, j, kk);
                    g_u0[c] = gb[c];
                }
    }
    if (g_eps)
        for (int b = 0; b < 3; ++b) g_eps[b] = (double)geps[b];
    free(states); free(ws); free(gb); free(lam); free(alam); free(gghost);
    return 0;
}

/* Forward-mode check of the eps gradient: the tangent t_b = dx/deps_b obeys
 *   t^{k+1} = t^k + omega M^{-1}(-D_b U^k - A_int t^k - (dM/deps_b) w^k),
 * t^0 = 0, and dL/deps_b = <gK, t^K>. */
int bso_line_jacobi_eps_tangent(int nx, int ny, int nz, const double eps[3], double h, int axis,
                                double omega, int K, const double *u0, const double *f,
                                const double *gK, double out[3])
{
    if (nx < 1 || ny < 1 || nz < 1 || axis < 0 || axis > 2 || K < 0) return 1;
    grid_t g = mkgrid(nx, ny, nz, eps, h);
    size_t tot = (size_t)(nz + 2) * (size_t)g.sy;
    double *x = (double *)malloc(sizeof(double) * tot);
    double *xn = (double *)malloc(sizeof(double) * tot);
    double *w = (double *)malloc(sizeof(double) * tot);
    double *t[3], *at = (double *)calloc(tot, sizeof(double)), *rhs = (double *)calloc(tot, sizeof(double));
    for (int b = 0; b < 3; ++b) t[b] = (double *)calloc(tot, sizeof(double));
    memcpy(x, u0, tot * sizeof(double));
    for (int k = 0; k < K; ++k) {
        /* w^k = M^{-1} r(x^k) and x^{k+1} */
        jacobi_line_step(&g, axis, omega, x, xn, f, w);
        for (int b = 0; b < 3; ++b) {
            apply_a_int(&g, t[b], at);
            for (int kk = 0; kk < nz; ++kk)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        ptrdiff_t c = uidx(&g, i, j, kk);
                        rhs[c] = -d_axis(&g, x, c, b) - at[c] - dm_apply(&g, axis, b, w, i, j, kk);
                    }
            apply_minv_lines(&g, axis, rhs, rhs);
            for (int kk = 0; kk < nz; ++kk)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        ptrdiff_t c = uidx(&g, i, j, kk);
                        t[b][c] = t[b][c] + omega * rhs[c];
                    }
        }
        double *sw = x; x = xn; xn = sw;
    }
    for (int b = 0; b < 3; ++b) {
        long double s = 0.0L;
        for (int kk = 0; kk < nz; ++kk)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    ptrdiff_t c = uidx(&g, i, j, kk);
                    s += (long double)gK[c] * (long double)t[b][c];
                }
        out[b] = (double)s;
    }
    free(x); free(xn); free(w); free(at); free(rhs);
    for (int b = 0; b < 3; ++b) free(t[b]);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Reverse mode for line or plane blocks under damped block Jacobi or         */
/* two-colour block GS.  A sweep is a sequence of half-steps                  */
/*   x <- x + omega P M^{-1} r(x),                                            */
/* P the projection onto the blocks updated by the half-step (all blocks for  */
/* Jacobi; colour 0, then colour 1 for GS).  M is block diagonal and P picks  */
/* whole blocks, so P M^{-1} = M^{-1} P, and with M, A symmetric the adjoint   */
/* of one half-step, for gbar = dL/dx after it, is the Jacobi one with        */
/*   lambda = M^{-1} P gbar,                                                  */
/*   w      = P M^{-1} r(x)        (x the state before the half-step),        */
/* and the half-steps are reversed (colour 1 before colour 0).  dM/deps_b is  */
/* the 1D operator tridiag(-1,2,-1) inside the block along an axis the block  */
/* spans, 2 I along the others.  Every state is stored (no checkpoints).      */
/* ------------------------------------------------------------------------- */

/* Is (i,j,k) in a block of colour `colour` (-1: every block)? */
static int in_colour(int kind, int axis, int colour, int i, int j, int k)
{
    if (colour < 0) return 1;
    if (kind == 1) return ((axis == 0 ? i : (axis == 1 ? j : k)) & 1) == colour;
    int pq = axis == 0 ? j + k : (axis == 1 ? i + k : i + j);
    return (pq & 1) == colour;
}

/* M^{-1} applied to every plane normal to `normal` (zero ghosts within a
 * plane): sine transform along the lower in-plane axis a, one tridiagonal
 * solve per mode along b, inverse transform.  out may alias in. */
static void apply_minv_planes(const grid_t *g, int normal, const double *in, double *out)
{
    int a, b;
    plane_axes(normal, &a, &b);
    int na = dim_of(g, a), nb = dim_of(g, b), ns = dim_of(g, normal);
    double eb = eps_of(g, b), ec = eps_of(g, normal);
    sine_basis_t B = make_basis(na, eps_of(g, a));
    double *r = (double *)malloc(sizeof(double) * (size_t)na * nb);
    double *rh = (double *)malloc(sizeof(double) * (size_t)na * nb);
    double *cp = (double *)malloc(sizeof(double) * (size_t)nb);
    int i, j, k;
    for (int sidx = 0; sidx < ns; ++sidx) {
        for (int ia = 0; ia < na; ++ia)
            for (int ib = 0; ib < nb; ++ib) {
                plane_cell(normal, sidx, ia, ib, &i, &j, &k);
                r[(size_t)ia * nb + ib] = in[uidx(g, i, j, k)];
            }
        for (int p = 0; p < na; ++p)
            for (int ib = 0; ib < nb; ++ib) {
                double acc = 0.0;
                for (int ia = 0; ia < na; ++ia) acc += B.S[(size_t)ia * na + p] * r[(size_t)ia * nb + ib];
                rh[(size_t)p * nb + ib] = acc;
            }
        for (int p = 0; p < na; ++p)
            thomas(nb, -eb, B.sigma[p] + 2.0 * eb + 2.0 * ec, rh + (size_t)p * nb, rh + (size_t)p * nb, cp);
        for (int ia = 0; ia < na; ++ia)
            for (int ib = 0; ib < nb; ++ib) {
                double acc = 0.0;
                for (int p = 0; p < na; ++p) acc += B.S[(size_t)ia * na + p] * rh[(size_t)p * nb + ib];
                plane_cell(normal, sidx, ia, ib, &i, &j, &k);
                out[uidx(g, i, j, k)] = acc;
            }
    }
    free(r); free(rh); free(cp); free_basis(&B);
}

static void apply_minv_blocks(const grid_t *g, int kind, int axis, const double *in, double *out)
{
    if (kind == 0) apply_minv_lines(g, axis, in, out);
    else apply_minv_planes(g, axis, in, out);
}

/* (dM/deps_b) w at interior cell (i,j,k) for blocks of `kind` along / normal
 * to `axis`: the block spans axis b for lines along b and for planes whose
 * normal is not b. */
static double dm_apply_blocks(const grid_t *g, int kind, int axis, int b, const double *w, int i, int j, int k)
{
    ptrdiff_t c = uidx(g, i, j, k);
    int spans = kind == 0 ? b == axis : b != axis;
    if (!spans) return 2.0 * w[c];
    int t = b == 0 ? i : (b == 1 ? j : k);
    int n = dim_of(g, b);
    ptrdiff_t s = ustride_of(g, b);
    double lo = t > 0 ? w[c - s] : 0.0, hi = t < n - 1 ? w[c + s] : 0.0;
    return 2.0 * w[c] - lo - hi;
}

/* kind 0: lines along axis, 1: planes normal to axis; scheme BSO_JACOBI or
 * BSO_COLORED_GS.  Outputs as bso_line_jacobi_adjoint. */
int bso_block_adjoint(int nx, int ny, int nz, const double eps[3], double h, int kind, int axis, int scheme,
                      double omega, int K, const double *u0, const double *f, const double *gK, double *g_u0,
                      double *g_f, double g_eps[3])
{
    if (nx < 1 || ny < 1 || nz < 1 || axis < 0 || axis > 2 || K < 0 || (kind != 0 && kind != 1)) return 1;
    if (scheme != BSO_JACOBI && scheme != BSO_COLORED_GS) return 1;
    grid_t g = mkgrid(nx, ny, nz, eps, h);
    size_t tot = (size_t)(nz + 2) * (size_t)g.sy;
    int H = scheme == BSO_JACOBI ? 1 : 2;
    int S = K * H;
    double *states = (double *)malloc(sizeof(double) * tot * (size_t)(S + 1));
    double *ws = (double *)calloc(tot * (size_t)(S > 0 ? S : 1), sizeof(double));
    memcpy(states, u0, tot * sizeof(double));
    /* forward: every half-step's state and its w = P M^{-1} r(x) */
    for (int st = 0; st < S; ++st) {
        int colour = H == 1 ? -1 : st % 2;
        const double *x = states + (size_t)st * tot;
        double *xn = states + (size_t)(st + 1) * tot;
        double *w = ws + (size_t)st * tot;
        memcpy(xn, x, tot * sizeof(double));
        for (int kk = 0; kk < nz; ++kk)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) w[uidx(&g, i, j, kk)] = cell_res(&g, x, f, i, j, kk);
        apply_minv_blocks(&g, kind, axis, w, w);
        for (int kk = 0; kk < nz; ++kk)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    ptrdiff_t c = uidx(&g, i, j, kk);
                    if (!in_colour(kind, axis, colour, i, j, kk)) w[c] = 0.0;
                    xn[c] = x[c] + omega * w[c];
                }
    }
    double *gb = (double *)calloc(tot, sizeof(double));
    double *lam = (double *)calloc(tot, sizeof(double));
    double *alam = (double *)calloc(tot, sizeof(double));
    double *gghost = (double *)calloc(tot, sizeof(double));
    long double geps[3] = {0.0L, 0.0L, 0.0L};
    for (int kk = 0; kk < nz; ++kk)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) gb[uidx(&g, i, j, kk)] = gK[uidx(&g, i, j, kk)];
    if (g_f) memset(g_f, 0, sizeof(double) * (size_t)nx * ny * nz);
    double ev[3] = {g.ex, g.ey, g.ez};
    for (int st = S - 1; st >= 0; --st) {
        int colour = H == 1 ? -1 : st % 2;
        const double *U = states + (size_t)st * tot;
        const double *W = ws + (size_t)st * tot;
        /* lambda = M^{-1} P gbar */
        for (int kk = 0; kk < nz; ++kk)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    ptrdiff_t c = uidx(&g, i, j, kk);
                    lam[c] = in_colour(kind, axis, colour, i, j, kk) ? gb[c] : 0.0;
                }
        apply_minv_blocks(&g, kind, axis, lam, lam);
        for (int b = 0; b < 3; ++b) {
            long double sacc = 0.0L;
            for (int kk = 0; kk < nz; ++kk)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        ptrdiff_t c = uidx(&g, i, j, kk);
                        double t = d_axis(&g, U, c, b) + dm_apply_blocks(&g, kind, axis, b, W, i, j, kk);
                        sacc += (long double)lam[c] * (long double)t;
                    }
            geps[b] += -(long double)omega * sacc;
        }
        if (g_f)
            for (int kk = 0; kk < nz; ++kk)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) g_f[fidx(&g, i, j, kk)] += omega * g.h2 * lam[uidx(&g, i, j, kk)];
        for (int kk = 0; kk < nz; ++kk)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    ptrdiff_t c = uidx(&g, i, j, kk);
                    double l = omega * lam[c];
                    if (i == 0) gghost[c - 1] += ev[0] * l;
                    if (i == nx - 1) gghost[c + 1] += ev[0] * l;
                    if (j == 0) gghost[c - g.sx] += ev[1] * l;
                    if (j == ny - 1) gghost[c + g.sx] += ev[1] * l;
                    if (kk == 0) gghost[c - g.sy] += ev[2] * l;
                    if (kk == nz - 1) gghost[c + g.sy] += ev[2] * l;
                }
        apply_a_int(&g, lam, alam);
        for (int kk = 0; kk < nz; ++kk)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    ptrdiff_t c = uidx(&g, i, j, kk);
                    gb[c] = gb[c] - omega * alam[c];
                }
    }
    if (g_u0) {
        for (size_t t = 0; t < tot; ++t) g_u0[t] = gghost[t];
        for (int kk = 0; kk < nz; ++kk)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) g_u0[uidx(&g, i, j, kk)] = gb[uidx(&g, i, j, kk)];
    }
    if (g_eps)
        for (int b = 0; b < 3; ++b) g_eps[b] = (double)geps[b];
    free(states); free(ws); free(gb); free(lam); free(alam); free(gghost);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Ghost exchange between adjacent patches (section 2: the ghost cells that   */
/* patches share are updated Jacobi-fashion once a full smoothing step is     */
/* done; section 1.1: such interior ghosts carry the values of the            */
/* neighbouring patch).  A link (a, axis, b) says that patch b lies on patch  */
/* a's high side along `axis`, face to face: both have the same extents along */
/* the two other axes.  The exchange copies b's first interior layer along    */
/* `axis` into a's ghost layer at index n_a, and a's last interior layer into */
/* b's ghost layer at index -1.  Every copy reads interior cells and writes   */
/* ghost cells, so the copies can run in any order.                          */
/* ------------------------------------------------------------------------- */
int bso_exchange_ghosts(int npatch, const int *dims, double *const *us, int nlinks, const int *links)
{
    for (int t = 0; t < nlinks; ++t) {
        int a = links[3 * t], axis = links[3 * t + 1], b = links[3 * t + 2];
        if (a < 0 || a >= npatch || b < 0 || b >= npatch || a == b || axis < 0 || axis > 2) return 1;
        for (int o = 0; o < 3; ++o)
            if (o != axis && dims[3 * a + o] != dims[3 * b + o]) return 2;
    }
    for (int t = 0; t < nlinks; ++t) {
        int a = links[3 * t], axis = links[3 * t + 1], b = links[3 * t + 2];
        const double eps1[3] = {1.0, 1.0, 1.0};
        grid_t ga = mkgrid(dims[3 * a], dims[3 * a + 1], dims[3 * a + 2], eps1, 1.0);
        grid_t gb = mkgrid(dims[3 * b], dims[3 * b + 1], dims[3 * b + 2], eps1, 1.0);
        int na = dim_of(&ga, axis);
        /* the two tangential axes, lower first */
        int t1 = axis == 0 ? 1 : 0, t2 = axis == 2 ? 1 : 2;
        int m1 = dim_of(&ga, t1), m2 = dim_of(&ga, t2);
        for (int q = 0; q < m2; ++q)
            for (int p = 0; p < m1; ++p) {
                int ia[3], ib[3];
                ia[t1] = ib[t1] = p;
                ia[t2] = ib[t2] = q;
                /* a's ghost at n_a <- b's cell 0 */
                ia[axis] = na;
                ib[axis] = 0;
                us[a][uidx(&ga, ia[0], ia[1], ia[2])] = us[b][uidx(&gb, ib[0], ib[1], ib[2])];
                /* b's ghost at -1 <- a's cell n_a - 1 */
                ia[axis] = na - 1;
                ib[axis] = -1;
                us[b][uidx(&gb, ib[0], ib[1], ib[2])] = us[a][uidx(&ga, ia[0], ia[1], ia[2])];
            }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Multigrid transfers on cell-centred grids (the line and plane smoothers    */
/* are components of geometric multigrid: section 1 and the future work of   */
/* section 5).  A coarse cell (I,J,K) covers the fine cells (2I+a, 2J+b,      */
/* 2K+c), a,b,c in {0,1}; fine dims are even.                                */
/*   restriction: the mean of the eight fine values, times `scale`;           */
/*   prolongation: trilinear interpolation between coarse cell centres: along */
/*   each axis a fine cell takes 3/4 of its parent and 1/4 of the parent's    */
/*   neighbour on the fine cell's side (a coarse ghost at the edge), so the   */
/*   eight weights are products of 3/4 and 1/4.                               */
/* ------------------------------------------------------------------------- */
int bso_restrict(int nx, int ny, int nz, const double *rfine, double scale, double *fcoarse)
{
    if (nx < 2 || ny < 2 || nz < 2 || (nx | ny | nz) & 1) return 1;
    int mx = nx / 2, my = ny / 2, mz = nz / 2;
    for (int K = 0; K < mz; ++K)
        for (int J = 0; J < my; ++J)
            for (int I = 0; I < mx; ++I) {
                double s = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a)
                            s += rfine[((size_t)(2 * K + c) * ny + (2 * J + b)) * nx + (2 * I + a)];
                fcoarse[((size_t)K * my + J) * mx + I] = scale * (s / 8.0);
            }
    return 0;
}

/* Coarse value at (I,J,K), any index one cell outside: read as stored, except
 * across a face whose bit is set in bc, where the value is the extrapolated
 * one, -(the reflected interior value) (per axis: an edge or corner ghost
 * flips sign once per extrapolated axis it lies beyond). */
static double coarse_at(const grid_t *gc, const double *uc, int I, int J, int K, int bc)
{
    int t[3] = {I, J, K};
    const int n[3] = {gc->nx, gc->ny, gc->nz};
    double sg = 1.0;
    for (int a = 0; a < 3; ++a) {
        if (t[a] < 0 && (bc >> (2 * a) & 1)) { t[a] = 0; sg = -sg; }
        if (t[a] >= n[a] && (bc >> (2 * a + 1) & 1)) { t[a] = n[a] - 1; sg = -sg; }
    }
    return sg * uc[uidx(gc, t[0], t[1], t[2])];
}

int bso_prolong_add_bc(int nx, int ny, int nz, const double *ucoarse, double *ufine, int bc)
{
    if (nx < 2 || ny < 2 || nz < 2 || (nx | ny | nz) & 1 || bc < 0 || bc > 63) return 1;
    const double eps1[3] = {1.0, 1.0, 1.0};
    grid_t gf = mkgrid(nx, ny, nz, eps1, 1.0);
    grid_t gc = mkgrid(nx / 2, ny / 2, nz / 2, eps1, 1.0);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int I = i / 2, J = j / 2, K = k / 2;
                /* the neighbour coarse cell on the fine cell's side */
                int di = (i & 1) ? 1 : -1, dj = (j & 1) ? 1 : -1, dk = (k & 1) ? 1 : -1;
                double v = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a) {
                            double w = (a ? 0.25 : 0.75) * (b ? 0.25 : 0.75) * (c ? 0.25 : 0.75);
                            v += w * coarse_at(&gc, ucoarse, I + a * di, J + b * dj, K + c * dk, bc);
                        }
                ufine[uidx(&gf, i, j, k)] += v;
            }
    return 0;
}

int bso_prolong_add(int nx, int ny, int nz, const double *ucoarse, double *ufine)
{
    return bso_prolong_add_bc(nx, ny, nz, ucoarse, ufine, 0);
}
