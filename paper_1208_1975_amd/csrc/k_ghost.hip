// Ghost updates between smoothing steps and the line blocks next to
// extrapolated faces.
//
// Section 2 updates the ghosts of a patch Jacobi-fashion after every full
// smoothing step, from the neighbouring patches' new values (section 1.1: the
// ghosts of interior patch faces keep the patches consistent).  A face that
// carries the extrapolated Dirichlet condition instead holds the negated
// adjacent interior value (the value at the face is zero), which folds into
// the operator as eps_a on the adjacent cells' diagonal.
#include "bs_internal.h"

namespace bs {

// One workgroup per item: up to kFaceItemCells cells of one face operation,
// the faster index a running across consecutive threads (contiguous for
// faces normal to y or z).
__global__ void __launch_bounds__(256) k_face_ops(double *u, const FaceOp *ops, const FaceItem *items)
{
    const FaceItem it = items[blockIdx.x];
    const FaceOp op = ops[it.op];
    for (int k = threadIdx.x; k < it.count; k += blockDim.x) {
        const int c = it.first + k;
        const int b = c / op.m1, a = c - b * op.m1;
        const double v = u[op.s0 + (int64_t)a * op.s1 + (int64_t)b * op.s2];
        u[op.d0 + (int64_t)a * op.d1 + (int64_t)b * op.d2] = op.sign * v;
    }
}

hipError_t launch_face_ops(double *u, const FaceOp *ops, const FaceItem *items, int nitems, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_face_ops, dim3(nitems), dim3(256), 0, s, u, ops, items);
    return hipGetLastError();
}

// Geometry of boundary line `line` along axis ax: first cell in u and f, the
// strides along the line, its length, and the diagonal shift from the
// extrapolated faces parallel to it.
struct BLineGeo {
    int64_t u0, f0, sa, fa, ub, uc;
    int na;
    double shift;
    bool xb_lo, xb_hi, xc_lo, xc_hi, lo_a, hi_a;
};

__device__ __forceinline__ BLineGeo bline_geo(const PatchDesc *pd, const BLineItem &it, int ax)
{
    BLineGeo g;
    const int b = ax == 0 ? 1 : 0, c = ax == 2 ? 1 : 2;   // the other axes, lower first
    const int n[3] = {pd->n[0], pd->n[1], pd->n[2]};
    const int64_t us[3] = {1, n[0] + 2, (int64_t)(n[0] + 2) * (n[1] + 2)};
    const int64_t fs[3] = {1, n[0], (int64_t)n[0] * n[1]};
    const int bc = pd->bc;
    g.xb_lo = ((bc >> (2 * b)) & 1) && it.p == 0;
    g.xb_hi = ((bc >> (2 * b + 1)) & 1) && it.p == n[b] - 1;
    g.xc_lo = ((bc >> (2 * c)) & 1) && it.q == 0;
    g.xc_hi = ((bc >> (2 * c + 1)) & 1) && it.q == n[c] - 1;
    g.lo_a = (bc >> (2 * ax)) & 1;
    g.hi_a = (bc >> (2 * ax + 1)) & 1;
    g.shift = (g.xb_lo ? pd->eps[b] : 0.0) + (g.xb_hi ? pd->eps[b] : 0.0) + (g.xc_lo ? pd->eps[c] : 0.0) +
              (g.xc_hi ? pd->eps[c] : 0.0);
    g.u0 = pd->uoff + us[0] + us[1] + us[2] + (int64_t)it.p * us[b] + (int64_t)it.q * us[c];
    g.f0 = pd->foff + (int64_t)it.p * fs[b] + (int64_t)it.q * fs[c];
    g.sa = us[ax];
    g.fa = fs[ax];
    g.ub = us[b];
    g.uc = us[c];
    g.na = n[ax];
    return g;
}

// Residuals of the boundary lines, one thread per cell (thread i: cell
// t = i / nitems of line first + i % nitems), into scratch row 2t + 1: the
// line's residual r = h^2 f - A u from the source, with every extrapolated
// neighbour taken as the negated cell itself.
__global__ void __launch_bounds__(256) k_bline_resid(BLineArgs a, int maxlen)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)a.nitems * maxlen) return;
    const int l = (int)(i % a.nitems), t = (int)(i / a.nitems);
    const int line = a.first + l;
    const BLineItem it = a.items[line];
    const PatchDesc *pd = a.pd + it.patch;
    const int ax = a.axis;
    const BLineGeo g = bline_geo(pd, it, ax);
    if (t >= g.na) return;
    const double *src = a.src;
    const int b = ax == 0 ? 1 : 0, c = ax == 2 ? 1 : 2;
    const double ea = pd->eps[ax], eb = pd->eps[b], ec = pd->eps[c];
    const double d = 2.0 * (pd->eps[0] + pd->eps[1] + pd->eps[2]);
    const int64_t cu = g.u0 + (int64_t)t * g.sa;
    const double uc = src[cu];
    const double lo = (t == 0 && g.lo_a) ? -uc : src[cu - g.sa];
    const double hi = (t == g.na - 1 && g.hi_a) ? -uc : src[cu + g.sa];
    const double bl = g.xb_lo ? -uc : src[cu - g.ub], bh = g.xb_hi ? -uc : src[cu + g.ub];
    const double cl = g.xc_lo ? -uc : src[cu - g.uc], ch = g.xc_hi ? -uc : src[cu + g.uc];
    const double nb = fma(ea, lo + hi, fma(eb, bl + bh, ec * (cl + ch)));
    a.scratch[(int64_t)(2 * t + 1) * a.nlines + line] = fma(-d, uc, fma(pd->h2, a.f[g.f0 + (int64_t)t * g.fa], nb));
}

// The LU factors of each boundary line's block tridiag(-eps_a, d_t, -eps_a),
// d_t = 2(eps_x + eps_y + eps_z) plus eps_b for every extrapolated face next
// to the line (its whole length) and eps_a at an extrapolated end: pivots
// m_0 = d_0, m_t = d_t - eps_a (eps_a / m_{t-1}); stored as the multiplier
// eps_a / m_{t-1} (0 for t = 0) and 1 / m_t, [t][line] like the scratch.
__global__ void __launch_bounds__(256) k_bline_factors(BLineArgs a)
{
    const int line = blockIdx.x * blockDim.x + threadIdx.x;
    if (line >= a.nitems) return;
    const BLineItem it = a.items[line];
    const PatchDesc *pd = a.pd + it.patch;
    const int ax = a.axis;
    const BLineGeo g = bline_geo(pd, it, ax);
    const double ea = pd->eps[ax];
    const double dd = 2.0 * (pd->eps[0] + pd->eps[1] + pd->eps[2]) + g.shift;
    const int64_t L = a.nlines;
    double mprev = 1.0;
    for (int t = 0; t < g.na; ++t) {
        const double dt = dd + (t == 0 && g.lo_a ? ea : 0.0) + (t == g.na - 1 && g.hi_a ? ea : 0.0);
        const double gm = t == 0 ? 0.0 : ea / mprev;
        const double m = fma(-ea, gm, dt);
        a.fac[(int64_t)(2 * t) * L + line] = gm;
        a.fac[(int64_t)(2 * t + 1) * L + line] = 1.0 / m;
        mprev = m;
    }
}

// One thread per line: the Thomas algorithm on the line block with the
// factors of k_bline_factors.  The forward elimination z_t = r_t + g_t z_{t-1}
// overwrites the residual with the eliminated right-hand side; the back
// substitution du_t = (z_t + eps_a du_{t+1}) / m_t writes dst = src + omega du.
// The loads of B cells are issued together before the recurrences consume
// them, so the chains are FMAs and a memory round trip is paid once per B
// cells.  In place (src == dst) every cell of the line is read before it is
// written.
__global__ void __launch_bounds__(256) k_bline(BLineArgs a)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= a.nitems) return;
    const int line = a.first + l;
    const BLineItem it = a.items[line];
    const PatchDesc *pd = a.pd + it.patch;
    const int ax = a.axis;
    const BLineGeo g = bline_geo(pd, it, ax);
    const double ea = pd->eps[ax];
    const int na = g.na;
    double *sc = a.scratch + line;
    const double *fc = a.fac + line;
    const int64_t L = a.nlines;
    constexpr int B = 16;
    double zprev = 0.0;
    for (int t0 = 0; t0 < na; t0 += B) {
        double rb[B], gb[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int t = t0 + k < na ? t0 + k : na - 1;
            rb[k] = sc[(int64_t)(2 * t + 1) * L];
            gb[k] = fc[(int64_t)(2 * t) * L];
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int t = t0 + k;
            if (t < na) {
                const double z = fma(gb[k], zprev, rb[k]);
                sc[(int64_t)(2 * t + 1) * L] = z;
                zprev = z;
            }
        }
    }
    double du = 0.0;
    for (int t1 = na - 1; t1 >= 0; t1 -= B) {
        // this batch's factors, eliminated right-hand sides and old values
        // (each cell's old value is read before its new value is stored)
        double qb[B], zb[B], ub[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int t = t1 - k >= 0 ? t1 - k : 0;
            qb[k] = fc[(int64_t)(2 * t + 1) * L];
            zb[k] = sc[(int64_t)(2 * t + 1) * L];
            ub[k] = a.src[g.u0 + (int64_t)t * g.sa];
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int t = t1 - k;
            if (t >= 0) {
                du = (t == na - 1 ? zb[k] : fma(ea, du, zb[k])) * qb[k];
                a.dst[g.u0 + (int64_t)t * g.sa] = fma(a.omega, du, ub[k]);
            }
        }
    }
}

hipError_t launch_bline_factors(const BLineArgs &a, hipStream_t s)
{
    if (a.nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bline_factors, dim3((a.nitems + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_bline(const BLineArgs &a, int maxlen, hipStream_t s)
{
    if (a.nitems <= 0) return hipSuccess;
    const int64_t cells = (int64_t)a.nitems * maxlen;
    hipLaunchKernelGGL(k_bline_resid, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, a, maxlen);
    hipLaunchKernelGGL(k_bline, dim3((a.nitems + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace bs
