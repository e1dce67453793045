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

// One thread per line.  The line's residual r = h^2 f - A u is formed from the
// source with every extrapolated neighbour taken as the negated cell itself;
// the line block tridiag(-eps_a, d_t, -eps_a) has d_t = 2(eps_x + eps_y +
// eps_z) plus eps_b for every extrapolated face next to the line (its whole
// length) and eps_a at an extrapolated end.  Thomas algorithm: the forward
// elimination stores the reciprocal pivots and the eliminated right-hand side
// in the scratch ([t][line], coalesced across the threads), the back
// substitution reads them and writes dst = src + omega du.  In place (src ==
// dst) every cell of the line is read before it is written.
__global__ void __launch_bounds__(256) k_bline(BLineArgs a)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= a.nitems) return;
    const int line = a.first + l;
    const BLineItem it = a.items[line];
    const PatchDesc *pd = a.pd + it.patch;
    const int ax = a.axis;
    const int b = ax == 0 ? 1 : 0, c = ax == 2 ? 1 : 2;   // the other axes, lower first
    const int n[3] = {pd->n[0], pd->n[1], pd->n[2]};
    const int64_t us[3] = {1, n[0] + 2, (int64_t)(n[0] + 2) * (n[1] + 2)};
    const int64_t fs[3] = {1, n[0], (int64_t)n[0] * n[1]};
    const int bc = pd->bc;
    const double e[3] = {pd->eps[0], pd->eps[1], pd->eps[2]};
    const double ea = e[ax];
    const double d = 2.0 * (e[0] + e[1] + e[2]);
    double shift = 0.0;
    if (((bc >> (2 * b)) & 1) && it.p == 0) shift += e[b];
    if (((bc >> (2 * b + 1)) & 1) && it.p == n[b] - 1) shift += e[b];
    if (((bc >> (2 * c)) & 1) && it.q == 0) shift += e[c];
    if (((bc >> (2 * c + 1)) & 1) && it.q == n[c] - 1) shift += e[c];
    const bool lo_a = (bc >> (2 * ax)) & 1, hi_a = (bc >> (2 * ax + 1)) & 1;
    // the line's first cell in u and f
    const int64_t u0 = pd->uoff + us[0] + us[1] + us[2] + (int64_t)it.p * us[b] + (int64_t)it.q * us[c];
    const int64_t f0 = pd->foff + (int64_t)it.p * fs[b] + (int64_t)it.q * fs[c];
    const int64_t sa = us[ax], fa = fs[ax];
    // off-line neighbours: +-1 along b and c, extrapolated ones replaced by -u
    const bool xb_lo = ((bc >> (2 * b)) & 1) && it.p == 0, xb_hi = ((bc >> (2 * b + 1)) & 1) && it.p == n[b] - 1;
    const bool xc_lo = ((bc >> (2 * c)) & 1) && it.q == 0, xc_hi = ((bc >> (2 * c + 1)) & 1) && it.q == n[c] - 1;
    const int na = n[ax];
    const double *src = a.src;
    const double h2 = pd->h2;
    // scratch row 2t: reciprocal pivot of cell t, row 2t + 1: eliminated rhs
    double uprev = 0.0, ucur = src[u0], mprev = 1.0, zprev = 0.0;
    for (int t = 0; t < na; ++t) {
        const int64_t cu = u0 + (int64_t)t * sa;
        const double unext = t + 1 < na ? src[cu + sa] : 0.0;
        const double lo = t == 0 ? (lo_a ? -ucur : src[cu - sa]) : uprev;
        const double hi = t == na - 1 ? (hi_a ? -ucur : src[cu + sa]) : unext;
        const double bl = xb_lo ? -ucur : src[cu - us[b]], bh = xb_hi ? -ucur : src[cu + us[b]];
        const double cl = xc_lo ? -ucur : src[cu - us[c]], ch = xc_hi ? -ucur : src[cu + us[c]];
        const double nb = ea * (lo + hi) + e[b] * (bl + bh) + e[c] * (cl + ch);
        const double r = fma(-d, ucur, fma(h2, a.f[f0 + (int64_t)t * fa], nb));
        const double dt = d + shift + (t == 0 && lo_a ? ea : 0.0) + (t == na - 1 && hi_a ? ea : 0.0);
        double m, z;
        if (t == 0) {
            m = dt;
            z = r;
        } else {
            const double g = ea / mprev;
            m = dt - ea * g;
            z = fma(g, zprev, r);
        }
        a.scratch[(int64_t)(2 * t) * a.nlines + line] = 1.0 / m;
        a.scratch[(int64_t)(2 * t + 1) * a.nlines + line] = z;
        mprev = m;
        zprev = z;
        uprev = ucur;
        ucur = unext;
    }
    double du = 0.0;
    for (int t = na - 1; t >= 0; --t) {
        const double q = a.scratch[(int64_t)(2 * t) * a.nlines + line];
        const double z = a.scratch[(int64_t)(2 * t + 1) * a.nlines + line];
        du = (t == na - 1 ? z : fma(ea, du, z)) * q;
        const int64_t cu = u0 + (int64_t)t * sa;
        a.dst[cu] = fma(a.omega, du, src[cu]);
    }
}

hipError_t launch_bline(const BLineArgs &a, hipStream_t s)
{
    if (a.nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bline, dim3((a.nitems + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace bs
