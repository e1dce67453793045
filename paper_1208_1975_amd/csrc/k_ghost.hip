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

// Two-ended (twisted) factorisation of each boundary line's block
// tridiag(-eps_a, d_t, -eps_a), d_t = 2(eps_x + eps_y + eps_z) plus eps_b for
// every extrapolated face next to the line (its whole length) and eps_a at an
// extrapolated end.  With the middle cell k = (na - 1) / 2, pivots are formed
// from the top for t < k (m_0 = d_0, m_t = d_t - eps_a^2 / m_{t-1}) and from
// the bottom for t > k (p_{na-1} = d_{na-1}, p_t = d_t - eps_a^2 / p_{t+1});
// the middle row then has gamma_k = d_k - eps_a^2 / m_{k-1} - eps_a^2 / p_{k+1}.
// Stored [t][line] like the scratch: row 2t the multiplier (eps_a / m_{t-1}
// above the middle, eps_a / p_{t+1} below it, 0 at the two ends and the
// middle), row 2t + 1 the reciprocal pivot (1 / m_t, 1 / p_t, 1 / gamma_k).
// They depend on eps and the faces only: formed once per patch set and axis.
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
    const int na = g.na, k = (na - 1) / 2;
    auto diag = [&](int t) { return dd + (t == 0 && g.lo_a ? ea : 0.0) + (t == na - 1 && g.hi_a ? ea : 0.0); };
    double m = 0.0, p = 0.0;
    for (int t = 0; t < k; ++t) {
        const double gm = t == 0 ? 0.0 : ea / m;
        m = fma(-ea, gm, diag(t));
        a.fac[(int64_t)(2 * t) * L + line] = gm;
        a.fac[(int64_t)(2 * t + 1) * L + line] = 1.0 / m;
    }
    for (int t = na - 1; t > k; --t) {
        const double hp = t == na - 1 ? 0.0 : ea / p;
        p = fma(-ea, hp, diag(t));
        a.fac[(int64_t)(2 * t) * L + line] = hp;
        a.fac[(int64_t)(2 * t + 1) * L + line] = 1.0 / p;
    }
    double gam = diag(k);
    if (k > 0) gam = fma(-ea, ea / m, gam);
    if (k < na - 1) gam = fma(-ea, ea / p, gam);
    a.fac[(int64_t)(2 * k) * L + line] = 0.0;
    a.fac[(int64_t)(2 * k + 1) * L + line] = 1.0 / gam;
}

// Two lanes per line (lanes 2l and 2l + 1 of a wavefront): lane 0 eliminates
// from the top towards the middle cell k, z_t = r_t + g_t z_{t-1} (t < k), lane
// 1 from the bottom, y_t = r_t + h_t y_{t+1} (t > k), in the same instruction
// stream (each walks max(k, na - 1 - k) steps of its own direction); the lanes
// exchange z_{k-1} / m_{k-1} and y_{k+1} / p_{k+1}, both form the middle value
// x_k = (r_k + eps_a z_{k-1} / m_{k-1} + eps_a y_{k+1} / p_{k+1}) / gamma_k, and
// each substitutes back along its half, x_t = (z_t + eps_a x_{t+1}) / m_t or
// (y_t + eps_a x_{t-1}) / p_t, writing dst = src + omega x.  The chains are
// half a line long and FMAs only; the loads of B cells are issued together
// before they are consumed.  In place (src == dst) every cell is read before
// it is written (each lane reads the old values of its own cells only; lane 0
// owns the middle cell).
__global__ void __launch_bounds__(256) k_bline(BLineArgs a)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int l = gid >> 1, side = gid & 1;
    const bool live = l < a.nitems;
    const int line = a.first + (live ? l : a.nitems - 1);   // both lanes of a pair run the exchange
    const BLineItem it = a.items[line];
    const PatchDesc *pd = a.pd + it.patch;
    const int ax = a.axis;
    const BLineGeo g = bline_geo(pd, it, ax);
    const double ea = pd->eps[ax];
    const int na = g.na, k = (na - 1) / 2;
    double *sc = a.scratch + line;
    const double *fc = a.fac + line;
    const int64_t L = a.nlines;
    // side 0: cells 0 .. k-1 (step +1); side 1: cells na-1 .. k+1 (step -1);
    // a pair past the last line (padding of the grid) steps nowhere and stores nothing
    const int nst = !live ? 0 : (side == 0 ? k : na - 1 - k);
    const int dir = side == 0 ? 1 : -1, tstart = side == 0 ? 0 : na - 1;
    const int nmax = na - 1 - k;   // >= k: the longer half
    constexpr int B = 16;
    double zprev = 0.0;
    for (int s0 = 0; s0 < nmax; s0 += B) {
        double rb[B], gb[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int s = s0 + j < nst ? s0 + j : (nst > 0 ? nst - 1 : 0);
            const int t = tstart + dir * s;
            rb[j] = sc[(int64_t)(2 * t + 1) * L];
            gb[j] = fc[(int64_t)(2 * t) * L];
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int s = s0 + j;
            if (s < nst) {
                const int t = tstart + dir * s;
                const double z = fma(gb[j], zprev, rb[j]);
                sc[(int64_t)(2 * t + 1) * L] = z;
                zprev = z;
            }
        }
    }
    // this lane's contribution to the middle row: eps_a z_{k-1} / m_{k-1}
    // (side 0) or eps_a y_{k+1} / p_{k+1} (side 1); 0 for an empty half
    const int tn = side == 0 ? k - 1 : k + 1;
    const double qn = nst > 0 ? fc[(int64_t)(2 * (nst > 0 ? tn : k) + 1) * L] : 0.0;
    const double mine = nst > 0 ? ea * zprev * qn : 0.0;
    const double other = __shfl_xor(mine, 1);
    const double rk = sc[(int64_t)(2 * k + 1) * L];
    const double gk = fc[(int64_t)(2 * k + 1) * L];
    const double x_mid = (rk + (side == 0 ? mine + other : other + mine)) * gk;
    if (!live) return;
    if (side == 0) {
        const int64_t cu = g.u0 + (int64_t)k * g.sa;
        a.dst[cu] = fma(a.omega, x_mid, a.src[cu]);
    }
    double x = x_mid;
    for (int s1 = nst - 1; s1 >= 0; s1 -= B) {
        // this batch's factors, eliminated right-hand sides and old values
        double qb[B], zb[B], ub[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int s = s1 - j >= 0 ? s1 - j : 0;
            const int t = tstart + dir * s;
            qb[j] = fc[(int64_t)(2 * t + 1) * L];
            zb[j] = sc[(int64_t)(2 * t + 1) * L];
            ub[j] = a.src[g.u0 + (int64_t)t * g.sa];
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int s = s1 - j;
            if (s >= 0) {
                const int t = tstart + dir * s;
                x = fma(ea, x, zb[j]) * qb[j];
                a.dst[g.u0 + (int64_t)t * g.sa] = fma(a.omega, x, ub[j]);
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
    hipLaunchKernelGGL(k_bline, dim3((2 * a.nitems + 255) / 256), dim3(256), 0, s, a);   // two lanes per line
    return hipGetLastError();
}

}  // namespace bs
