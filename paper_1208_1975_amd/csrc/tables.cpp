// Host precompute of the exact block solves (section 2: the block inverse is
// formed once, before the smoothing iterations; section 4.3: for constant
// coefficients one set per block shape suffices).  Everything is computed in
// long double and rounded once to double.
#include "tables.h"

#include <cmath>
#include <stdexcept>
#include <vector>

namespace bs {

namespace {

using ld = long double;

// LU of the Toeplitz tridiagonal T = tridiag(-e, d, -e) of order len:
// pivots m_t (m_0 = d, m_t = d - e^2 / m_{t-1}).
std::vector<ld> pivots(int len, ld e, ld d)
{
    std::vector<ld> m(len);
    m[0] = d;
    for (int t = 1; t < len; ++t) m[t] = d - e * e / m[t - 1];
    return m;
}

// x = T^{-1} rhs for T of order len, with its pivots m.
std::vector<ld> tsolve(const std::vector<ld> &m, int len, ld e, std::vector<ld> rhs)
{
    for (int t = 1; t < len; ++t) rhs[t] += e / m[t - 1] * rhs[t - 1];
    rhs[len - 1] /= m[len - 1];
    for (int t = len - 2; t >= 0; --t) rhs[t] = (rhs[t] + e * rhs[t + 1]) / m[t];
    return rhs;
}

// In-place inverse of a dense n x n matrix (row-major) by Gauss-Jordan with
// partial pivoting.
void invert(std::vector<ld> &a, int n)
{
    std::vector<ld> inv(static_cast<size_t>(n) * n, 0.0L);
    for (int i = 0; i < n; ++i) inv[static_cast<size_t>(i) * n + i] = 1.0L;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(a[static_cast<size_t>(r) * n + c]) > std::fabs(a[static_cast<size_t>(piv) * n + c])) piv = r;
        if (a[static_cast<size_t>(piv) * n + c] == 0.0L) throw std::runtime_error("singular interface system");
        if (piv != c)
            for (int k = 0; k < n; ++k) {
                std::swap(a[static_cast<size_t>(piv) * n + k], a[static_cast<size_t>(c) * n + k]);
                std::swap(inv[static_cast<size_t>(piv) * n + k], inv[static_cast<size_t>(c) * n + k]);
            }
        const ld s = 1.0L / a[static_cast<size_t>(c) * n + c];
        for (int k = 0; k < n; ++k) {
            a[static_cast<size_t>(c) * n + k] *= s;
            inv[static_cast<size_t>(c) * n + k] *= s;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const ld fct = a[static_cast<size_t>(r) * n + c];
            if (fct == 0.0L) continue;
            for (int k = 0; k < n; ++k) {
                a[static_cast<size_t>(r) * n + k] -= fct * a[static_cast<size_t>(c) * n + k];
                inv[static_cast<size_t>(r) * n + k] -= fct * inv[static_cast<size_t>(c) * n + k];
            }
        }
    }
    a.swap(inv);
}

}  // namespace

bool line_split(int n, int preq, int &Lr, int &P, int &Llast)
{
    if (n < 1 || preq < 1) return false;
    Lr = (n + preq - 1) / preq;
    if (Lr > kMaxChunkLen) return false;
    P = (n + Lr - 1) / Lr;
    Llast = n - (P - 1) * Lr;
    return true;
}

std::vector<double> build_line_table(int n, double eps_a, double d, int preq, double dlo, double dhi)
{
    int Lr, P, Llast;
    if (!line_split(n, preq, Lr, P, Llast)) throw std::runtime_error("line split");
    const ld e = eps_a, dd = d;
    std::vector<double> out(static_cast<size_t>(line_table_size(Lr, P)), 0.0);
    std::vector<ld> m = pivots(Lr, e, dd);
    if (P == 1 && (dlo != 0.0 || dhi != 0.0)) {
        // one chunk: the exact LU factors of the line's own matrix, whose end
        // diagonals carry the extrapolated faces (no interface coupling)
        std::vector<ld> dg(n, dd);
        dg[0] += dlo;
        dg[n - 1] += dhi;
        m[0] = dg[0];
        for (int t = 1; t < n; ++t) m[t] = dg[t] - e * e / m[t - 1];
    }
    out[0] = 0.0;
    for (int t = 1; t < Lr; ++t) out[t] = static_cast<double>(e / m[t - 1]);
    for (int t = 0; t < Lr; ++t) out[Lr + t] = static_cast<double>(1.0L / m[t]);

    // spikes of a chunk of length len: eps_a T^{-1} e_0 and eps_a T^{-1} e_{len-1}
    auto spikes = [&](int len, std::vector<ld> &ev, std::vector<ld> &ew) {
        std::vector<ld> e0(len, 0.0L), el(len, 0.0L);
        e0[0] = 1.0L;
        el[len - 1] = 1.0L;
        ev = tsolve(m, len, e, e0);
        ew = tsolve(m, len, e, el);
        for (auto &v : ev) v *= e;
        for (auto &v : ew) v *= e;
    };
    std::vector<ld> evF, ewF, evT, ewT;
    spikes(Lr, evF, ewF);
    spikes(Llast, evT, ewT);
    for (int t = 0; t < Lr; ++t) {
        out[2 * Lr + t] = static_cast<double>(evF[t]);
        out[3 * Lr + t] = static_cast<double>(ewF[t]);
    }
    for (int t = 0; t < Llast; ++t) {
        out[4 * Lr + t] = static_cast<double>(evT[t]);
        out[5 * Lr + t] = static_cast<double>(ewT[t]);
    }

    // Interface system over z = (alpha_0, beta_0, ..., alpha_{P-1}, beta_{P-1}),
    // alpha_p / beta_p = correction at the first / last cell of chunk p:
    //   alpha_p - beta_{p-1} ev_p[0]      - alpha_{p+1} ew_p[0]      = y_p[0]
    //   beta_p  - beta_{p-1} ev_p[last]   - alpha_{p+1} ew_p[last]   = y_p[last]
    const int N = 2 * P;
    std::vector<ld> S(static_cast<size_t>(N) * N, 0.0L);
    for (int p = 0; p < P; ++p) {
        const bool lastc = (p == P - 1);
        const std::vector<ld> &ev = lastc ? evT : evF;
        const std::vector<ld> &ew = lastc ? ewT : ewF;
        const int len = lastc ? Llast : Lr;
        const int ra = 2 * p, rb = 2 * p + 1;
        S[static_cast<size_t>(ra) * N + ra] = 1.0L;
        S[static_cast<size_t>(rb) * N + rb] = 1.0L;
        if (p > 0) {
            S[static_cast<size_t>(ra) * N + (2 * p - 1)] -= ev[0];
            S[static_cast<size_t>(rb) * N + (2 * p - 1)] -= ev[len - 1];
        }
        if (p < P - 1) {
            S[static_cast<size_t>(ra) * N + (2 * p + 2)] -= ew[0];
            S[static_cast<size_t>(rb) * N + (2 * p + 2)] -= ew[len - 1];
        }
    }
    // Extrapolated ends (P > 1): the line matrix is the Toeplitz one plus dlo
    // at its first and dhi at its last diagonal entry.  Chunk 0 then solves
    // T x = r - dlo x_0 e_0 (+ the coupling to chunk 1), i.e. it takes the
    // spike ev with the coefficient beta_prev = -(dlo / eps_a) alpha_0, as if
    // a previous chunk ended in that value; likewise the last chunk takes ew
    // with alpha_next = -(dhi / eps_a) beta_{P-1}.  The interface rows gain
    // those terms, and the rows of the inverse that give beta_prev for chunk
    // 0 and alpha_next for the last chunk are the scaled rows of alpha_0 and
    // beta_{P-1}: an exact reformulation, with kernels unchanged.
    if (P > 1 && dlo != 0.0) {
        const ld c = static_cast<ld>(dlo) / e;
        S[0 * static_cast<size_t>(N) + 0] += c * evF[0];
        S[1 * static_cast<size_t>(N) + 0] += c * evF[Lr - 1];
    }
    if (P > 1 && dhi != 0.0) {
        const ld c = static_cast<ld>(dhi) / e;
        const int ra = 2 * (P - 1), rb = ra + 1;
        S[static_cast<size_t>(ra) * N + rb] += c * ewT[0];
        S[static_cast<size_t>(rb) * N + rb] += c * ewT[Llast - 1];
    }
    invert(S, N);
    const size_t kb = 6 * static_cast<size_t>(Lr), ka = kb + 2 * static_cast<size_t>(P) * P;
    for (int p = 0; p < P; ++p)
        for (int jj = 0; jj < N; ++jj) {
            if (p > 0) out[kb + static_cast<size_t>(p) * N + jj] = static_cast<double>(S[static_cast<size_t>(2 * p - 1) * N + jj]);
            if (p < P - 1) out[ka + static_cast<size_t>(p) * N + jj] = static_cast<double>(S[static_cast<size_t>(2 * p + 2) * N + jj]);
        }
    if (P > 1 && dlo != 0.0)
        for (int jj = 0; jj < N; ++jj)
            out[kb + jj] = static_cast<double>(-(static_cast<ld>(dlo) / e) * S[jj]);
    if (P > 1 && dhi != 0.0)
        for (int jj = 0; jj < N; ++jj)
            out[ka + static_cast<size_t>(P - 1) * N + jj] =
                static_cast<double>(-(static_cast<ld>(dhi) / e) * S[static_cast<size_t>(2 * P - 1) * N + jj]);
    return out;
}

std::vector<double> sine_basis(int n)
{
    std::vector<double> S(static_cast<size_t>(n) * n);
    const ld scale = std::sqrt(2.0L / static_cast<ld>(n + 1));
    const ld pi = 3.141592653589793238462643383279502884L;
    const long period = 2L * (n + 1);
    for (int i = 0; i < n; ++i)
        for (int p = 0; p < n; ++p) {
            // reduce the argument in integers before the library sine
            const long m = (static_cast<long>(i + 1) * (p + 1)) % period;
            S[static_cast<size_t>(i) * n + p] = static_cast<double>(scale * std::sin(pi * m / (n + 1)));
        }
    return S;
}

std::vector<long double> sine_eigenvalues(int n, double eps)
{
    std::vector<long double> sg(n);
    const ld pi = 3.141592653589793238462643383279502884L;
    for (int p = 0; p < n; ++p) {
        const ld s = std::sin(pi * (p + 1) / (2.0L * (n + 1)));
        sg[p] = 4.0L * eps * s * s;
    }
    return sg;
}

std::vector<double> bc_sine_basis(int n, int lo, int hi)
{
    if (!lo && !hi) return sine_basis(n);
    const ld pi = 3.141592653589793238462643383279502884L;
    // angle = pi * m / den, m reduced in integers modulo 2 den
    const long den = (lo && hi) ? 2L * n : 2L * n + 1;
    std::vector<ld> V(static_cast<size_t>(n) * n);
    for (int k = 0; k < n; ++k) {
        ld ss = 0.0L;
        for (int i = 0; i < n; ++i) {
            long m;
            if (lo && hi)
                m = static_cast<long>(k + 1) * (2 * i + 1);
            else
                m = 2L * (k + 1) * (hi ? i + 1 : n - i);
            m %= 2 * den;
            const ld v = std::sin(pi * static_cast<ld>(m) / static_cast<ld>(den));
            V[static_cast<size_t>(i) * n + k] = v;
            ss += v * v;
        }
        const ld sc = 1.0L / std::sqrt(ss);
        for (int i = 0; i < n; ++i) V[static_cast<size_t>(i) * n + k] *= sc;
    }
    return std::vector<double>(V.begin(), V.end());
}

std::vector<long double> bc_sine_eigenvalues(int n, double eps, int lo, int hi)
{
    if (!lo && !hi) return sine_eigenvalues(n, eps);
    const ld pi = 3.141592653589793238462643383279502884L;
    const ld den = (lo && hi) ? 2.0L * n : 2.0L * n + 1.0L;
    std::vector<long double> sg(n);
    for (int k = 0; k < n; ++k) {
        const ld s = std::sin(pi * (k + 1) / den);
        sg[k] = 4.0L * eps * s * s;
    }
    return sg;
}

}  // namespace bs
