// Host precompute of the exact line and plane block solves.
#pragma once

#include <vector>

#include "bs_internal.h"

namespace bs {

// Split of a line of n cells for preq chunks: chunk length Lr, chunk count P,
// last chunk length Llast.  False if Lr would exceed kMaxChunkLen.
bool line_split(int n, int preq, int &Lr, int &P, int &Llast);

// Line table (layout in bs_internal.h) for tridiag(-eps_a, d, -eps_a) of order n
// with dlo / dhi added to its first / last diagonal entry (extrapolated faces
// at the line's ends; zero for ghosts read as data).
std::vector<double> build_line_table(int n, double eps_a, double d, int preq, double dlo = 0.0, double dhi = 0.0);

// Orthonormal DST-I basis of order n, row-major n x n (symmetric, its own
// inverse): S[i][p] = sqrt(2/(n+1)) sin(pi (i+1)(p+1) / (n+1)).
std::vector<double> sine_basis(int n);

// Eigenvalues of tridiag(-eps, 2 eps, -eps) of order n, in the basis order:
// sigma_p = 4 eps sin^2((p+1) pi / (2(n+1))).
std::vector<long double> sine_eigenvalues(int n, double eps);

// Eigenbasis of the line block tridiag(-eps, 2 eps, -eps) of order n whose
// first (lo) and / or last (hi) diagonal entry is raised by eps (an
// extrapolated face at that end), row-major V[i][k] with orthonormal columns
// in the order of bc_sine_eigenvalues.  lo = hi = 0 is sine_basis (DST-I);
// lo = hi = 1 the DST-II basis sin(pi (k+1)(2i+1) / (2n)); one raised end the
// sines sin(2 pi (k+1) m / (2n+1)) with m = i+1 (hi) or n-i (lo).
std::vector<double> bc_sine_basis(int n, int lo, int hi);
std::vector<long double> bc_sine_eigenvalues(int n, double eps, int lo, int hi);

}  // namespace bs
