// Host precompute of the exact line and plane block solves.
#pragma once

#include <vector>

#include "bs_internal.h"

namespace bs {

// Split of a line of n cells for preq chunks: chunk length Lr, chunk count P,
// last chunk length Llast.  False if Lr would exceed kMaxChunkLen.
bool line_split(int n, int preq, int &Lr, int &P, int &Llast);

// Line table (layout in bs_internal.h) for tridiag(-eps_a, d, -eps_a) of order n.
std::vector<double> build_line_table(int n, double eps_a, double d, int preq);

}  // namespace bs
