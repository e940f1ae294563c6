// Host-side sizing of the chunks of iterations the solvers enqueue between
// status read-backs (plain arithmetic, no HIP): near convergence a chunk
// covers only the iterations the residual's rate of decrease says are left.
#pragma once

#include <algorithm>
#include <cmath>

namespace lqcd {

// Iterations a solve still needs for ||r||^2 to fall from rr to thresh, from
// two read-backs (||r||^2 = rr_prev after it_prev iterations, rr after it):
// 0 when rr is already at or below thresh, -1 when the two read-backs give no
// decrease to extrapolate (too few iterations between them, ||r||^2 not
// falling, values that are not positive).
inline int iterations_left(double rr_prev, int it_prev, double rr, int it, double thresh)
{
    if (!(thresh > 0.0) || !(rr > 0.0)) return -1;
    if (rr <= thresh) return 0;
    if (it_prev < 0 || it <= it_prev || !(rr_prev > 0.0)) return -1;
    const double rate = std::pow(rr / rr_prev, 1.0 / (it - it_prev));
    if (!(rate > 0.0 && rate < 1.0)) return -1;
    const double n = std::ceil(std::log(thresh / rr) / std::log(rate));
    return n < 1e6 ? (int)n : 1000000;
}

// Length of the next chunk: `need` iterations are still needed (-1:
// unknown) and `in_flight` are enqueued but not yet reported; at least one,
// at most `chunk`.
inline int next_chunk(int need, int in_flight, int chunk)
{
    if (need < 0) return chunk;
    return std::min(chunk, std::max(1, need - in_flight + 1));
}

}  // namespace lqcd
