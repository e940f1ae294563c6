// Device side of the solvers' scalar steps: the finalize of a reduction runs
// the step of solver_ctl.h on the grand totals, and kernels test their
// predicate on the control block at the top.  Keeping the scalars on the
// device lets a whole iteration run without a host round trip.
#pragma once

#include "lqcd.h"
#include "lqcd_kernels.h"
#include "solver_ctl.h"

namespace lqcd {

template <int N>
__device__ inline void finalize(int fin, Ctl* c, const double (&v)[N])
{
    double t[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < N && j < 6; ++j) t[j] = v[j];
    finalize_totals(fin, c, t);
}

__device__ inline bool pred_skip(int pred, const Ctl* c)
{
    if (pred == PRED_ALWAYS || c == nullptr) return false;
    const int done = __hip_atomic_load(&c->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (done) return true;
    if (pred == PRED_UPDATE) return c->update == 0;
    if (pred == PRED_NO_UPDATE) return c->update != 0;
    return false;
}

}  // namespace lqcd
