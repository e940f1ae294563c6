// Persistent batched solver: one cooperative launch runs every iteration of
// a batched CGNR (several lattices of different volumes, each with its own
// kappa, mu, links and right-hand sides) until all systems are done.
//
// The iteration is the one the batched launches replay (the steps recorded
// per system and their per-system argument tables, see BatchProgram in
// abi.cpp).  Here each step is a phase: the blocks of the grid stride over
// the step's blocks of all systems and run the same block routine the
// standalone kernel would (dslash_block, blas_block, convert_block); a step
// with a reduction is followed by its finalize as a phase of its own (one
// block per system and right-hand side sums the partials in block order and
// runs the solver's scalar step).  Phases are separated by a grid barrier:
// an agent-scope release of each block's writes, one arrival counter and a
// generation word, and an agent-scope acquire.  Every wait is bounded: a
// barrier gives up after spin_limit polls, or at once when the host has set
// the give-up word, and then records the failure so that every block leaves
// at its next barrier; every wave always reaches the end of the kernel.
//
// The grid never exceeds the blocks the device keeps resident at once (the
// launch is cooperative, so the runtime refuses a larger one), which the
// barrier needs.
#include "dslash_impl.h"
#include "site_ops.h"

namespace lqcd {

namespace {

// Block routines a phase may run (the ones of the mixed FP32/12-inner,
// FP64/18-outer CGNR iteration on several right-hand sides).
__device__ __forceinline__ void run_routine(int routine, const void* tab, int s, int bx, int by)
{
    switch (routine) {
#define LQCD_PHOP(ID, P, RC, DG, RD)                                                    \
    case ID: {                                                                          \
        const DslashArgs& a = static_cast<const DslashArgs*>(tab)[s];                   \
        if (bx < a.gx) dslash_block<P, RC, DG, RD, 1, false>(a, bx, a.gx, by);          \
        break;                                                                          \
    }
        LQCD_PHOP(PR_HOP32_12_D0_NONE, 32, 12, false, RED_NONE)
        LQCD_PHOP(PR_HOP32_12_D0_NORM, 32, 12, false, RED_NORM)
        LQCD_PHOP(PR_HOP32_12_D1_NONE, 32, 12, true, RED_NONE)
        LQCD_PHOP(PR_HOP32_12_D1_NORM, 32, 12, true, RED_NORM)
        // the FP64 hops of the reliable updates (a few per hundred iterations)
        // tip the kernel over 256 registers: they spill a little, the rest does not
        LQCD_PHOP(PR_HOP64_18_D0_NONE, 64, 18, false, RED_NONE)
        LQCD_PHOP(PR_HOP64_18_D0_NORM, 64, 18, false, RED_NORM)
#undef LQCD_PHOP
    case PR_BLAS32_CG_XR: {
        const BlasArgs& a = static_cast<const BlasArgs*>(tab)[s];
        if (bx < a.gx) blas_block<32, KIND_SPINOR, BLAS_CG_XR>(a, bx, a.gx, by);
        break;
    }
    case PR_BLAS32_CG_P: {
        const BlasArgs& a = static_cast<const BlasArgs*>(tab)[s];
        if (bx < a.gx) blas_block<32, KIND_SPINOR, BLAS_CG_P>(a, bx, a.gx, by);
        break;
    }
    case PR_CONV64_32_ACC: {
        const ConvertArgs& a = static_cast<const ConvertArgs*>(tab)[s];
        if (bx < a.gx) convert_block<64, 32, true>(a, bx, a.gx, by);
        break;
    }
    case PR_CONV32_64: {
        const ConvertArgs& a = static_cast<const ConvertArgs*>(tab)[s];
        if (bx < a.gx) convert_block<32, 64, false>(a, bx, a.gx, by);
        break;
    }
    default:
        break;
    }
}

// The blocks of one step: virtual block v = x + total * y over all systems.
__device__ void run_step(const PStep& st, int nsys)
{
    const int total = st.total * st.gy;
    for (int v = blockIdx.x; v < total; v += gridDim.x) {
        const int x = v % st.total, y = v / st.total;
        int s = 0;
        while (s + 1 < nsys && x >= st.offs[s + 1]) ++s;
        run_routine(st.routine, st.tab, s, x - st.offs[s], y);
        __syncthreads();  // the block reductions' LDS is reused by the next virtual block
    }
}

// Sum of one right-hand side's N partials in block order by the block's
// threads (strided), folded in LDS in thread order.
template <int N>
__device__ void finalize_one(const FinArgs& f, int rhs)
{
    Ctl* c = f.ctl + rhs;
    if (pred_skip(f.pred, c)) return;  // uniform over the block
    const double* p = f.partials + (int64_t)rhs * f.nblocks * N;
    double v[N];
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = 0.0;
    for (int b = threadIdx.x; b < f.nblocks; b += blockDim.x)
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] += p[(int64_t)b * N + j];
    __shared__ double tot[N];
    block_reduce_store<N>(v, tot, 0);
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[N];
#pragma unroll
        for (int j = 0; j < N; ++j) t[j] = tot[j];
        finalize<N>(f.fin, c, t);
    }
}

__device__ void run_finalize(const PStep& st, int nsys, int nrhs)
{
    for (int v = blockIdx.x; v < nsys * nrhs; v += gridDim.x) {
        const FinArgs& f = st.fin[v / nrhs];
        const int rhs = v % nrhs;
        if (st.nfin == 1) finalize_one<1>(f, rhs);
        else if (st.nfin == 2) finalize_one<2>(f, rhs);
        else finalize_one<3>(f, rhs);
        __syncthreads();
    }
}

// Grid barrier.  Returns false when this or another block gave up (then the
// caller leaves the kernel).
__device__ bool grid_sync(const PProgram& P)
{
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned* bar = P.bar;
        int* flag = P.flag;
        int good = 1;
        // a give-up request or an earlier failure: leave without arriving
        if (__hip_atomic_load(&flag[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
            __hip_atomic_load(&flag[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            good = 0;
        } else {
            __threadfence();  // release this block's writes to the other XCDs
            const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned arrived =
                __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
            if (arrived == gridDim.x) {
                __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&bar[1], gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                int polls = 0;
                while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                    if (__hip_atomic_load(&flag[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                        __hip_atomic_load(&flag[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                        ++polls > P.spin_limit) {
                        good = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
        }
        if (!good) __hip_atomic_store(&flag[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__hip_atomic_load(&flag[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) good = 0;
        __threadfence();  // acquire the other blocks' writes
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

// Every system's every right-hand side done (read after a barrier that
// follows the last write of a control block, so all blocks agree).
__device__ bool all_done(const PProgram& P)
{
    __shared__ int done;
    if (threadIdx.x == 0) {
        int d = 1;
        for (int s = 0; s < P.nsys && d; ++s)
            for (int r = 0; r < P.nrhs && d; ++r)
                d = __hip_atomic_load(&P.ctl[s * P.ctl_stride + r].done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        done = d;
    }
    __syncthreads();
    return done != 0;
}

// Blocks of kPersistThreads; the register budget of the FP64 hop (two
// waves per SIMD) bounds the whole kernel.
__global__ void __launch_bounds__(kPersistThreads) __attribute__((amdgpu_waves_per_eu(2)))
k_batch_persistent(const PProgram* __restrict__ prog)
{
    const PProgram& P = *prog;
    for (int it = 0; it < P.max_iter; ++it) {
        for (int k = 0; k < P.nsteps; ++k) {
            const PStep& st = P.step[k];
            run_step(st, P.nsys);
            if (!grid_sync(P)) return;
            if (st.nfin) {
                run_finalize(st, P.nsys, P.nrhs);
                if (!grid_sync(P)) return;
            }
        }
        if (all_done(P)) return;
    }
}

}  // namespace

hipError_t persistent_grid(int* blocks)
{
    int dev = 0, cus = 0, per_cu = 0, coop = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_batch_persistent),
                                                         kPersistThreads, 0);
    if (e != hipSuccess) return e;
    if (!coop || cus < 1 || per_cu < 1) return hipErrorNotSupported;
    *blocks = cus * per_cu;
    return hipSuccess;
}

hipError_t launch_batch_persistent(const PProgram* prog_dev, int blocks, hipStream_t s)
{
    void* args[] = {static_cast<void*>(&prog_dev)};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_batch_persistent), dim3((unsigned)blocks),
                                      dim3(kPersistThreads), args, 0, s);
}

}  // namespace lqcd
