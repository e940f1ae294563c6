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
// runs the solver's scalar step).  A step that would do nothing for every
// system (the reliable-update steps of an iteration that requested no update)
// is skipped with its barrier; every block takes that decision from the same
// control blocks after the same barrier, so all agree.
//
// Phases are separated by a grid barrier without read-modify-write atomics:
// block b stores the barrier's number into its arrival slot, block 0 waits
// for every arrival and stores the number into every release slot, and each
// block waits for its own.  Each block releases its writes with one
// agent-scope fence before it arrives and acquires the others' with one after
// it is released; the polls themselves are relaxed loads (an acquire load
// would invalidate the caches on every poll, which made a barrier of 512
// blocks cost tens of microseconds).  Every wait is bounded: it gives up
// after spin_limit polls, or at once when the host has set the give-up word
// or another block has given up, and records the failure so that every block
// leaves at its next barrier; every wave always reaches the end of the kernel.
//
// The grid never exceeds the blocks the device keeps resident at once (the
// launch is cooperative, so the runtime refuses a larger one), which the
// barrier needs, nor the largest phase (more blocks would only wait).
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

// Wait until *w holds `want` (relaxed polls).  Returns 0 when the host asked
// to give up, another block gave up, or after spin_limit polls.
__device__ int wait_word(const unsigned* w, unsigned want, const PProgram& P)
{
    for (int polls = 0; __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != want; ++polls) {
        if (polls >= P.spin_limit) return 0;
        if ((polls & 63) == 63 && (__hip_atomic_load(&P.flag[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                                   __hip_atomic_load(&P.flag[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0))
            return 0;
        __builtin_amdgcn_s_sleep(1);
    }
    return 1;
}

// Grid barrier number `epoch` (1, 2, ... within a launch; the slots start at
// zero).  A block's arrival slot holds epoch - 1 or epoch while block 0 waits
// on it, its release slot likewise.  Returns false when this or another block
// gave up (then the caller leaves the kernel).
__device__ bool grid_sync(const PProgram& P, unsigned epoch)
{
    __shared__ int ok;
    unsigned* arrive = P.bar;
    unsigned* release = P.bar + kMaxPersistBlocks;
    __syncthreads();
    int good = 1;
    if (threadIdx.x == 0) {
        if (__hip_atomic_load(&P.flag[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
            __hip_atomic_load(&P.flag[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
            good = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this block's writes, before its arrival
        __hip_atomic_store(arrive + blockIdx.x, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (blockIdx.x == 0) {
        int mine = 1;
        for (int b = threadIdx.x; b < (int)gridDim.x && mine; b += blockDim.x) mine = wait_word(arrive + b, epoch, P);
        mine = __syncthreads_and(mine);
        if (mine) {
            // every block's release happened before its arrival, which this
            // block has seen: pass it on to the release slots
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x)
                __hip_atomic_store(release + b, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (threadIdx.x == 0) good = good && mine;
    }
    if (threadIdx.x == 0) {
        if (good && blockIdx.x != 0) good = wait_word(release + blockIdx.x, epoch, P);
        if (!good) __hip_atomic_store(&P.flag[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the other blocks' writes
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

// True when some system's right-hand side is not skipped by predicate
// `pred` (the test every block routine and finalize applies per control
// block); read after a barrier, so all blocks agree.
__device__ bool any_active(const PProgram& P, int pred)
{
    const int n = P.nsys * P.nrhs;
    int act = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        act |= !pred_skip(pred, P.ctl + (i / P.nrhs) * P.ctl_stride + i % P.nrhs);
    return __syncthreads_or(act) != 0;
}

// Every system's every right-hand side done.
__device__ bool all_done(const PProgram& P)
{
    const int n = P.nsys * P.nrhs;
    int open = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        open |= __hip_atomic_load(&P.ctl[(i / P.nrhs) * P.ctl_stride + i % P.nrhs].done, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT) == 0;
    return __syncthreads_or(open) == 0;
}

// Blocks of kPersistThreads; the register budget of the FP64 hop (two
// waves per SIMD) bounds the whole kernel.
__global__ void __launch_bounds__(kPersistThreads) __attribute__((amdgpu_waves_per_eu(2)))
k_batch_persistent(const PProgram* __restrict__ prog)
{
    const PProgram& P = *prog;
    unsigned epoch = 0;
    for (int it = 0; it < P.max_iter; ++it) {
        // the reliable-update steps run only when some system requested an
        // update; requests come from a finalize, so a "no" holds until the
        // next finalize phase
        bool no_update = false;
        for (int k = 0; k < P.nsteps; ++k) {
            const PStep& st = P.step[k];
            if (st.pred == PRED_UPDATE) {
                if (!no_update) no_update = !any_active(P, PRED_UPDATE);
                if (no_update) continue;
            }
            run_step(st, P.nsys);
            if (!grid_sync(P, ++epoch)) return;
            if (st.nfin) {
                run_finalize(st, P.nsys, P.nrhs);
                if (!grid_sync(P, ++epoch)) return;
                no_update = false;
            }
        }
        if (all_done(P)) return;
    }
}

// The barrier slots to zero and the two flags to (give_up, 0): a kernel, so
// that a captured graph holds no memset node.
__global__ void k_persist_reset(unsigned* words, int nslots, int give_up)
{
    for (int i = (int)(blockIdx.x * blockDim.x + threadIdx.x); i < nslots + 2; i += (int)(gridDim.x * blockDim.x))
        words[i] = i < nslots ? 0u : (i == nslots ? (unsigned)give_up : 0u);
}

}  // namespace

hipError_t launch_persist_reset(unsigned* words, int nslots, int give_up, hipStream_t s)
{
    hipLaunchKernelGGL(k_persist_reset, dim3(16), dim3(256), 0, s, words, nslots, give_up);
    return hipGetLastError();
}

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
