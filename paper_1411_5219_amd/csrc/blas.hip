// Site-local kernels: the fused BLAS-1 steps of CGNR and BiCGStab with
// FP64 reductions, precision conversion, canonical <-> internal packing,
// and small utilities (zero fill, control-block set-up).
//
// Every kernel maps one work-item to one site of a parity field and walks
// that site's planes, so loads of one plane are coalesced across the
// wavefront and padding sites are never touched.
#include "lqcd.h"
#include "lqcd_device.h"
#include "lqcd_fin.h"
#include "lqcd_kernels.h"
#include "site_ops.h"

namespace lqcd {

template <int PREC, int KIND, int OP>
__global__ void __launch_bounds__(256) k_blas(const BlasArgs a)
{
    blas_block<PREC, KIND, OP>(a, blockIdx.x, gridDim.x, blockIdx.y);
}

template <int PREC, int KIND, int OP>
__global__ void __launch_bounds__(256) k_blas_batch(const BlasArgs* __restrict__ tab, const int* __restrict__ offs,
                                                   int nsys)
{
    const int x = blockIdx.x;
    int s = 0;
    while (s + 1 < nsys && x >= offs[s + 1]) ++s;
    const int bx = x - offs[s];
    if (bx >= tab[s].gx) return;  // padding of the system's range
    blas_block<PREC, KIND, OP>(tab[s], bx, tab[s].gx, blockIdx.y);
}

struct BlasLaunch {
    const BlasArgs* a;
    const BlasArgs* tab;
    const int* offs;
    int nsys;
};

template <int PREC, int KIND, int OP>
static hipError_t blas_one(const BlasLaunch& L, dim3 grid, dim3 block, hipStream_t s)
{
    if (L.tab) hipLaunchKernelGGL((k_blas_batch<PREC, KIND, OP>), grid, block, 0, s, L.tab, L.offs, L.nsys);
    else hipLaunchKernelGGL((k_blas<PREC, KIND, OP>), grid, block, 0, s, *L.a);
    return hipGetLastError();
}

#define LQCD_BLAS_CASE(OP) \
    case OP: return blas_one<PREC, KIND, OP>(L, grid, block, s);

// Spinor fields: every operation.
template <int PREC, int KIND>
static hipError_t blas_op(int op, const BlasLaunch& L, dim3 grid, dim3 block, hipStream_t s)
{
    if constexpr (KIND == KIND_SPINOR) {
        switch (op) {
            LQCD_BLAS_CASE(BLAS_CG_XR)
            LQCD_BLAS_CASE(BLAS_CG_P)
            LQCD_BLAS_CASE(BLAS_COPY)
            LQCD_BLAS_CASE(BLAS_ZERO)
            LQCD_BLAS_CASE(BLAS_SPIN_SCALE)
            LQCD_BLAS_CASE(BLAS_NORM)
            LQCD_BLAS_CASE(BLAS_BI_P)
            LQCD_BLAS_CASE(BLAS_BI_S)
            LQCD_BLAS_CASE(BLAS_BI_XR)
            LQCD_BLAS_CASE(BLAS_XPY)
            LQCD_BLAS_CASE(BLAS_NORM_DOT)
            LQCD_BLAS_CASE(BLAS_BL_U0)
            LQCD_BLAS_CASE(BLAS_BL_XR0)
            LQCD_BLAS_CASE(BLAS_BL_U01)
            LQCD_BLAS_CASE(BLAS_BL_XR01)
            LQCD_BLAS_CASE(BLAS_BL_GRAM)
            LQCD_BLAS_CASE(BLAS_BL_ORTH)
            LQCD_BLAS_CASE(BLAS_BL_MR)
        default: return hipErrorInvalidValue;
        }
    } else {
        // colour vectors: what the staggered CG and multi-shift CG use
        switch (op) {
            LQCD_BLAS_CASE(BLAS_CG_XR)
            LQCD_BLAS_CASE(BLAS_CG_P)
            LQCD_BLAS_CASE(BLAS_COPY)
            LQCD_BLAS_CASE(BLAS_ZERO)
            LQCD_BLAS_CASE(BLAS_SPIN_SCALE)
            LQCD_BLAS_CASE(BLAS_NORM)
            LQCD_BLAS_CASE(BLAS_XPY)
            LQCD_BLAS_CASE(BLAS_MS_AXPY)
            LQCD_BLAS_CASE(BLAS_MS_P)
            LQCD_BLAS_CASE(BLAS_AXMY_NORM)
        default: return hipErrorInvalidValue;
        }
    }
}
#undef LQCD_BLAS_CASE

static hipError_t blas_prec(int prec, int kind, int op, const BlasLaunch& L, dim3 grid, dim3 block, hipStream_t s)
{
    if (kind == KIND_SPINOR) {
        if (prec == 64) return blas_op<64, KIND_SPINOR>(op, L, grid, block, s);
        if (prec == 32) return blas_op<32, KIND_SPINOR>(op, L, grid, block, s);
        if (prec == 16) return blas_op<16, KIND_SPINOR>(op, L, grid, block, s);
    } else if (kind == KIND_COLOUR) {
        if (prec == 64) return blas_op<64, KIND_COLOUR>(op, L, grid, block, s);
        if (prec == 32) return blas_op<32, KIND_COLOUR>(op, L, grid, block, s);
    }
    return hipErrorInvalidValue;
}

hipError_t plan_blas(int prec, int op, const BlasArgs& a, int nrhs, const Launch& cfg, BlasPlan* out)
{
    if (prec != 64 && prec != 32 && prec != 16) return hipErrorInvalidValue;
    BlasPlan& p = *out;
    p.a = a;
    p.prec = prec;
    p.op = op;
    p.nrhs = nrhs;
    const int blk = cfg.block;
    const unsigned nbs = (unsigned)((a.Vh + blk - 1) / blk);
    p.grid = dim3(nbs * a.nsub, nrhs);
    p.a.gx = (int)p.grid.x;
    p.block = dim3(blk);
    p.nfin = (op == BLAS_CG_XR || op == BLAS_NORM || op == BLAS_AXMY_NORM)                       ? 1
             : (op == BLAS_BI_XR || op == BLAS_NORM_DOT || op == BLAS_BL_ORTH || op == BLAS_BL_MR) ? 3
             : op == BLAS_BL_GRAM                                                                 ? 5
                                                                                                  : 0;
    p.slots = (int)p.grid.x;
    if (p.nfin && p.slots > a.r.capacity) return hipErrorInvalidValue;  // partials too small
    return hipSuccess;
}

hipError_t exec_blas(const BlasPlan& p, hipStream_t s)
{
    BlasLaunch L{&p.a, nullptr, nullptr, 1};
    const hipError_t e = blas_prec(p.prec, p.a.kind, p.op, L, p.grid, p.block, s);
    if (e != hipSuccess || p.nfin == 0) return e;
    return launch_finalize(p.nfin, p.a.r.partials, p.slots, p.a.r.fin, p.a.ctl, p.a.pred, p.nrhs, s);
}

hipError_t exec_blas_batch(const BlasPlan* plans, int n, const BlasArgs* tab, const int* offs, int total_blocks,
                           const FinArgs* fin_tab, hipStream_t s)
{
    if (n < 1) return hipErrorInvalidValue;
    const BlasPlan& p0 = plans[0];
    BlasLaunch L{nullptr, tab, offs, n};
    const hipError_t e = blas_prec(p0.prec, p0.a.kind, p0.op, L, dim3((unsigned)total_blocks, p0.grid.y), p0.block, s);
    if (e != hipSuccess || p0.nfin == 0) return e;
    return launch_finalize_batch(p0.nfin, fin_tab, n, p0.nrhs, s);
}

hipError_t launch_blas(int prec, int op, const BlasArgs& a, int nrhs, const Launch& cfg, hipStream_t s)
{
    BlasPlan p;
    hipError_t e = plan_blas(prec, op, a, nrhs, cfg, &p);
    if (e != hipSuccess) return e;
    if (Recorder* r = active_recorder()) {
        r->steps.push_back(Step{});
        r->steps.back().kind = STEP_BLAS;
        r->steps.back().b = p;
        return hipSuccess;
    }
    return exec_blas(p, s);
}

thread_local Recorder* g_recorder = nullptr;
Recorder* active_recorder() { return g_recorder; }
void set_recorder(Recorder* r) { g_recorder = r; }

template <int N>
__global__ void __launch_bounds__(kFinThreads) k_finalize(const double* partials, int nblocks, int count, int fin,
                                                          Ctl* ctl, int pred)
{
    const int rhs = blockIdx.x;
    Ctl* c = ctl + rhs;
    if (pred_skip(pred, c)) return;
    double v[N];
    sum_partials<N>(partials + (int64_t)rhs * nblocks * N, count, v);
    __shared__ double tot[N];
    block_reduce_store<N>(v, tot, 0);
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[N];
#pragma unroll
        for (int j = 0; j < N; ++j) t[j] = tot[j];
        finalize<N>(fin, c, t);
    }
}

// One block per (system, right-hand side): the finalize of every system of a batched launch.
template <int N>
__global__ void __launch_bounds__(kFinThreads) k_finalize_batch(const FinArgs* __restrict__ tab, int nrhs)
{
    const FinArgs& f = tab[blockIdx.x / nrhs];
    const int rhs = blockIdx.x % nrhs;
    Ctl* c = f.ctl + rhs;
    if (pred_skip(f.pred, c)) return;
    double v[N];
    sum_partials<N>(f.partials + (int64_t)rhs * f.nblocks * N, f.nblocks, v);
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

hipError_t launch_finalize_batch(int N, const FinArgs* tab, int nsys, int nrhs, hipStream_t s)
{
    dim3 g((unsigned)(nsys * nrhs)), b(kFinThreads);
    if (N == 1) hipLaunchKernelGGL(k_finalize_batch<1>, g, b, 0, s, tab, nrhs);
    else if (N == 2) hipLaunchKernelGGL(k_finalize_batch<2>, g, b, 0, s, tab, nrhs);
    else if (N == 3) hipLaunchKernelGGL(k_finalize_batch<3>, g, b, 0, s, tab, nrhs);
    else if (N == 5) hipLaunchKernelGGL(k_finalize_batch<5>, g, b, 0, s, tab, nrhs);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_finalize(int N, const double* partials, int nblocks, int fin, Ctl* ctl, int pred, int nrhs,
                           hipStream_t s, int count)
{
    if (!ctl) return hipErrorInvalidValue;
    if (count < 0 || count > nblocks) count = nblocks;
    dim3 g(nrhs), b(kFinThreads);
    if (N == 1) hipLaunchKernelGGL(k_finalize<1>, g, b, 0, s, partials, nblocks, count, fin, ctl, pred);
    else if (N == 2) hipLaunchKernelGGL(k_finalize<2>, g, b, 0, s, partials, nblocks, count, fin, ctl, pred);
    else if (N == 3) hipLaunchKernelGGL(k_finalize<3>, g, b, 0, s, partials, nblocks, count, fin, ctl, pred);
    else if (N == 5) hipLaunchKernelGGL(k_finalize<5>, g, b, 0, s, partials, nblocks, count, fin, ctl, pred);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Precision conversion

template <int PD, int PS, bool ACC>
__global__ void __launch_bounds__(256) k_convert(const ConvertArgs a)
{
    convert_block<PD, PS, ACC>(a, blockIdx.x, gridDim.x, blockIdx.y);
}

template <int PD, int PS, bool ACC>
__global__ void __launch_bounds__(256) k_convert_batch(const ConvertArgs* __restrict__ tab,
                                                      const int* __restrict__ offs, int nsys)
{
    const int x = blockIdx.x;
    int s = 0;
    while (s + 1 < nsys && x >= offs[s + 1]) ++s;
    const int bx = x - offs[s];
    if (bx >= tab[s].gx) return;  // padding of the system's range
    convert_block<PD, PS, ACC>(tab[s], bx, tab[s].gx, blockIdx.y);
}

struct ConvertLaunch {
    const ConvertArgs* a;
    const ConvertArgs* tab;
    const int* offs;
    int nsys;
};

template <int PD, int PS, bool ACC>
static hipError_t convert_one(const ConvertLaunch& L, dim3 g, dim3 b, hipStream_t s)
{
    if (L.tab) hipLaunchKernelGGL((k_convert_batch<PD, PS, ACC>), g, b, 0, s, L.tab, L.offs, L.nsys);
    else hipLaunchKernelGGL((k_convert<PD, PS, ACC>), g, b, 0, s, *L.a);
    return hipGetLastError();
}

template <int PD, int PS>
static hipError_t convert2(bool acc, const ConvertLaunch& L, dim3 g, dim3 b, hipStream_t s)
{
    return acc ? convert_one<PD, PS, true>(L, g, b, s) : convert_one<PD, PS, false>(L, g, b, s);
}

static hipError_t convert_any(int pd, int ps, bool acc, const ConvertLaunch& L, dim3 g, dim3 b, hipStream_t s)
{
    if (acc && pd != 64) return hipErrorInvalidValue;
#define LQCD_CONV(D, S_)                               \
    if (pd == D && ps == S_) return convert2<D, S_>(acc, L, g, b, s);
    LQCD_CONV(64, 64)
    LQCD_CONV(64, 32)
    LQCD_CONV(64, 16)
    LQCD_CONV(32, 64)
    LQCD_CONV(32, 32)
    LQCD_CONV(32, 16)
    LQCD_CONV(16, 64)
    LQCD_CONV(16, 32)
    LQCD_CONV(16, 16)
#undef LQCD_CONV
    return hipErrorInvalidValue;
}

hipError_t plan_convert(int pd, int ps, const ConvertArgs& a, int nrhs, ConvertPlan* out)
{
    const int blk = 256;
    const unsigned nbs = (unsigned)((a.Vh + blk - 1) / blk);
    out->a = a;
    out->pd = pd;
    out->ps = ps;
    out->grid = dim3(nbs * a.nsub, nrhs);
    out->a.gx = (int)out->grid.x;
    out->block = dim3(blk);
    return hipSuccess;
}

hipError_t exec_convert(const ConvertPlan& p, hipStream_t s)
{
    ConvertLaunch L{&p.a, nullptr, nullptr, 1};
    return convert_any(p.pd, p.ps, p.a.accumulate != 0, L, p.grid, p.block, s);
}

hipError_t exec_convert_batch(const ConvertPlan* plans, int n, const ConvertArgs* tab, const int* offs,
                              int total_blocks, hipStream_t s)
{
    if (n < 1) return hipErrorInvalidValue;
    const ConvertPlan& p0 = plans[0];
    ConvertLaunch L{nullptr, tab, offs, n};
    return convert_any(p0.pd, p0.ps, p0.a.accumulate != 0, L, dim3((unsigned)total_blocks, p0.grid.y), p0.block, s);
}

hipError_t launch_convert(int pd, int ps, const ConvertArgs& a, int nrhs, hipStream_t s)
{
    ConvertPlan p;
    hipError_t e = plan_convert(pd, ps, a, nrhs, &p);
    if (e != hipSuccess) return e;
    if (Recorder* r = active_recorder()) {
        r->steps.push_back(Step{});
        r->steps.back().kind = STEP_CONVERT;
        r->steps.back().c = p;
        return hipSuccess;
    }
    return exec_convert(p, s);
}

// ---------------------------------------------------------------------------
// Canonical complex128 <-> internal layouts

__device__ __forceinline__ int64_t canonical_site(const Geom& g, int p, int64_t h)
{
    const int Lxh = g.Lxh;
    const int xh = (int)(h % Lxh);
    int64_t r = h / Lxh;
    const int y = (int)(r % g.L[1]);
    r /= g.L[1];
    const int z = (int)(r % g.L[2]);
    const int t = (int)(r / g.L[2]);
    const int x = 2 * xh + ((y + z + t + p) & 1);
    return x + (int64_t)g.L[0] * (y + (int64_t)g.L[1] * (z + (int64_t)g.L[2] * t));
}

// Canonical (V, NC) complex128 per right-hand side <-> internal parity
// fields of kind KIND (NC = 12 for spinors, 3 for colour vectors).
template <int PREC, int KIND, bool PACK>
__global__ void __launch_bounds__(256) k_pack_field(const Geom g, const double2* canon_c, double2* canon_m,
                                                    const char* in, char* out)
{
    using F = FieldIO<PREC, KIND>;
    using R = typename F::R;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int rhs = blockIdx.y;
    const int p = (int)(gid / g.Vh);
    const int64_t h = gid - (int64_t)p * g.Vh;
    if (p >= 2) return;
    const int64_t V = 2 * (int64_t)g.Vh;
    const int64_t i = canonical_site(g, p, h);
    const int64_t par_bytes = field_parity_bytes(KIND, PREC, g.S);
    const int64_t foff = (int64_t)rhs * 2 * par_bytes + p * par_bytes;
    typename F::Vec v;
    if (PACK) {
        const double2* c = canon_c + ((int64_t)rhs * V + i) * F::NC;
#pragma unroll
        for (int k = 0; k < F::NC; ++k) F::at(v, k) = {R(c[k].x), R(c[k].y)};
        F::store(out + foff, g.S, h, v);
    } else {
        F::load(in + foff, g.S, h, v);
        double2* c = canon_m + ((int64_t)rhs * V + i) * F::NC;
#pragma unroll
        for (int k = 0; k < F::NC; ++k) c[k] = make_double2((double)F::at(v, k).x, (double)F::at(v, k).y);
    }
}

template <int KIND>
static hipError_t pack_kind(int prec, bool pack, const Geom& g, const void* canon, const void* in, void* out, int nrhs,
                            hipStream_t s)
{
    dim3 b(256), gr((unsigned)((2 * (int64_t)g.Vh + 255) / 256), nrhs);
    const double2* cc = static_cast<const double2*>(canon);
    double2* cm = static_cast<double2*>(const_cast<void*>(canon));
    const char* i = static_cast<const char*>(in);
    char* o = static_cast<char*>(out);
#define LQCD_PACK(P)                                                                                         \
    if (prec == P) {                                                                                         \
        if (pack) hipLaunchKernelGGL((k_pack_field<P, KIND, true>), gr, b, 0, s, g, cc, nullptr, nullptr, o); \
        else hipLaunchKernelGGL((k_pack_field<P, KIND, false>), gr, b, 0, s, g, nullptr, cm, i, nullptr);    \
        return hipGetLastError();                                                                            \
    }
    LQCD_PACK(64)
    LQCD_PACK(32)
    LQCD_PACK(16)
#undef LQCD_PACK
    return hipErrorInvalidValue;
}

hipError_t launch_pack_spinor(int prec, const Geom& g, const void* canon, void* out, int nrhs, hipStream_t s)
{
    return pack_kind<KIND_SPINOR>(prec, true, g, canon, nullptr, out, nrhs, s);
}

hipError_t launch_unpack_spinor(int prec, const Geom& g, const void* in, void* canon, int nrhs, hipStream_t s)
{
    return pack_kind<KIND_SPINOR>(prec, false, g, canon, in, nullptr, nrhs, s);
}

hipError_t launch_pack_colour(int prec, const Geom& g, const void* canon, void* out, int nrhs, hipStream_t s)
{
    return pack_kind<KIND_COLOUR>(prec, true, g, canon, nullptr, out, nrhs, s);
}

hipError_t launch_unpack_colour(int prec, const Geom& g, const void* in, void* canon, int nrhs, hipStream_t s)
{
    return pack_kind<KIND_COLOUR>(prec, false, g, canon, in, nullptr, nrhs, s);
}

// Links into storage (PREC, RECON), from canonical complex128 (FROM_CANON)
// or from the internal FP64 field with SRC_RECON reals per link (a 12-real
// source has its third row rebuilt in FP64 first).
template <int PREC, int RECON, bool FROM_CANON, int SRC_RECON = 18>
__global__ void __launch_bounds__(256) k_pack_gauge(const Geom g, const double2* canon, const void* U64, void* out)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int blk = blockIdx.y;  // mu * 2 + parity
    const int mu = blk >> 1, p = blk & 1;
    if (gid >= g.Vh) return;
    const int64_t h = gid;
    Link<double> U;
    if (FROM_CANON) {
        const int64_t V = 2 * (int64_t)g.Vh;
        const int64_t i = canonical_site(g, p, h);
        const double2* c = canon + ((int64_t)mu * V + i) * 9;
#pragma unroll
        for (int k = 0; k < 9; ++k) U.u[k / 3][k % 3] = {c[k].x, c[k].y};
    } else {
        LinkIO<64, SRC_RECON>::load(U64, g.S, blk, h, U);
    }
    LinkIO<PREC, RECON>::store(out, g.S, blk, h, U);
}

template <bool FC, int SRC = 18>
static hipError_t pack_gauge_any(int prec, int recon, const Geom& g, const void* canon, const void* U64, void* out,
                                 hipStream_t s)
{
    dim3 b(256), gr((unsigned)((g.Vh + 255) / 256), 8);
    const double2* c = static_cast<const double2*>(canon);
    if (prec == 64 && recon == 18) hipLaunchKernelGGL((k_pack_gauge<64, 18, FC, SRC>), gr, b, 0, s, g, c, U64, out);
    else if (prec == 64 && recon == 12) hipLaunchKernelGGL((k_pack_gauge<64, 12, FC, SRC>), gr, b, 0, s, g, c, U64, out);
    else if (prec == 32 && recon == 18) hipLaunchKernelGGL((k_pack_gauge<32, 18, FC, SRC>), gr, b, 0, s, g, c, U64, out);
    else if (prec == 32 && recon == 12) hipLaunchKernelGGL((k_pack_gauge<32, 12, FC, SRC>), gr, b, 0, s, g, c, U64, out);
    else if (prec == 16 && recon == 12) hipLaunchKernelGGL((k_pack_gauge<16, 12, FC, SRC>), gr, b, 0, s, g, c, U64, out);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_pack_gauge(int prec, int recon, const Geom& g, const void* canon, void* out, hipStream_t s)
{
    return pack_gauge_any<true>(prec, recon, g, canon, nullptr, out, s);
}

hipError_t launch_convert_gauge(int prec, int recon, const Geom& g, const void* U64, int src_recon, void* out,
                                hipStream_t s)
{
    if (src_recon == 12) return pack_gauge_any<false, 12>(prec, recon, g, nullptr, U64, out, s);
    if (src_recon == 18) return pack_gauge_any<false, 18>(prec, recon, g, nullptr, U64, out, s);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------

__global__ void k_fill_zero(uint4* p, int64_t n16, unsigned char* tail, int ntail)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) p[i] = make_uint4(0u, 0u, 0u, 0u);
    if (i < ntail) tail[i] = 0;
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    const int64_t n16 = (int64_t)(bytes / 16);
    const int ntail = (int)(bytes - 16 * n16);
    const int64_t n = n16 > ntail ? n16 : ntail;
    dim3 b(256), g((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(k_fill_zero, g, b, 0, s, static_cast<uint4*>(p), n16,
                       static_cast<unsigned char*>(p) + 16 * n16, ntail);
    return hipGetLastError();
}

__global__ void k_ctl_init(Ctl* ctl, int nrhs, CtlInit in)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrhs) return;
    ctl[i] = ctl_make(in);
}

hipError_t launch_ctl_init(Ctl* ctl, int nrhs, const CtlInit& in, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_init, dim3((nrhs + 63) / 64), dim3(64), 0, s, ctl, nrhs, in);
    return hipGetLastError();
}

hipError_t launch_ctl_init(Ctl* ctl, int nrhs, double tol, double delta, int iter_limit, hipStream_t s)
{
    CtlInit in{};
    in.tol = tol;
    in.delta = delta;
    in.iter_limit = iter_limit;
    return launch_ctl_init(ctl, nrhs, in, s);
}

__global__ void k_ctl_init_shifts(Ctl* ctl, int n, int base, ShiftList shifts)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ctl[i].sigma = shifts.s[i] - shifts.s[base];
    ctl[i].ms_index = i;
    ctl[i].ms_n = n;
    ctl[i].ms_base = base;
}

hipError_t launch_ctl_init_shifts(Ctl* ctl, int n, int base, const ShiftList& shifts, hipStream_t s)
{
    if (n < 1 || n > kMaxShifts || base < 0 || base >= n) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ctl_init_shifts, dim3(1), dim3(64), 0, s, ctl, n, base, shifts);
    return hipGetLastError();
}

__global__ void k_ctl_reopen(Ctl* ctl, int nrhs, unsigned mask, int no_fallback)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrhs || !((mask >> i) & 1u)) return;
    ctl[i].done = 0;
    ctl[i].status = 0;
    ctl[i].update = 0;
    ctl[i].reset_p = 0;
    ctl[i].outer_req = 0;
    if (no_fallback) ctl[i].fallback_ok = 0;
}

hipError_t launch_ctl_reopen(Ctl* ctl, int nrhs, unsigned mask, hipStream_t s, bool no_fallback)
{
    hipLaunchKernelGGL(k_ctl_reopen, dim3((nrhs + 63) / 64), dim3(64), 0, s, ctl, nrhs, mask, no_fallback ? 1 : 0);
    return hipGetLastError();
}

}  // namespace lqcd
