// Even-odd Wilson / twisted-mass Dslash for gfx950 (kernel templates; each
// storage precision is instantiated in its own translation unit).
//
// One work-item per output site of parity p.  For each of the 8 hops it
// loads the neighbour spinor of parity 1-p, projects it to a 2x3 half
// spinor with (1 -+ gamma_mu), multiplies by the link (or its adjoint),
// applies the boundary phase on hops that cross the boundary, and rebuilds
// the lower spin components from the upper ones.  The site-diagonal
// twisted-mass terms are fused into the store (out = add + a*site + c*hop)
// together with FP64 reductions, so a Schur-complement application or a
// residual never needs a separate vector pass.
//
// In the chiral basis gamma_mu = [[0, B_mu], [B_mu^+, 0]] with
//   B_x = -i sigma_1, B_y = -i sigma_2, B_z = -i sigma_3, B_t = 1,
// so (1 - s gamma_mu) psi = (h ; -s B_mu^+ h) with h = psi_up - s B_mu psi_lo;
// only h is multiplied by the link.
#pragma once

#include "block_order.h"
#include "lqcd.h"
#include "lqcd_device.h"
#include "lqcd_fin.h"
#include "lqcd_kernels.h"

namespace lqcd {

// h = u - SIG * B_MU l   (u = spins 0,1; l = spins 2,3)
template <class R, int MU, int SIG>
__device__ __forceinline__ void project(const Spinor<R>& p, cplx<R> (&h)[2][3])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cplx<R> u0 = p.s[0][c], u1 = p.s[1][c], l0 = p.s[2][c], l1 = p.s[3][c];
        cplx<R> b0, b1;
        if (MU == 0) { b0 = mti(l1); b1 = mti(l0); }        // -i sigma_1
        else if (MU == 1) { b0 = -l1; b1 = l0; }            // -i sigma_2
        else if (MU == 2) { b0 = mti(l0); b1 = ti(l1); }    // -i sigma_3
        else { b0 = l0; b1 = l1; }                          // 1
        if (SIG > 0) { h[0][c] = u0 - b0; h[1][c] = u1 - b1; }
        else { h[0][c] = u0 + b0; h[1][c] = u1 + b1; }
    }
}

// acc += (w ; -SIG * B_MU^+ w)
template <class R, int MU, int SIG>
__device__ __forceinline__ void accumulate(Spinor<R>& acc, const cplx<R> (&w)[2][3])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cplx<R> w0 = w[0][c], w1 = w[1][c];
        acc.s[0][c] = acc.s[0][c] + w0;
        acc.s[1][c] = acc.s[1][c] + w1;
        cplx<R> d0, d1;  // B^+ w
        if (MU == 0) { d0 = ti(w1); d1 = ti(w0); }          // i sigma_1
        else if (MU == 1) { d0 = w1; d1 = -w0; }            // i sigma_2
        else if (MU == 2) { d0 = ti(w0); d1 = mti(w1); }    // i sigma_3
        else { d0 = w0; d1 = w1; }
        if (SIG > 0) { acc.s[2][c] = acc.s[2][c] - d0; acc.s[3][c] = acc.s[3][c] - d1; }
        else { acc.s[2][c] = acc.s[2][c] + d0; acc.s[3][c] = acc.s[3][c] + d1; }
    }
}

// w = U h (ADJ = false) or U^+ h (ADJ = true), on both spin components.
template <class R, bool ADJ>
__device__ __forceinline__ void link_mul(const Link<R>& U, const cplx<R> (&h)[2][3], cplx<R> (&w)[2][3])
{
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) w[s][a] = su3_row<R, ADJ>(U.u, a, h[s]);
}

template <class R>
__device__ __forceinline__ void phase_mul(cplx<R> (&w)[2][3], cplx<R> ph)
{
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) w[s][a] = ph * w[s][a];
}

// Operands of one hop for a tile of NR right-hand sides: the link (loaded
// once for the tile) and the neighbour spinor of each right-hand side.
template <int PREC, int NR>
struct HopBuf {
    Link<typename SpinorIO<PREC>::R> L;
    Spinor<typename SpinorIO<PREC>::R> p[NR];
};

// LNT selects the streaming (non-temporal) cache policy for the link loads,
// for launches in which no other block reads the same links.  A tile of one
// right-hand side is active whenever its block runs, so NR = 1 carries no
// per-hop branch that would keep the loads of consecutive hops apart.
template <int PREC, int RECON, int NR, bool LNT>
__device__ __forceinline__ void hop_load(const char* const (&in)[NR], const bool (&act)[NR], const void* U,
                                         int64_t S, const Nbr& n, HopBuf<PREC, NR>& b, uint32_t xo, int64_t span)
{
    if constexpr (LNT) LinkIO<PREC, RECON>::template load<>(U, S, n.lblk, n.lsite, b.L);
    else LinkIO<PREC, RECON>::template load<0>(U, S, n.lblk, n.lsite, b.L);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (NR > 1 && !act[r]) continue;
        SpinorIO<PREC>::load(in[r], S, n.nb, b.p[r], xo, span);
    }
}

template <int PREC, int MU, bool FWD, int SIG, int NR>
__device__ __forceinline__ void hop_apply(const HopBuf<PREC, NR>& b, const bool (&act)[NR], bool cross,
                                          cplx<typename SpinorIO<PREC>::R> ph,
                                          Spinor<typename SpinorIO<PREC>::R> (&acc)[NR])
{
    using R = typename SpinorIO<PREC>::R;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (NR > 1 && !act[r]) continue;
        cplx<R> h[2][3];
        project<R, MU, SIG>(b.p[r], h);
        cplx<R> w[2][3];
        link_mul<R, !FWD>(b.L, h, w);
        if (cross) phase_mul(w, FWD ? ph : conj(ph));
        accumulate<R, MU, SIG>(acc[r], w);
    }
}

// One hop applied right after its loads (pipeline depth 1).  With one
// right-hand side the neighbour spinor is loaded and projected to its half
// spinor before the link is loaded, so the full spinor and the link are not
// live together; a tile of several right-hand sides loads the link first and
// then each neighbour spinor in turn.
template <int PREC, int RECON, int MU, bool FWD, int SIG, int NR, bool LNT>
__device__ __forceinline__ void hop_fused(const char* const (&in)[NR], const bool (&act)[NR], const void* U,
                                          int64_t S, const Nbr& n, cplx<typename SpinorIO<PREC>::R> ph,
                                          Spinor<typename SpinorIO<PREC>::R> (&acc)[NR], uint32_t xo, int64_t span)
{
    using R = typename SpinorIO<PREC>::R;
    if constexpr (NR == 1) {
        Spinor<R> p;
        SpinorIO<PREC>::load(in[0], S, n.nb, p, xo, span);
        cplx<R> h[2][3];
        project<R, MU, SIG>(p, h);
        Link<R> L;
        if constexpr (LNT) LinkIO<PREC, RECON>::template load<>(U, S, n.lblk, n.lsite, L);
        else LinkIO<PREC, RECON>::template load<0>(U, S, n.lblk, n.lsite, L);
        cplx<R> w[2][3];
        link_mul<R, !FWD>(L, h, w);
        if (n.cross) phase_mul(w, FWD ? ph : conj(ph));
        accumulate<R, MU, SIG>(acc[0], w);
        return;
    }
    Link<R> L;
    if constexpr (LNT) LinkIO<PREC, RECON>::template load<>(U, S, n.lblk, n.lsite, L);
    else LinkIO<PREC, RECON>::template load<0>(U, S, n.lblk, n.lsite, L);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (NR > 1 && !act[r]) continue;
        Spinor<R> p;
        SpinorIO<PREC>::load(in[r], S, n.nb, p, xo, span);
        cplx<R> h[2][3];
        project<R, MU, SIG>(p, h);
        cplx<R> w[2][3];
        link_mul<R, !FWD>(L, h, w);
        if (n.cross) phase_mul(w, FWD ? ph : conj(ph));
        accumulate<R, MU, SIG>(acc[r], w);
    }
}

// Per storage precision: waves per SIMD the register allocation must allow
// (a block of 256 is one wave on each of a compute unit's four SIMDs), and
// the depth of the software pipeline over the eight hops (the loads of hop
// K + depth are issued right after hop K has been applied).  FP64 holds 84
// registers of operands per hop and already needs about 250 registers for
// two waves per SIMD with one hop in flight; FP32 and FP16 keep three waves
// with two hops in flight.
#ifndef LQCD_DEPTH_64
#define LQCD_DEPTH_64 1
#endif
#ifndef LQCD_DEPTH_32
#define LQCD_DEPTH_32 2
#endif
#ifndef LQCD_DEPTH_16
#define LQCD_DEPTH_16 2
#endif

// Tiles of several right-hand sides hold NR accumulators and run at depth 1
// with the register count the compiler chooses.
template <int PREC, int NR>
struct HopTune {
    static constexpr int waves = NR > 1 ? 1 : hop_waves(PREC);
    static constexpr int depth = NR > 1 ? 1 : PREC == 64 ? LQCD_DEPTH_64 : PREC == 32 ? LQCD_DEPTH_32 : LQCD_DEPTH_16;
    static_assert(depth >= 1 && depth <= 4, "hop pipeline depth 1..4");
    static_assert(waves >= 1 && waves <= 8, "waves per SIMD 1..8");
};

// Largest block of a hop launch: 256 work-items, or for the tile-1 launches
// with cached links (right-hand sides across lanes: up to 16 lanes per site
// and whole x-rows per block) one block per compute unit at the kernel's
// waves per SIMD: 8 waves in FP64, 12 in FP32 and FP16.
template <int PREC, int NR, bool LNT>
struct HopBlock {
    static constexpr int max_threads = (NR == 1 && !LNT) ? hop_lane_block_limit(PREC) : 256;
};

template <int PREC, int RECON, int NR, bool LNT, int SF, int D>
struct HopPipe {
    using R = typename SpinorIO<PREC>::R;
    const char* const (&in)[NR];
    const bool (&act)[NR];
    const void* U;
    int64_t S;
    const SiteGeo& g;
    const cplx<R> (&ph)[4];
    Spinor<R> (&acc)[NR];
    uint32_t xo;      // per-lane byte offset of the input field (right-hand sides across lanes)
    int64_t span;     // bytes the input buffer resource covers (0: one field)
    HopBuf<PREC, NR> buf[D > 1 ? D : 1];

    template <int K>
    __device__ __forceinline__ void load()
    {
        hop_load<PREC, RECON, NR, LNT>(in, act, U, S, g.template get<K>(), buf[K % D], xo, span);
    }
    template <int K>
    __device__ __forceinline__ void step()
    {
        constexpr int MU = K >> 1;
        constexpr bool FWD = (K & 1) == 0;
        hop_apply<PREC, MU, FWD, FWD ? SF : -SF, NR>(buf[K % D], act, g.template get<K>().cross, ph[MU], acc);
        if constexpr (K + D < 8) load<K + D>();
    }
    template <int K>
    __device__ __forceinline__ void fused()
    {
        constexpr int MU = K >> 1;
        constexpr bool FWD = (K & 1) == 0;
        hop_fused<PREC, RECON, MU, FWD, FWD ? SF : -SF, NR, LNT>(in, act, U, S, g.template get<K>(), ph[MU], acc,
                                                                 xo, span);
    }
    __device__ __forceinline__ void run()
    {
        if constexpr (D == 1) {
            fused<0>();
            fused<1>();
            fused<2>();
            fused<3>();
            fused<4>();
            fused<5>();
            fused<6>();
            fused<7>();
            return;
        }
        load<0>();
        if constexpr (D > 1) load<1>();
        if constexpr (D > 2) load<2>();
        if constexpr (D > 3) load<3>();
        step<0>();
        step<1>();
        step<2>();
        step<3>();
        step<4>();
        step<5>();
        step<6>();
        step<7>();
    }
};

template <int RED>
struct RedN {
    static constexpr int N = RED == RED_NONE ? 1 : RED == RED_NORM ? 1 : RED == RED_DOT_AUX ? 2 : 3;
};

// Block part of the reductions of a right-hand-side tile: NR x N sums per
// work-item, folded per wavefront and over waves in wave order; thread 0
// writes partials[rhs][bid][j] for each right-hand side of the tile.
template <int NR, int N>
__device__ void block_reduce_tile(double (&v)[NR][N], double* partials, int nb, int rhs0, int nrhs, int bid)
{
    __shared__ double sm[NR * N][16];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int j = 0; j < N; ++j) v[r][j] += __shfl_xor(v[r][j], off, 64);
    if (lane == 0)
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int j = 0; j < N; ++j) sm[r * N + j][wave] = v[r][j];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int r = 0; r < NR; ++r) {
            if (rhs0 + r >= nrhs) break;
            double* out = partials + ((int64_t)(rhs0 + r) * nb + bid) * N;
            for (int j = 0; j < N; ++j) {
                double s = 0.0;
                for (int w = 0; w < nwaves; ++w) s += sm[r * N + j][w];
                out[j] = s;
            }
        }
    }
}

// Block part of the reductions with right-hand sides across L lanes (L a
// power of two up to 64; L = 1 is one right-hand side per block): lanes with
// the same right-hand side (equal lane index mod L) fold their N sums per
// wavefront, the waves are combined in LDS in wave order, and work-item r < L
// writes partials[rhs0 + r][bid][j].  Blocks of up to 16 waves.
template <int N>
__device__ void block_reduce_lanes(double (&v)[N], double* partials, int nb, int rhs0, int L, int nrhs, int bid)
{
    __shared__ double sm[N][16][16];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    for (int off = 32; off >= L; off >>= 1)
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] += __shfl_xor(v[j], off, 64);
    if (lane < L)
#pragma unroll
        for (int j = 0; j < N; ++j) sm[j][wave][lane] = v[j];
    __syncthreads();
    const int r = threadIdx.x;
    if (r < L && rhs0 + r < nrhs) {
        double* out = partials + ((int64_t)(rhs0 + r) * nb + bid) * N;
        for (int j = 0; j < N; ++j) {
            double s = 0.0;
            for (int w = 0; w < nwaves; ++w) s += sm[j][w][r];
            out[j] = s;
        }
    }
}

// The work of one block: block bx of nbx along x and by along y of the
// launch that serves this set of arguments.
template <int PREC, int RECON, bool DAG, int RED, int NR, bool LNT>
__device__ __forceinline__ void dslash_block(const DslashArgs& a, int bx, int nbx, int by)
{
    using R = typename SpinorIO<PREC>::R;
    constexpr int N = RedN<RED>::N;
    // right-hand sides across lanes: the tile-1 launches with cached links
    constexpr bool kLanes = NR == 1 && !LNT;
    const int L = kLanes ? a.lanes : 1;
    const int lr = kLanes ? (int)(threadIdx.x & (unsigned)(L - 1)) : 0;
    const int tid = kLanes ? (int)(threadIdx.x >> a.lanes_log2) : (int)threadIdx.x;
    const BlockPos bp = block_pos(a, bx, nbx, by);
    const int p = bp.p, tile = bp.tile;
    const int rhs0 = tile * NR * L;  // first right-hand side of the block's tile (uniform)
    bool act[NR];
    bool any = false;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int rr = rhs0 + lr + r;
        act[r] = tile < a.ntiles && rr < a.nrhs && !pred_skip(a.pred, a.ctl ? a.ctl + rr : nullptr);
        any = any || act[r];
    }
    if (L == 1 && !any) return;  // uniform over the block unless the right-hand sides are across lanes
    const SitePos sp = site_pos(a, bp.bid, p, tid);
    const int h = sp.h;
    const int64_t poff = bp.poff, ioff = bp.ioff;
    const int64_t S = a.g.S;
    // per-lane offsets and buffer spans of the fields (right-hand side rhs0 + lr)
    const bool wide = L > 1;
    const uint32_t xo_in = (uint32_t)(lr * a.st_in), xo_out = (uint32_t)(lr * a.st_out);
    const uint32_t xo_site = (uint32_t)(lr * a.st_site), xo_add = (uint32_t)(lr * a.st_add);
    const uint32_t xo_aux = (uint32_t)(lr * a.st_aux);
    const int64_t sp_in = wide ? L * a.st_in : 0, sp_out = wide ? L * a.st_out : 0;
    const int64_t sp_site = wide ? L * a.st_site : 0, sp_add = wide ? L * a.st_add : 0;
    const int64_t sp_aux = wide ? L * a.st_aux : 0;

    double tot[NR][N];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int j = 0; j < N; ++j) tot[r][j] = 0.0;

    if (sp.valid && any) {
        const char* in[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) in[r] = static_cast<const char*>(a.in) + (int64_t)(rhs0 + r) * a.st_in + ioff;
        constexpr int SF = DAG ? -1 : 1;  // projector sign of forward hops: (1 - SF gamma)
        Spinor<R> acc[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[r].s[s][c] = {R(0), R(0)};

        const cplx<R> ph[4] = {{R(a.g.ph[0][0]), R(a.g.ph[0][1])},
                               {R(a.g.ph[1][0]), R(a.g.ph[1][1])},
                               {R(a.g.ph[2][0]), R(a.g.ph[2][1])},
                               {R(a.g.ph[3][0]), R(a.g.ph[3][1])}};
        const SiteGeo geo = site_geo(a.g, sp, p);
        HopPipe<PREC, RECON, NR, LNT, SF, HopTune<PREC, NR>::depth> pipe{in, act, a.U, S, geo, ph, acc, xo_in, sp_in};
        pipe.run();

        // epilogue per right-hand side: out = add + a * site + c * acc
        const cplx<R> cu = {R(a.c.up[0]), R(a.c.up[1])}, cl = {R(a.c.lo[0]), R(a.c.lo[1])};
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (NR > 1 && !act[r]) continue;
            const int64_t rr = rhs0 + r;
            Spinor<R> o;
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int c = 0; c < 3; ++c) o.s[s][c] = (s < 2 ? cu : cl) * acc[r].s[s][c];
            Spinor<R> st;
            if (a.site) {
                const cplx<R> au = {R(a.a.up[0]), R(a.a.up[1])}, al = {R(a.a.lo[0]), R(a.a.lo[1])};
                SpinorIO<PREC>::load(static_cast<const char*>(a.site) + rr * a.st_site + poff, S, h, st, xo_site,
                                     sp_site);
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int c = 0; c < 3; ++c) o.s[s][c] = o.s[s][c] + (s < 2 ? au : al) * st.s[s][c];
            }
            if (a.add) {
                Spinor<R> ad;
                SpinorIO<PREC>::load(static_cast<const char*>(a.add) + rr * a.st_add + poff, S, h, ad, xo_add, sp_add);
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int c = 0; c < 3; ++c) o.s[s][c] = o.s[s][c] + ad.s[s][c];
            }
            if (a.out)
                SpinorIO<PREC>::template store<LQCD_OUT_AUX>(static_cast<char*>(a.out) + rr * a.st_out + poff, S, h, o,
                                                             xo_out, sp_out);

            if (RED == RED_NORM || RED == RED_NORM_DS) {
                double n2 = 0.0;
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int c = 0; c < 3; ++c) n2 += (double)norm2(o.s[s][c]);
                tot[r][0] = n2;
            }
            if (RED == RED_NORM_DS) {  // <out, site>
                double re = 0.0, im = 0.0;
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const cplx<R> v = cmulc(o.s[s][c], st.s[s][c]);
                        re += (double)v.x;
                        im += (double)v.y;
                    }
                tot[r][N - 2] = re;
                tot[r][N - 1] = im;
            }
            if (RED == RED_DOT_AUX) {  // <aux, out>
                Spinor<R> ax;
                SpinorIO<PREC>::load(static_cast<const char*>(a.aux) + rr * a.st_aux + poff, S, h, ax, xo_aux, sp_aux);
                double re = 0.0, im = 0.0;
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const cplx<R> v = cmulc(ax.s[s][c], o.s[s][c]);
                        re += (double)v.x;
                        im += (double)v.y;
                    }
                tot[r][N - 2] = re;
                tot[r][N - 1] = im;
            }
        }
    }

    if constexpr (RED != RED_NONE) {
        if constexpr (kLanes) block_reduce_lanes<N>(tot[0], a.r.partials, bp.nslots, rhs0, L, a.nrhs, bp.pslot);
        else block_reduce_tile<NR, N>(tot, a.r.partials, bp.nslots, rhs0, a.nrhs, bp.pslot);
    }
}

template <int PREC, int RECON, bool DAG, int RED, int NR, bool LNT>
__global__ void __launch_bounds__((HopBlock<PREC, NR, LNT>::max_threads))
    __attribute__((amdgpu_waves_per_eu(HopTune<PREC, NR>::waves))) k_dslash_eo(const DslashArgs a)
{
    dslash_block<PREC, RECON, DAG, RED, NR, LNT>(a, blockIdx.x, gridDim.x, blockIdx.y);
}

// Several systems (lattices of different sizes) in one launch: block x of the
// flattened grid belongs to system s with offs[s] <= x < offs[s + 1]; each
// system's arguments come from the device table tab.
template <int PREC, int RECON, bool DAG, int RED, int NR, bool LNT>
__global__ void __launch_bounds__((HopBlock<PREC, NR, LNT>::max_threads))
    __attribute__((amdgpu_waves_per_eu(HopTune<PREC, NR>::waves))) k_dslash_eo_batch(const DslashArgs* __restrict__ tab,
                                                        const int* __restrict__ offs, int nsys)
{
    const int x = blockIdx.x;
    int s = 0;
    while (s + 1 < nsys && x >= offs[s + 1]) ++s;
    // each system's range starts at a multiple of 8 (XCD remap); blocks past
    // the system's own grid are padding
    const int bx = x - offs[s];
    if (bx >= tab[s].gx) return;  // (a tile index past ntiles finds no active right-hand side)
    dslash_block<PREC, RECON, DAG, RED, NR, LNT>(tab[s], bx, tab[s].gx, blockIdx.y);
}

template <int PREC, int RECON, bool DAG, int RED, int NR, bool LNT>
static hipError_t launch_one(const DslashLaunch& L, dim3 grid, dim3 block, hipStream_t s)
{
    if (L.tab)
        hipLaunchKernelGGL((k_dslash_eo_batch<PREC, RECON, DAG, RED, NR, LNT>), grid, block, 0, s, L.tab, L.offs, L.nsys);
    else hipLaunchKernelGGL((k_dslash_eo<PREC, RECON, DAG, RED, NR, LNT>), grid, block, 0, s, *L.a);
    return hipGetLastError();
}

template <int PREC, int RECON, bool DAG, int NR, bool LNT>
static hipError_t launch_red(int red, const DslashLaunch& L, dim3 grid, dim3 block, hipStream_t s)
{
    switch (red) {
    case RED_NONE: return launch_one<PREC, RECON, DAG, RED_NONE, NR, LNT>(L, grid, block, s);
    case RED_NORM: return launch_one<PREC, RECON, DAG, RED_NORM, NR, LNT>(L, grid, block, s);
    case RED_NORM_DS: return launch_one<PREC, RECON, DAG, RED_NORM_DS, NR, LNT>(L, grid, block, s);
    case RED_DOT_AUX: return launch_one<PREC, RECON, DAG, RED_DOT_AUX, NR, LNT>(L, grid, block, s);
    default: return hipErrorInvalidValue;
    }
}

template <int PREC, int RECON, int NR, bool LNT>
static hipError_t launch_dag(bool dag, int red, const DslashLaunch& L, dim3 grid, dim3 block, hipStream_t s)
{
    return dag ? launch_red<PREC, RECON, true, NR, LNT>(red, L, grid, block, s)
               : launch_red<PREC, RECON, false, NR, LNT>(red, L, grid, block, s);
}

// Right-hand-side tiles compiled per storage: 1, 2 and 4 for FP32 and FP16
// (the multi-RHS inner solves), 1 and 2 for FP64.  Streaming link loads are
// compiled for the one-tile case only: with several tiles (or a tile of
// several right-hand sides sharing the loaded link) links stay cached.
template <int PREC, int RECON>
inline hipError_t launch_tile(int nr, bool lnt, bool dag, int red, const DslashLaunch& L, dim3 grid, dim3 block,
                              hipStream_t s)
{
    if (nr == 1)
        return lnt ? launch_dag<PREC, RECON, 1, true>(dag, red, L, grid, block, s)
                   : launch_dag<PREC, RECON, 1, false>(dag, red, L, grid, block, s);
    if (nr == 2) return launch_dag<PREC, RECON, 2, false>(dag, red, L, grid, block, s);
    if constexpr (PREC != 64)
        if (nr == 4) return launch_dag<PREC, RECON, 4, false>(dag, red, L, grid, block, s);
    return hipErrorInvalidValue;
}

}  // namespace lqcd
