// Even-odd staggered (Kogut-Susskind) hop for gfx950 (kernel templates; each
// storage precision is instantiated in its own translation unit).
//
// One work-item per output site x of parity p:
//
//   acc = sum_mu eta_mu(x) [ f+ U_mu(x) chi(x + mu) - f- U_mu(x - mu)^+ chi(x - mu) ]
//
// with the staggered phases eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y),
// eta_3 = (-1)^(x+y+z) and the boundary factors f+- on hops that cross the
// lattice boundary; D = acc / 2.  The store fuses the site term and FP64
// reductions: out = add + a * site + c * acc (the 1/2 and the sign of D or
// of its adjoint -D travel in c).  Block order, parity split and neighbour
// indices are those of the Wilson hop.
#pragma once

#include "block_order.h"
#include "lqcd.h"
#include "lqcd_device.h"
#include "lqcd_fin.h"
#include "lqcd_kernels.h"

namespace lqcd {

template <class R, bool ADJ>
__device__ __forceinline__ void su3_vec(const Link<R>& U, const Colour<R>& v, Colour<R>& w)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        w.c[a] = su3_row<R, ADJ>(U.u, a, v.c);
    }
}

// One hop: the neighbour colour vector, then its link (the link is the larger
// operand; loading the vector first lets its load overlap the link's).
template <int PREC, int RECON, int K, bool LNT>
__device__ __forceinline__ void stag_hop(const char* in, const void* U, int64_t S, const SiteGeo& g,
                                         const cplx<typename ColourIO<PREC>::R> (&ph)[4],
                                         typename ColourIO<PREC>::R eta, Colour<typename ColourIO<PREC>::R>& acc)
{
    using R = typename ColourIO<PREC>::R;
    constexpr int MU = K >> 1;
    constexpr bool FWD = (K & 1) == 0;
    const Nbr n = g.template get<K>();
    Colour<R> v;
    ColourIO<PREC>::load(in, S, n.nb, v);
    Link<R> L;
    if constexpr (LNT) LinkIO<PREC, RECON>::template load<>(U, S, n.lblk, n.lsite, L);
    else LinkIO<PREC, RECON>::template load<0>(U, S, n.lblk, n.lsite, L);
    Colour<R> w;
    su3_vec<R, !FWD>(L, v, w);
    if (n.cross) {
        const cplx<R> f = FWD ? ph[MU] : conj(ph[MU]);
#pragma unroll
        for (int a = 0; a < 3; ++a) w.c[a] = f * w.c[a];
    }
    const R sg = FWD ? eta : -eta;
#pragma unroll
    for (int a = 0; a < 3; ++a) acc.c[a] = acc.c[a] + sg * w.c[a];
}

template <int RED>
struct StagRedN {
    static constexpr int N = RED == RED_NORM_DS ? 3 : 1;
};

template <int PREC, int RECON, int RED, bool LNT>
__device__ __forceinline__ void stag_block(const DslashArgs& a, int bx, int nbx, int by)
{
    using R = typename ColourIO<PREC>::R;
    constexpr int N = StagRedN<RED>::N;
    const BlockPos bp = block_pos(a, bx, nbx, by);
    const int p = bp.p, rhs = bp.tile;
    if (rhs >= a.nrhs || pred_skip(a.pred, a.ctl ? a.ctl + rhs : nullptr)) return;
    const SitePos sp = site_pos(a, bp.bid, p, (int)threadIdx.x);
    const int64_t S = a.g.S;
    double tot[N];
#pragma unroll
    for (int j = 0; j < N; ++j) tot[j] = 0.0;

    if (sp.valid) {
        const SiteGeo geo = site_geo(a.g, sp, p);
        const char* in = static_cast<const char*>(a.in) + (int64_t)rhs * a.st_in + bp.ioff;
        const cplx<R> ph[4] = {{R(a.g.ph[0][0]), R(a.g.ph[0][1])},
                               {R(a.g.ph[1][0]), R(a.g.ph[1][1])},
                               {R(a.g.ph[2][0]), R(a.g.ph[2][1])},
                               {R(a.g.ph[3][0]), R(a.g.ph[3][1])}};
        const R e1 = (sp.x & 1) ? R(-1) : R(1);
        const R e2 = ((sp.x + sp.y) & 1) ? R(-1) : R(1);
        const R e3 = ((sp.x + sp.y + sp.z) & 1) ? R(-1) : R(1);
        Colour<R> acc;
#pragma unroll
        for (int c = 0; c < 3; ++c) acc.c[c] = {R(0), R(0)};
        stag_hop<PREC, RECON, 0, LNT>(in, a.U, S, geo, ph, R(1), acc);
        stag_hop<PREC, RECON, 1, LNT>(in, a.U, S, geo, ph, R(1), acc);
        stag_hop<PREC, RECON, 2, LNT>(in, a.U, S, geo, ph, e1, acc);
        stag_hop<PREC, RECON, 3, LNT>(in, a.U, S, geo, ph, e1, acc);
        stag_hop<PREC, RECON, 4, LNT>(in, a.U, S, geo, ph, e2, acc);
        stag_hop<PREC, RECON, 5, LNT>(in, a.U, S, geo, ph, e2, acc);
        stag_hop<PREC, RECON, 6, LNT>(in, a.U, S, geo, ph, e3, acc);
        stag_hop<PREC, RECON, 7, LNT>(in, a.U, S, geo, ph, e3, acc);

        // out = add + a * site + c * acc
        const cplx<R> cc = {R(a.c.up[0]), R(a.c.up[1])};
        Colour<R> o;
#pragma unroll
        for (int c = 0; c < 3; ++c) o.c[c] = cc * acc.c[c];
        Colour<R> st;
        if (a.site) {
            const cplx<R> ca = {R(a.a.up[0]), R(a.a.up[1])};
            ColourIO<PREC>::load(static_cast<const char*>(a.site) + rhs * a.st_site + bp.poff, S, sp.h, st);
#pragma unroll
            for (int c = 0; c < 3; ++c) o.c[c] = o.c[c] + ca * st.c[c];
        }
        if (a.add) {
            Colour<R> ad;
            ColourIO<PREC>::load(static_cast<const char*>(a.add) + rhs * a.st_add + bp.poff, S, sp.h, ad);
#pragma unroll
            for (int c = 0; c < 3; ++c) o.c[c] = o.c[c] + ad.c[c];
        }
        if (a.out)
            ColourIO<PREC>::template store<LQCD_OUT_AUX>(static_cast<char*>(a.out) + rhs * a.st_out + bp.poff, S,
                                                        sp.h, o);
        if (RED == RED_NORM || RED == RED_NORM_DS) {
#pragma unroll
            for (int c = 0; c < 3; ++c) tot[0] += (double)norm2(o.c[c]);
        }
        if (RED == RED_NORM_DS) {  // <out, site>
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const cplx<R> v = cmulc(o.c[c], st.c[c]);
                tot[1] += (double)v.x;
                tot[2] += (double)v.y;
            }
        }
    }
    if (RED != RED_NONE) block_reduce_store<N>(tot, a.r.partials + ((int64_t)rhs * bp.nslots) * N, bp.pslot);
}

template <int PREC, int RECON, int RED, bool LNT>
__global__ void __launch_bounds__(256) k_stag_eo(const DslashArgs a)
{
    stag_block<PREC, RECON, RED, LNT>(a, blockIdx.x, gridDim.x, blockIdx.y);
}

template <int PREC, int RECON, int RED, bool LNT>
static hipError_t stag_one(const DslashLaunch& L, dim3 grid, dim3 block, hipStream_t s)
{
    if (L.tab) return hipErrorInvalidValue;  // no batched staggered launches
    hipLaunchKernelGGL((k_stag_eo<PREC, RECON, RED, LNT>), grid, block, 0, s, *L.a);
    return hipGetLastError();
}

template <int PREC, int RECON>
inline hipError_t launch_stag_red(int red, bool lnt, const DslashLaunch& L, dim3 grid, dim3 block, hipStream_t s)
{
    switch (red) {
    case RED_NONE: return lnt ? stag_one<PREC, RECON, RED_NONE, true>(L, grid, block, s)
                              : stag_one<PREC, RECON, RED_NONE, false>(L, grid, block, s);
    case RED_NORM: return lnt ? stag_one<PREC, RECON, RED_NORM, true>(L, grid, block, s)
                              : stag_one<PREC, RECON, RED_NORM, false>(L, grid, block, s);
    case RED_NORM_DS: return lnt ? stag_one<PREC, RECON, RED_NORM_DS, true>(L, grid, block, s)
                                 : stag_one<PREC, RECON, RED_NORM_DS, false>(L, grid, block, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lqcd
