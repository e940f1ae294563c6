// Where a block and a work-item of a stencil launch work: the block's
// parity, spatial block and right-hand-side tile (with the XCD remap, the
// both-parities mode and the right-hand-side groups of the launch), the
// output site of the work-item in the launch's block order, and the
// neighbours of that site.  Shared by the Wilson and the staggered hop
// kernels, which walk the lattice the same way.
#pragma once

#include "lqcd_device.h"
#include "lqcd_kernels.h"

namespace lqcd {

struct BlockPos {
    int p;            // output parity
    int bid;          // spatial block within the parity
    int tile;         // right-hand-side tile
    int pslot;        // partials slot of this block within its right-hand side
    int nslots;       // partials slots per right-hand side
    int64_t poff;     // byte offset of the output-parity half of full-lattice fields
    int64_t ioff;     // byte offset of the neighbour-parity half
};

__device__ __forceinline__ BlockPos block_pos(const DslashArgs& a, int bx, int nb, int by)
{
    BlockPos b;
    int bid = a.swizzle ? xcd_swizzle(bx, nb) : bx;
    b.p = a.parity;
    b.poff = 0;
    b.ioff = 0;
    if (a.full) {  // both parities in one launch: the first nb/2 blocks even, the rest odd
        const int nbh = nb >> 1;
        b.p = bid >= nbh;
        bid -= b.p * nbh;
        b.poff = b.p * a.par_bytes;
        b.ioff = (1 - b.p) * a.par_bytes;
    }
    b.tile = by;
    int nsp = a.full ? nb >> 1 : nb;  // spatial blocks per parity (per tile)
    if (a.rhs_group > 0) {
        const int G = a.rhs_group;
        const int ti = bid % G;
        const int rest = bid / G;
        nsp = a.nsp;
        b.tile = (rest / nsp) * G + ti;
        bid = rest % nsp;
    }
    b.bid = bid;
    b.pslot = bid + b.p * nsp;
    b.nslots = nsp * (a.full ? 2 : 1);
    return b;
}

struct SitePos {
    int h;            // parity-local index of the output site
    int xh, x, y, z, t;
    bool valid;       // false for work-items past the lattice (padding lanes)
};

// Output site of site work-item tid (threadIdx.x, or threadIdx.x >> lanes_log2
// with right-hand sides across lanes) in spatial block bid of parity p
// (memory order, t-fastest row tiles or z-slabs of row tiles; see DslashArgs).
__device__ __forceinline__ SitePos site_pos(const DslashArgs& a, int bid, int p, int tid)
{
    const int Ly = a.g.L[1], Lz = a.g.L[2], Lt = a.g.L[3];
    const int Lxh = a.g.Lxh;
    SitePos s;
    if (a.rows == 0) {
        s.h = bid * a.bdim + tid;
        s.valid = tid < a.bdim && s.h < a.g.Vh;
        s.xh = s.h % Lxh;
        int r = s.h / Lxh;
        s.y = r % Ly;
        r /= Ly;
        s.z = r % Lz;
        s.t = r / Lz;
    } else {
        int yc;
        if (a.ztile <= 1 && a.ygroup > 1) {
            const int G = a.ygroup;
            s.t = bid % Lt;
            int r = bid / Lt;
            const int yi = r % G;
            r /= G;
            s.z = r % Lz;
            yc = (r / Lz) * G + yi;
        } else if (a.ztile <= 1) {
            s.t = bid % Lt;
            const int r = bid / Lt;
            s.z = r % Lz;
            yc = r / Lz;
        } else {
            const int T = a.ztile, nzs = Lz / T;
            const int zl = bid % T;
            int r = bid / T;
            s.t = r % Lt;
            r /= Lt;
            s.z = (r % nzs) * T + zl;
            yc = r / nzs;
        }
        const int yr = tid / Lxh;
        s.xh = tid - yr * Lxh;
        s.y = yc * a.rows + yr;
        s.valid = yr < a.rows && s.y < Ly;
        s.h = s.xh + Lxh * (s.y + Ly * (s.z + Lz * s.t));
    }
    s.x = 2 * s.xh + ((s.y + s.z + s.t + p) & 1);
    return s;
}

// Neighbour of an output site for hop K = 2 mu + (0 forward, 1 backward):
// the neighbour's parity-local index, the link block (mu, parity) and the
// parity-local site the link is stored at, and whether the hop crosses the
// lattice boundary (and so takes the boundary phase).
// Parity-local indices fit 32 bits (the library limits V/2 to 21 * 2^20),
// which keeps them in one register each.
struct Nbr {
    int nb, lsite;
    int lblk;
    bool cross;
};

struct SiteGeo {
    int x, y, z, t, p, Lx, Ly, Lz, Lt;
    int h, base, hy, hz, ht;

    template <int K>
    __device__ __forceinline__ Nbr get() const
    {
        constexpr int MU = K >> 1;
        constexpr bool FWD = (K & 1) == 0;
        Nbr n;
        if constexpr (MU == 0) {
            if constexpr (FWD) {
                n.cross = x == Lx - 1;
                n.nb = base + ((n.cross ? 0 : x + 1) >> 1);
            } else {
                n.cross = x == 0;
                n.nb = base + ((n.cross ? Lx - 1 : x - 1) >> 1);
            }
        } else {
            const int c = MU == 1 ? y : MU == 2 ? z : t;
            const int Lc = MU == 1 ? Ly : MU == 2 ? Lz : Lt;
            const int hc = MU == 1 ? hy : MU == 2 ? hz : ht;
            if constexpr (FWD) {
                n.cross = c == Lc - 1;
                n.nb = n.cross ? h - (Lc - 1) * hc : h + hc;
            } else {
                n.cross = c == 0;
                n.nb = n.cross ? h + (Lc - 1) * hc : h - hc;
            }
        }
        // U_mu(x) for forward hops, U_mu(x - mu) (stored at the neighbour) for backward ones
        n.lblk = 2 * MU + (FWD ? p : 1 - p);
        n.lsite = FWD ? h : n.nb;
        return n;
    }
};

__device__ __forceinline__ SiteGeo site_geo(const Geom& g, const SitePos& s, int p)
{
    const int Lxh = g.Lxh, Ly = g.L[1], Lz = g.L[2];
    return SiteGeo{s.x, s.y, s.z, s.t, p, g.L[0], Ly, Lz, g.L[3], s.h, s.h - s.xh, Lxh, Lxh * Ly, Lxh * Ly * Lz};
}

}  // namespace lqcd
