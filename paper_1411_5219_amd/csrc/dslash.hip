// Host side of the Dslash launches: block order and shape, right-hand-side
// tile, grid, and the finalize step of fused reductions.  The kernels are
// instantiated per storage precision in dslash64/32/16.hip.
#include "lqcd.h"
#include "lqcd_kernels.h"

namespace lqcd {

hipError_t launch_dslash_64(int recon, int nr, bool lnt, bool dag, int red, const DslashLaunch& L, dim3 grid, dim3 block,
                            hipStream_t s);
hipError_t launch_dslash_32(int recon, int nr, bool lnt, bool dag, int red, const DslashLaunch& L, dim3 grid, dim3 block,
                            hipStream_t s);
hipError_t launch_dslash_16(int recon, int nr, bool lnt, bool dag, int red, const DslashLaunch& L, dim3 grid, dim3 block,
                            hipStream_t s);

hipError_t launch_stag_64(int recon, int red, bool lnt, const DslashLaunch& L, dim3 grid, dim3 block, hipStream_t s);
hipError_t launch_stag_32(int recon, int red, bool lnt, const DslashLaunch& L, dim3 grid, dim3 block, hipStream_t s);
hipError_t launch_stag_16(int recon, int red, bool lnt, const DslashLaunch& L, dim3 grid, dim3 block, hipStream_t s);

static hipError_t launch_dslash_prec(const DslashPlan& p, const DslashLaunch& L, dim3 grid, hipStream_t s)
{
    if (p.kind == PLAN_STAG) {
        if (p.prec == 64) return launch_stag_64(p.recon, p.red, p.lnt, L, grid, p.block, s);
        if (p.prec == 32) return launch_stag_32(p.recon, p.red, p.lnt, L, grid, p.block, s);
        if (p.prec == 16) return launch_stag_16(p.recon, p.red, p.lnt, L, grid, p.block, s);
        return hipErrorInvalidValue;
    }
    if (p.prec == 64) return launch_dslash_64(p.recon, p.nr, p.lnt, p.dag, p.red, L, grid, p.block, s);
    if (p.prec == 32) return launch_dslash_32(p.recon, p.nr, p.lnt, p.dag, p.red, L, grid, p.block, s);
    if (p.prec == 16) return launch_dslash_16(p.recon, p.nr, p.lnt, p.dag, p.red, L, grid, p.block, s);
    return hipErrorInvalidValue;
}

int dslash_rhs_tile(int prec, int want, int nrhs)
{
    int nr = want < 1 ? 1 : want;
    if (prec == 64 && nr > 2) nr = 2;
    if (nr > 4) nr = 4;
    if (nr == 3) nr = 2;
    while (nr > 1 && nr > nrhs) nr >>= 1;
    return nr;
}

hipError_t plan_dslash(int prec, int recon, bool dagger, int red, const DslashArgs& args, int nrhs, const Launch& cfg,
                       DslashPlan* out)
{
    if (!((prec == 64 && (recon == 18 || recon == 12)) || (prec == 32 && (recon == 18 || recon == 12)) ||
          (prec == 16 && recon == 12)))
        return hipErrorInvalidValue;
    DslashPlan& p = *out;
    p.kind = PLAN_WILSON;
    p.prec = prec;
    p.recon = recon;
    p.dag = dagger;
    p.red = red;
    DslashArgs& a = p.a;
    a = args;
    a.swizzle = cfg.swizzle;
    a.nrhs = nrhs;
    // right-hand sides across lanes: L = the next power of two of nrhs, at
    // most the request and 16; every field's lane offsets must fit 31 bits
    int L = 1;
    if (nrhs > 1 && cfg.rhs_lanes > 1 && cfg.rhs_tile == 1) {
        while (L < nrhs && 2 * L <= cfg.rhs_lanes && L < 16) L *= 2;
        int64_t st = a.st_in;
        for (int64_t v : {a.st_out, a.st_site, a.st_add, a.st_aux}) st = v > st ? v : st;
        if ((int64_t)L * st >= ((int64_t)1 << 31)) L = 1;
    }
    int blk = cfg.block;
    unsigned nbh = (unsigned)((a.g.Vh + blk - 1) / blk);
    a.rows = 0;
    a.nyc = 0;
    a.ztile = 1;
    a.ygroup = 1;
    const int Lxh = a.g.Lxh, Ly = a.g.L[1];
    if (L > 1) {
        // whole x-rows per block only (the block order and the partials
        // count of the row tiles): the largest divisor R of Ly with R rows
        // within the site budget cfg.block / L (at least one row) and
        // R * Lxh * L lanes within the block limit, where 3/4 of the lanes
        // are busy; otherwise tiles in registers (L = 1)
        const int tmax = hop_lane_block_limit(prec);
        const int sites = cfg.block / L;
        int R = 0;
        if (cfg.order >= 1)
            for (int d = 1; d <= Ly; ++d)
                if (Ly % d == 0 && (d * Lxh <= sites || d == 1) && d * Lxh * L <= tmax) R = d;
        const int B = (R * Lxh * L + 63) / 64 * 64;
        if (R > 0 && B <= tmax && 4 * R * Lxh * L >= 3 * B) {
            a.rows = R;
            a.nyc = (Ly + R - 1) / R;
            for (int d = 1; d <= a.g.L[2] && d <= cfg.order; ++d)
                if (a.g.L[2] % d == 0) a.ztile = d;
            if (a.ztile == 1)
                for (int d = 1; d <= a.nyc && d <= cfg.ygroup; ++d)
                    if (a.nyc % d == 0) a.ygroup = d;
            blk = R * Lxh;
            nbh = (unsigned)a.nyc * a.g.L[2] * a.g.L[3];
        } else {
            L = 1;
        }
    }
    a.lanes = L;
    a.lanes_log2 = 0;
    while ((1 << a.lanes_log2) < L) ++a.lanes_log2;
    if (L == 1 && cfg.order >= 1 && Lxh <= 256) {
        // R whole x-rows per block: the largest divisor of Ly with R*Lxh at
        // most the requested block size (at least one row); the block is
        // rounded up to whole wavefronts.
        int R = 1;
        for (int d = 1; d <= Ly; ++d)
            if (Ly % d == 0 && d * Lxh <= cfg.block) R = d;
        int B = (R * Lxh + 63) / 64 * 64;
        if (B > 256) {  // one row per block: keep the block within the kernel's bound
            R = 1;
            B = (Lxh + 63) / 64 * 64;
        }
        // row tiles only where they keep at least 3/4 of the lanes busy
        if (4 * R * Lxh >= 3 * B) {
            a.rows = R;
            a.nyc = (Ly + R - 1) / R;
            // z-slabs: the largest divisor of Lz not above the requested depth
            for (int d = 1; d <= a.g.L[2] && d <= cfg.order; ++d)
                if (a.g.L[2] % d == 0) a.ztile = d;
            // y-chunk groups (t-fastest order only): the largest divisor of
            // the chunk count not above the request
            if (a.ztile == 1)
                for (int d = 1; d <= a.nyc && d <= cfg.ygroup; ++d)
                    if (a.nyc % d == 0) a.ygroup = d;
            blk = B;
            nbh = (unsigned)a.nyc * a.g.L[2] * a.g.L[3];
        }
    }
    a.bdim = blk;
    p.nr = L > 1 ? 1 : dslash_rhs_tile(prec, cfg.rhs_tile, nrhs);
    a.ntiles = (nrhs + p.nr * L - 1) / (p.nr * L);
    // links are streamed past the caches when no other block of the launch
    // reads them (one right-hand side per site); with right-hand sides across
    // lanes the L lanes of a site share one cached load
    p.lnt = p.nr == 1 && a.ntiles == 1 && L == 1;
    a.nsp = (int)nbh;
    // interleave right-hand-side tiles into the block order when there are several
    a.rhs_group = (L == 1 && cfg.rhs_group > 1 && a.ntiles > 1) ? (cfg.rhs_group < a.ntiles ? cfg.rhs_group : a.ntiles)
                                                                 : 0;
    p.block = dim3(L > 1 ? (unsigned)((blk * L + 63) / 64 * 64) : (unsigned)blk);
    if (a.rhs_group > 0) {
        const unsigned groups = (unsigned)((a.ntiles + a.rhs_group - 1) / a.rhs_group);
        p.grid = dim3(nbh * (unsigned)a.rhs_group * groups * (a.full ? 2u : 1u), 1);
    } else {
        p.grid = dim3(nbh * (a.full ? 2u : 1u), (unsigned)a.ntiles);
    }
    a.gx = (int)p.grid.x;
    // partials hold one slot per spatial block and parity for each right-hand side
    p.slots = (int)nbh * (a.full ? 2 : 1);
    if (red != RED_NONE && p.slots > a.r.capacity) return hipErrorInvalidValue;  // partials too small
    p.nfin = red == RED_NONE ? 0 : red == RED_NORM ? 1 : red == RED_DOT_AUX ? 2 : 3;
    return hipSuccess;
}

hipError_t exec_dslash(const DslashPlan& p, hipStream_t s)
{
    DslashLaunch L{&p.a, nullptr, nullptr, 1};
    const hipError_t e = launch_dslash_prec(p, L, p.grid, s);
    if (e != hipSuccess || p.nfin == 0) return e;
    const hipError_t f = launch_finalize(p.nfin, p.a.r.partials, p.slots, p.a.r.fin, p.a.ctl, p.a.pred, p.a.nrhs, s);
    // both parities in one launch: the even-parity blocks hold the first half of the partials
    if (f != hipSuccess || !p.a.full || !p.a.r.fin_even) return f;
    return launch_finalize(p.nfin, p.a.r.partials, p.slots, p.a.r.fin_even, p.a.ctl, p.a.pred, p.a.nrhs, s,
                           p.slots / 2);
}

hipError_t exec_dslash_batch(const DslashPlan* plans, int n, const DslashArgs* tab, const int* offs, int total_blocks,
                             const FinArgs* fin_tab, hipStream_t s)
{
    if (n < 1) return hipErrorInvalidValue;
    const DslashPlan& p0 = plans[0];
    unsigned gy = p0.grid.y, bx = p0.block.x;
    for (int i = 1; i < n; ++i) {
        gy = plans[i].grid.y > gy ? plans[i].grid.y : gy;
        bx = plans[i].block.x > bx ? plans[i].block.x : bx;
    }
    DslashPlan q = p0;
    q.block = dim3(bx);
    DslashLaunch L{nullptr, tab, offs, n};
    const hipError_t e = launch_dslash_prec(q, L, dim3((unsigned)total_blocks, gy), s);
    if (e != hipSuccess || p0.nfin == 0) return e;
    return launch_finalize_batch(p0.nfin, fin_tab, n, p0.a.nrhs, s);
}

hipError_t launch_dslash(int prec, int recon, bool dagger, int red, const DslashArgs& args, int nrhs,
                         const Launch& cfg, hipStream_t s)
{
    DslashPlan p;
    hipError_t e = plan_dslash(prec, recon, dagger, red, args, nrhs, cfg, &p);
    if (e != hipSuccess) return e;
    if (Recorder* r = active_recorder()) {
        r->steps.push_back(Step{});
        r->steps.back().kind = STEP_DSLASH;
        r->steps.back().d = p;
        return hipSuccess;
    }
    return exec_dslash(p, s);
}

hipError_t launch_stag(int prec, int recon, int red, const DslashArgs& args, int nrhs, const Launch& cfg,
                       hipStream_t s)
{
    if (red != RED_NONE && red != RED_NORM && red != RED_NORM_DS) return hipErrorInvalidValue;
    Launch c = cfg;
    c.rhs_tile = 1;   // one right-hand side per work-item, tiles along grid.y
    c.rhs_group = 0;
    c.rhs_lanes = 1;
    DslashPlan p;
    hipError_t e = plan_dslash(prec, recon, false, red, args, nrhs, c, &p);
    if (e != hipSuccess) return e;
    p.kind = PLAN_STAG;
    p.nfin = red == RED_NONE ? 0 : red == RED_NORM ? 1 : 3;
    if (Recorder* r = active_recorder()) {
        r->steps.push_back(Step{});
        r->steps.back().kind = STEP_DSLASH;
        r->steps.back().d = p;
        return hipSuccess;
    }
    return exec_dslash(p, s);
}

}  // namespace lqcd
