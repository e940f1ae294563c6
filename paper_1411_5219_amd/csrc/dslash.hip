// Host side of the Dslash launches: block order and shape, right-hand-side
// tile, grid, and the finalize step of fused reductions.  The kernels are
// instantiated per storage precision in dslash64/32/16.hip.
#include "lqcd.h"
#include "lqcd_kernels.h"

namespace lqcd {

hipError_t launch_dslash_64(int recon, int nr, bool dag, int red, const DslashArgs& a, dim3 grid, dim3 block,
                            hipStream_t s);
hipError_t launch_dslash_32(int recon, int nr, bool dag, int red, const DslashArgs& a, dim3 grid, dim3 block,
                            hipStream_t s);
hipError_t launch_dslash_16(int recon, int nr, bool dag, int red, const DslashArgs& a, dim3 grid, dim3 block,
                            hipStream_t s);

static hipError_t launch_dslash_prec(int prec, int recon, int nr, bool dag, int red, const DslashArgs& a, dim3 grid,
                                     dim3 block, hipStream_t s)
{
    if (prec == 64) return launch_dslash_64(recon, nr, dag, red, a, grid, block, s);
    if (prec == 32) return launch_dslash_32(recon, nr, dag, red, a, grid, block, s);
    if (prec == 16) return launch_dslash_16(recon, nr, dag, red, a, grid, block, s);
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

hipError_t launch_dslash(int prec, int recon, bool dagger, int red, const DslashArgs& args, int nrhs,
                         const Launch& cfg, hipStream_t s)
{
    DslashArgs a = args;
    a.swizzle = cfg.swizzle;
    a.nrhs = nrhs;
    int blk = cfg.block;
    unsigned nbh = (unsigned)((a.g.Vh + blk - 1) / blk);
    a.rows = 0;
    a.nyc = 0;
    const int Lxh = a.g.Lxh, Ly = a.g.L[1];
    if (cfg.order == 1 && Lxh <= 256) {
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
            blk = B;
            nbh = (unsigned)a.nyc * a.g.L[2] * a.g.L[3];
        }
    }
    const int nr = dslash_rhs_tile(prec, cfg.rhs_tile, nrhs);
    a.ntiles = (nrhs + nr - 1) / nr;
    a.nsp = (int)nbh;
    // interleave right-hand-side tiles into the block order when there are several
    a.rhs_group = (cfg.rhs_group > 1 && a.ntiles > 1) ? (cfg.rhs_group < a.ntiles ? cfg.rhs_group : a.ntiles) : 0;
    dim3 block(blk);
    dim3 grid;
    if (a.rhs_group > 0) {
        const unsigned groups = (unsigned)((a.ntiles + a.rhs_group - 1) / a.rhs_group);
        grid = dim3(nbh * (unsigned)a.rhs_group * groups * (a.full ? 2u : 1u), 1);
    } else {
        grid = dim3(nbh * (a.full ? 2u : 1u), (unsigned)a.ntiles);
    }
    // partials hold one slot per spatial block and parity for each right-hand side
    const int slots = (int)nbh * (a.full ? 2 : 1);
    if (red != RED_NONE && slots > a.r.capacity) return hipErrorInvalidValue;  // partials too small
    const hipError_t e = launch_dslash_prec(prec, recon, nr, dagger, red, a, grid, block, s);
    if (e != hipSuccess || red == RED_NONE) return e;
    return launch_finalize((red == RED_NORM ? 1 : red == RED_DOT_AUX ? 2 : 3), a.r.partials, slots, a.r.fin, a.ctl,
                           a.pred, nrhs, s);
}

}  // namespace lqcd
