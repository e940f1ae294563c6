// Kernel argument blocks and the host-side launchers of every kernel in the
// library (the solvers' control block is in solver_ctl.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "solver_ctl.h"

namespace lqcd {

// Lattice geometry as the kernels see it.
struct Geom {
    int L[4];        // extents x, y, z, t (all even)
    int Lxh;         // L[0] / 2
    int Vh;          // sites per parity
    int64_t S;       // plane stride in sites (Vh rounded up to 256)
    double ph[4][2]; // exp(i theta_mu): applied on hops that cross the boundary
};

// Spin-block coefficients (upper spins 0,1 / lower spins 2,3), complex.
struct SpinCoef {
    double up[2];
    double lo[2];
};

// Which scalars a reduction produces (totals per right-hand side):
//   RED_NONE
//   RED_NORM    : ||out||^2
//   RED_NORM_DS : ||out||^2, <out, site>          (re, im)
//   RED_DOT_AUX : <aux, out>                      (re, im)
enum Red { RED_NONE = 0, RED_NORM = 1, RED_NORM_DS = 2, RED_DOT_AUX = 3 };

// Predicates on the control block evaluated at the top of a kernel.
enum Pred {
    PRED_ALWAYS = 0,      // ignore the control block
    PRED_ACTIVE = 1,      // skip when done
    PRED_UPDATE = 2,      // run only while a reliable update is pending (and not done)
    PRED_NO_UPDATE = 3,   // run only while no update is pending (and not done)
};

// Most values one reduction produces per block (BiCGStab(2)'s Gram step).
constexpr int kMaxFin = 5;

struct RedArgs {
    double* partials;       // [nrhs][nblocks][N]
    int capacity;           // blocks the partials hold per right-hand side (N <= kMaxFin)
    int fin;                // Fin
    int fin_even;           // full-lattice launches: a second Fin on the even-parity blocks' partials (0: none)
};

// Dslash_eo with a fused epilogue:
//   out = add + a * site + c * (sum of the 8 hops of `in` onto parity `parity`)
// with a, c spin-block coefficients; `add`, `site`, `out` may be null.
struct DslashArgs {
    Geom g;
    int parity;
    int pred;
    const void* in;
    void* out;
    const void* site;
    const void* add;
    const void* aux;
    const void* U;
    SpinCoef a, c;
    // bytes between right-hand sides of each field
    int64_t st_in, st_out, st_site, st_add, st_aux;
    int full;               // 1: both parities in one launch (fields are full-lattice)
    int64_t par_bytes;      // bytes of one parity field (full = 1)
    RedArgs r;
    Ctl* ctl;               // per right-hand side, or null
    int swizzle;
    // Block order.  rows = 0: block b covers eo sites [b*B, (b+1)*B) in
    // memory order.  rows = R > 0: a block covers R whole x-rows at one
    // (z, t) (a contiguous chunk of sites) and blocks run t fastest, then z,
    // then the y-chunk, so the t and z neighbours a block reads were loaded
    // by blocks that ran just before it on the same XCD.  ztile = T > 1
    // (T divides Lz): z-slabs of T planes, z fastest within a slab, then t,
    // then the slab, then the y-chunk; a spinor's z and t neighbours are then
    // at most T blocks away except on slab faces.
    // ygroup = G > 1 (ztile 1; G divides nyc): G neighbouring y-chunks run
    // after t and before z (t fastest, then the G chunks, then z, then the
    // group), so the rows just outside a chunk, which its y-hops read, were
    // loaded by blocks a few places before it on the same XCD.
    int rows;
    int nyc;                // y-chunks of R rows (rows > 0)
    int ztile;              // z-planes per slab (rows > 0; 1: t fastest)
    int ygroup;             // y-chunks interleaved after t (rows > 0, ztile 1)
    int nrhs;               // right-hand sides (set by the launcher)
    // Right-hand-side tiles in the block order.  rhs_group = 0: tile index
    // is blockIdx.y.  rhs_group = G > 0: grid.y = 1 and the tiles are
    // interleaved into blockIdx.x, G tiles fastest over the same spatial
    // block, then the spatial blocks, then the groups of G tiles, so a link
    // loaded for one tile is re-read from L2 by the next G - 1 blocks.
    int rhs_group;
    int ntiles;             // right-hand-side tiles (ceil(nrhs / tile))
    int nsp;                // spatial blocks per parity (rhs_group > 0)
    // Right-hand sides across lanes: lanes = L > 1 (a power of two, tile 1):
    // work-item t of a block serves site t >> lanes_log2 of the block and
    // right-hand side (tile L + (t & (L - 1))), so the L right-hand sides of
    // a site sit in adjacent lanes of one wave, their link loads are one
    // coalesced request, and the link comes from memory once per hop for all
    // of them.  The right-hand-side offset travels in the per-lane buffer
    // offset (the buffer base stays uniform).
    int lanes;
    int lanes_log2;
    int bdim;               // site work-items of a block that this argument set uses
    int gx;                 // planned grid.x (batched launches pad each system's range)
};

// Waves per SIMD the one-right-hand-side hop kernels are compiled for (their
// register budget): FP64 holds about 250 registers at two waves, FP32 and FP16
// keep three.  The tile-1 launches with right-hand sides across lanes take
// blocks of up to one compute unit's worth of those waves.
#ifndef LQCD_WAVES_64
#define LQCD_WAVES_64 2
#endif
#ifndef LQCD_WAVES_32
#define LQCD_WAVES_32 3
#endif
#ifndef LQCD_WAVES_16
#define LQCD_WAVES_16 3
#endif
__host__ __device__ constexpr int hop_waves(int prec)
{
    return prec == 64 ? LQCD_WAVES_64 : prec == 32 ? LQCD_WAVES_32 : LQCD_WAVES_16;
}
__host__ __device__ constexpr int hop_lane_block_limit(int prec) { return 256 * hop_waves(prec); }

// Launch configuration picked per kernel (autotuned).
struct Launch {
    int block = 128;
    int swizzle = 1;
    int order = 0;     // 0: memory order, 1: t-fastest tiles of whole x-rows, k > 1: z-slabs of k planes (Dslash)
    int rhs_tile = 4;  // right-hand sides one Dslash work-item handles (links loaded once)
    int rhs_group = 4; // right-hand-side tiles interleaved per spatial block (0: grid.y)
    int ygroup = 1;    // y-chunks interleaved after t in the row-tile order (1: none)
    int rhs_lanes = 1; // right-hand sides across adjacent lanes of a site (1: none; 2..16, tile 1)
};

// Right-hand-side tile the Dslash uses for a request (clamped to the tiles
// compiled for the precision and to nrhs).
int dslash_rhs_tile(int prec, int want, int nrhs);

// Sum N block partials per right-hand side in block order and run the
// solver's scalar step (Fin) on the totals; one block per right-hand side.
// count < nblocks sums only the first count partials of each right-hand
// side (nblocks stays the stride between right-hand sides).
hipError_t launch_finalize(int N, const double* partials, int nblocks, int fin, Ctl* ctl, int pred, int nrhs,
                           hipStream_t s, int count = -1);

// ---- launchers (return hipError_t) ----
hipError_t launch_dslash(int prec, int recon, bool dagger, int red, const DslashArgs& a, int nrhs,
                         const Launch& cfg, hipStream_t s);
// The staggered even-odd hop with the same arguments: out = add + a * site +
// c * sum_mu eta_mu [U chi(x + mu) - U^+ chi(x - mu)] (a, c: the up entries of
// the coefficients), one right-hand side per work-item, reductions NONE, NORM
// or NORM_DS.
hipError_t launch_stag(int prec, int recon, int red, const DslashArgs& args, int nrhs, const Launch& cfg,
                       hipStream_t s);

// One Dslash launch, or a batch of nsys argument sets in device memory.
struct DslashLaunch {
    const DslashArgs* a;
    const DslashArgs* tab;
    const int* offs;
    int nsys;
};

// Finalize of one reduction of one system (batched finalize tables).
struct FinArgs {
    const double* partials;
    int nblocks;
    int fin;
    Ctl* ctl;
    int pred;
};

// A planned Dslash launch (final arguments, grid, kernel selectors).
// Stencil of a planned hop launch.
enum PlanKind { PLAN_WILSON = 0, PLAN_STAG = 1 };

struct DslashPlan {
    DslashArgs a;
    dim3 grid, block;
    int kind;   // PlanKind
    int prec, recon, nr, red;
    bool dag;
    bool lnt;   // streaming link loads (one right-hand-side tile of one)
    int nfin;   // values per finalize (0: no reduction)
    int slots;  // partial slots per right-hand side
};
hipError_t plan_dslash(int prec, int recon, bool dagger, int red, const DslashArgs& args, int nrhs, const Launch& cfg,
                       DslashPlan* out);
hipError_t exec_dslash(const DslashPlan& p, hipStream_t s);
// plans[0..n) share kernel selectors; tab / offs / fin_tab are their device
// tables (arguments, block offsets with offs[n] = total_blocks, finalizes).
hipError_t exec_dslash_batch(const DslashPlan* plans, int n, const DslashArgs* tab, const int* offs, int total_blocks,
                             const FinArgs* fin_tab, hipStream_t s);
hipError_t launch_finalize_batch(int N, const FinArgs* tab, int nsys, int nrhs, hipStream_t s);

// Site-local BLAS-1 on parity fields of precision prec (all operands the same).
enum Blas {
    BLAS_CG_XR = 0,       // x += alpha p; r -= alpha w;           red ||r||^2
    BLAS_CG_P = 1,        // p = z + beta p
    BLAS_COPY = 2,        // y = x
    BLAS_ZERO = 3,        // y = 0
    BLAS_SPIN_SCALE = 4,  // y = coef * x                          (spin-block coefficient)
    BLAS_NORM = 5,        // red ||x||^2
    BLAS_BI_P = 6,        // p = r + beta (p - omega v), beta = (rho/rho_old)(alpha/omega)
    BLAS_BI_S = 7,        // s = r - alpha v
    BLAS_BI_XR = 8,       // x += alpha p + omega s; r = s - omega t; red ||r||^2, <r0, r>
    BLAS_XPY = 9,         // y += x
    BLAS_NORM_DOT = 10,   // red ||x||^2, <r0, x>
    BLAS_MS_AXPY = 11,    // x += alpha p                          (alpha of each right-hand side's Ctl)
    BLAS_MS_P = 12,       // p = zeta z + beta p                   (zeta, beta of each Ctl)
    BLAS_AXMY_NORM = 13,  // z -= alpha w;                         red ||z||^2
    // BiCGStab(2) (coefficients from each right-hand side's Ctl): y = u_0,
    // z = r_0, w = u_1 or r_1, v = u_2, r_1 or r_2, r0 = u_2 or rt
    BLAS_BL_U0 = 14,      // u_0 = r_0 - beta (u_0 - g1 u_1 - g2 u_2)         (y, z, w = u_1, v = u_2)
    BLAS_BL_XR0 = 15,     // x += alpha u_0; r_0 -= alpha u_1                 (x, y, z, w = u_1)
    BLAS_BL_U01 = 16,     // u_0 = r_0 - beta u_0; u_1 = r_1 - beta u_1       (y, z, w = u_1, v = r_1)
    BLAS_BL_XR01 = 17,    // x += alpha u_0; r_0 -= alpha u_1; r_1 -= alpha u_2 (x, y, z, w = u_1, v = r_1, r0 = u_2)
    BLAS_BL_GRAM = 18,    // red ||r_1||^2, <r_1, r_2>, <r_1, r_0>            (z, w = r_1, v = r_2)
    BLAS_BL_ORTH = 19,    // r_2 -= tau r_1; red ||r_2||^2, <r_2, r_0>         (z, w = r_1, v = r_2)
    BLAS_BL_MR = 20,      // x += g1 r_0 + g2 r_1; r_0 -= gp1 r_1 + gp2 r_2; red ||r_0||^2, <rt, r_0>
                          //                                                  (x, z, w = r_1, v = r_2, r0 = rt)
};

struct BlasArgs {
    int kind;               // FieldKind of every operand (0: spinor, 1: colour vector)
    int Vh;
    int64_t S;
    int nsub;               // sub-fields of Vh sites each (1: parity field, 2: full lattice)
    int64_t sub_stride;     // bytes between sub-fields
    int pred;
    void* x;
    void* y;
    void* z;
    void* w;
    void* v;
    const void* r0;
    SpinCoef coef;
    // bytes between right-hand sides of each operand
    int64_t st_x, st_y, st_z, st_w, st_v, st_r0;
    RedArgs r;
    Ctl* ctl;
    int gx;                 // planned grid.x (batched launches)
};

hipError_t launch_blas(int prec, int op, const BlasArgs& a, int nrhs, const Launch& cfg, hipStream_t s);

struct BlasPlan {
    BlasArgs a;
    dim3 grid, block;
    int prec, op, nrhs;
    int nfin, slots;
};
hipError_t plan_blas(int prec, int op, const BlasArgs& a, int nrhs, const Launch& cfg, BlasPlan* out);
hipError_t exec_blas(const BlasPlan& p, hipStream_t s);
hipError_t exec_blas_batch(const BlasPlan* plans, int n, const BlasArgs* tab, const int* offs, int total_blocks,
                           const FinArgs* fin_tab, hipStream_t s);

// Precision conversion of a parity field: dst(prec_dst) = src(prec_src);
// with accumulate, dst += src (dst FP64).  Optional FP64 ||dst||^2 reduction.
struct ConvertArgs {
    int Vh;
    int64_t S;
    int nsub;
    int64_t sub_stride_dst, sub_stride_src;
    int64_t rhs_stride_dst, rhs_stride_src;
    void* dst;
    void* src;
    int accumulate;         // dst += src
    int zero_src;           // src = 0 afterwards
    int pred;
    Ctl* ctl;
    int gx;                 // planned grid.x (batched launches)
};
hipError_t launch_convert(int prec_dst, int prec_src, const ConvertArgs& a, int nrhs, hipStream_t s);

struct ConvertPlan {
    ConvertArgs a;
    dim3 grid, block;
    int pd, ps;
};
hipError_t plan_convert(int prec_dst, int prec_src, const ConvertArgs& a, int nrhs, ConvertPlan* out);
hipError_t exec_convert(const ConvertPlan& p, hipStream_t s);
hipError_t exec_convert_batch(const ConvertPlan* plans, int n, const ConvertArgs* tab, const int* offs, int total_blocks,
                              hipStream_t s);

// Recording: while a recorder is active on the calling thread, launch_dslash,
// launch_blas and launch_convert append their plans instead of launching.
// The solver uses it to record one iteration per system and replay the
// recorded steps of all systems as batched launches.
enum StepKind { STEP_DSLASH = 0, STEP_BLAS = 1, STEP_CONVERT = 2 };
struct Step {
    int kind;
    DslashPlan d;
    BlasPlan b;
    ConvertPlan c;
};
struct Recorder {
    std::vector<Step> steps;
};
Recorder* active_recorder();
void set_recorder(Recorder* r);

// Canonical complex128 <-> internal layouts.
hipError_t launch_pack_spinor(int prec, const Geom& g, const void* canon, void* out, int nrhs, hipStream_t s);
hipError_t launch_unpack_spinor(int prec, const Geom& g, const void* in, void* canon, int nrhs, hipStream_t s);
// The twisted-mass pseudo-fermion force of full-lattice FP64 fields X and Wf
// (Z = gamma_5 Wf) into canonical F[mu][site][3][3]: F = scale * force
// (accumulate = 0) or F += scale * force.
hipError_t launch_tm_force(int recon, const Geom& g, const void* U, const void* X, const void* Wf, void* F,
                           double kappa, double scale, int accumulate, hipStream_t s);
hipError_t launch_pack_colour(int prec, const Geom& g, const void* canon, void* out, int nrhs, hipStream_t s);
hipError_t launch_unpack_colour(int prec, const Geom& g, const void* in, void* canon, int nrhs, hipStream_t s);
hipError_t launch_pack_gauge(int prec, int recon, const Geom& g, const void* canon, void* out, hipStream_t s);
// Re-encode an internal FP64/18 gauge field at another precision / recon.
hipError_t launch_convert_gauge(int prec, int recon, const Geom& g, const void* U64, int src_recon, void* out,
                                hipStream_t s);

// Fill memory with zero bytes through a kernel (graph-capture safe).
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);

// ---- persistent batched solver (persist.hip)
// Block routines a phase of the persistent kernel runs: the steps of the
// mixed-precision CGNR iteration with FP32/12 inner and FP64/18 outer hops on
// several right-hand sides (tile 1, cached links).
enum PRoutine {
    PR_HOP32_12_D0_NONE = 0,
    PR_HOP32_12_D0_NORM,
    PR_HOP32_12_D1_NONE,
    PR_HOP32_12_D1_NORM,
    PR_HOP64_18_D0_NONE,
    PR_HOP64_18_D0_NORM,
    PR_BLAS32_CG_XR,
    PR_BLAS32_CG_P,
    PR_CONV64_32_ACC,
    PR_CONV32_64,
    PR_NONE = -1,
};
constexpr int kPersistThreads = 256;   // block size of the persistent kernel
constexpr int kMaxPersistSteps = 32;

// One step of the batched iteration as a phase: its routine, the blocks of
// all systems (total along x, each system's range starting at offs[s]; gy
// along y), the per-system argument table, and the finalize of its
// reduction (nfin values, per-system FinArgs; 0: none).
struct PStep {
    int routine;
    int total;
    int gy;
    int nfin;
    int pred;  // the step's predicate (the same for every system)
    const void* tab;
    const int* offs;
    const FinArgs* fin;
};

struct PProgram {
    PStep step[kMaxPersistSteps];
    int nsteps;
    int nsys, nrhs;
    int ctl_stride;        // control block of system s, right-hand side r: ctl[s * ctl_stride + r]
    Ctl* ctl;
    int max_iter;          // iterations this launch may run
    int spin_limit;        // polls of a barrier word before the kernel gives up
    unsigned* bar;         // arrival slots [kMaxPersistBlocks], then release slots (zero before the launch)
    int* flag;             // [0] give-up request from the host, [1] a barrier gave up (zero before the launch)
};

// Largest grid of the persistent kernel (one arrival and one release slot each).
constexpr int kMaxPersistBlocks = 2048;

// Blocks the device keeps resident at once for the persistent kernel
// (hipErrorNotSupported without cooperative launch).
hipError_t persistent_grid(int* blocks);
// Cooperative launch of the persistent kernel on prog_dev (device memory).
hipError_t launch_batch_persistent(const PProgram* prog_dev, int blocks, hipStream_t s);
// Zero the nslots barrier slots at words and set the two flags after them to
// (give_up, 0), with a kernel (capturable without a memset node).
hipError_t launch_persist_reset(unsigned* words, int nslots, int give_up, hipStream_t s);

// Initialise control blocks on the device (every right-hand side from in;
// the short form: a plain or reliable-update solve without stagnation
// handling or outer steps).
hipError_t launch_ctl_init(Ctl* ctl, int nrhs, const CtlInit& in, hipStream_t s);
hipError_t launch_ctl_init(Ctl* ctl, int nrhs, double tol, double delta, int iter_limit, hipStream_t s);
// Multi-shift control blocks: ctl[i].sigma = shifts[i] - shifts[base],
// ms_index = i, ms_n = n, ms_base = base (after launch_ctl_init).
constexpr int kMaxShifts = 32;
struct ShiftList {
    double s[kMaxShifts];
};
hipError_t launch_ctl_init_shifts(Ctl* ctl, int n, int base, const ShiftList& shifts, hipStream_t s);
// Re-open the solves whose bit is set in mask (done = 0, status = 0) after a
// failed true-residual check or a fall back to FP32 storage (no_fallback:
// the reopened solves may not fall back again).
hipError_t launch_ctl_reopen(Ctl* ctl, int nrhs, unsigned mask, hipStream_t s, bool no_fallback = false);

}  // namespace lqcd
