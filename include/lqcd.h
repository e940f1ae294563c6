/*
 * lqcd.h - C ABI of the MI355X (gfx950) Wilson / twisted-mass Wilson
 * Dslash and Krylov solver library.
 *
 * The operation is the inversion D phi = psi of the lattice fermion matrix
 * with Krylov methods, whose cost is dominated by repeated applications of
 * the Wilson Dslash (arxiv 1411.5219, section 1; twisted-mass Wilson
 * fermions: section 3; measured Dslash bandwidth: section 6).  The paper
 * prints no formulas; the library implements the standard forms below.
 *
 * Operator (mu = 0,1,2,3 are x,y,z,t):
 *   (H psi)(x) = sum_mu [ (1 - gamma_mu) U_mu(x) f+ psi(x + mu)
 *                       + (1 + gamma_mu) U_mu(x - mu)^+ f- psi(x - mu) ]
 *   M = 1 + 2 i kappa mu gamma_5 - kappa H         (mu = 0: plain Wilson)
 *   M^+ = 1 - 2 i kappa mu gamma_5 - kappa H^+, H^+ swaps the projector signs.
 * f+ = exp(i theta_mu) on hops that cross the boundary forwards (x_mu = L_mu - 1),
 * f- = exp(-i theta_mu) on hops that cross it backwards (x_mu = 0), 1 otherwise;
 * theta = (0, 0, 0, pi) is periodic in space and antiperiodic in time.
 * Gamma matrices in the chiral basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]
 * (k = x, y, z), gamma_t = [[0, 1], [1, 0]], gamma_5 = diag(1, 1, -1, -1).
 *
 * Even-odd: parity of a site is (x + y + z + t) mod 2, even = 0.  With
 * A = 1 + 2 i kappa mu gamma_5 the Schur complement on even sites is
 *   Mhat = A - kappa^2 H_eo A^-1 H_oe.
 *
 * Memory: every field pointer is a DEVICE pointer owned by the caller, in
 * the library's internal layout (structure of arrays, split by parity; sizes
 * from lqcd_field_bytes).  lqcd_pack_* / lqcd_unpack_spinor convert from /
 * to the canonical layout:
 *   gauge  complex128 U[4][V][3][3]  (link from site to site + mu, row, column)
 *   spinor complex128 psi[V][4][3]   (spin, colour), site = x + Lx*(y + Ly*(z + Lz*t)),
 *          nrhs fields stacked: psi[nrhs][V][4][3].
 * The library never allocates or frees caller memory; scratch comes from a
 * caller workspace of lqcd_workspace_bytes() bytes (device memory).  A
 * small pinned host buffer per thread is kept for reading back solver status.
 *
 * Streams: `stream` is a hipStream_t (NULL = default stream).  dslash_* and
 * pack calls only enqueue work and return.  Solvers return once x is final
 * on the device and *info is filled.
 *
 * Errors: functions return LQCD_OK (0) or a negative code; the message of
 * the last error on the calling thread is lqcd_last_error().  Arguments are
 * validated before any device work is enqueued.
 */
#ifndef LQCD_H
#define LQCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LQCD_API __attribute__((visibility("default")))

enum {
    LQCD_OK = 0,
    LQCD_EINVAL = -1,        /* null pointer, bad extent (< 2 or odd), bad nrhs or parameter */
    LQCD_EUNSUPPORTED = -2,  /* precision / recon combination not built (FP16 needs recon 12) */
    LQCD_ENOCONV = -3,       /* maxiter reached: x holds the last iterate, info is valid */
    LQCD_EBREAKDOWN = -4,    /* BiCGStab breakdown (rho = 0 or omega = 0) */
    LQCD_ENONFINITE = -5,    /* NaN or Inf met (source or recursion) */
    LQCD_EHIP = -6           /* HIP runtime error */
};

enum { LQCD_PREC_64 = 64, LQCD_PREC_32 = 32, LQCD_PREC_16 = 16 };
enum { LQCD_RECON_18 = 18, LQCD_RECON_12 = 12 };
enum { LQCD_OP_HOP = 0, LQCD_OP_SCHUR = 1, LQCD_OP_NORMAL = 2 };
enum {
    LQCD_FIELD_SPINOR_PARITY = 0,
    LQCD_FIELD_SPINOR_FULL = 1,
    LQCD_FIELD_GAUGE = 2,
    LQCD_FIELD_COLOUR_PARITY = 3,  /* staggered colour vector, one parity */
    LQCD_FIELD_COLOUR_FULL = 4     /* staggered colour vector, full lattice */
};

/* Lattice extents (x, y, z, t; all even, >= 2) and boundary phases:
 * psi(x + L_mu mu-hat) = exp(i theta_mu) psi(x). */
typedef struct {
    int32_t L[4];
    double theta[4];
} lqcd_geom;

/* kappa, twisted mass a*mu (lattice units), and the storage of the fields
 * handed to dslash_apply / dslash_eo_apply: prec 64, 32 or 16 (FP16 storage
 * with FP32 arithmetic), recon 18 (full links) or 12 (two rows; the third
 * is rebuilt as conj(row0 x row1), valid for SU(3) links). */
typedef struct {
    double kappa;
    double mu;
    int32_t prec;
    int32_t recon;
} lqcd_op;

/* Solver parameters.
 *   tol            stop when ||b - M x||_2 / ||b||_2 <= tol (full system, FP64)
 *   maxiter        iteration limit (inner iterations for mixed precision)
 *   eo             1: even-odd Schur complement; 0: full lattice
 *   inner_prec     64: plain FP64; 32 or 16: mixed precision with an inner
 *                  Dslash in FP32 or FP16 storage and FP64 reliable updates
 *   inner_recon    18 or 12: links of the inner Dslash (built from the FP64
 *                  links, 18- or 12-real, at the start of the solve)
 *   nrhs           right-hand sides (1..16), solved together
 *   delta_reliable reliable-update trigger (||r_low|| < delta * max ||r_low||
 *                  since the last update), in (0, 1)
 * Mixed precision only (the inner solve is CGNR at low precision inside an
 * outer FP64 defect correction; reliable updates fold the low-precision x
 * into the FP64 x and replace the low-precision residual by the FP64 one):
 *   tol_inner      0: one outer step (the search direction survives every
 *                  reliable update); in (0, 1): an outer step ends when
 *                  ||r_low|| <= tol_inner ||r|| of the step's start, and the
 *                  next starts from the FP64 residual with a fresh search
 *                  direction
 *   stag_window    stagnation test of the inner solve: stag_window iterations
 *                  without a reliable update (no reduction of ||r_low|| by
 *                  delta) count as a stagnation, and so does a reliable update
 *                  whose FP64 residual is not below the previous one; each
 *                  stagnation restarts the search direction at the next
 *                  update.  0: 500 iterations; < 0: no iteration window
 *   max_stagnations inner_prec 16: after this many stagnations the solve
 *                  continues from its current x with FP32 inner storage (the
 *                  workspace then holds FP32 inner fields).  0: 3; < 0: never.
 *                  Batched solves (cg_solve_batch) never fall back.
 *   use_graph      1: replay iterations from a captured HIP graph
 *   check_every    iterations enqueued between status read-backs (>= 1; near
 *                  convergence fewer, as many as the residual's rate of
 *                  decrease says are left, except with use_graph)
 *   persistent     cg_solve_batch only (other solvers: 0).  0: every step of
 *                  an iteration is one batched launch (replayed from a graph
 *                  with use_graph); 1: all iterations run in one persistent
 *                  cooperative launch (grid barriers between the steps, no
 *                  host round trip until every system is done; needs nrhs >= 2,
 *                  inner FP32/12 and outer 18-real links, else
 *                  LQCD_EUNSUPPORTED; with use_graph the reset of the barrier
 *                  words and the cooperative launch are captured once per call
 *                  and replayed at each start); 2: as 1 with the kernel's give-up word
 *                  set at launch, so that its first grid barrier gives up and
 *                  the call fails with LQCD_EHIP (the failure path, for tests)
 *   bicgstab_ell   bicgstab_solve only (the other solvers ignore it; values
 *                  outside {0, 1, 2} are LQCD_EINVAL everywhere).  0 or 1:
 *                  BiCGStab; 2: BiCGStab(2) (Sleijpen and Fokkema 1993):
 *                  cycles of two BiCG steps and a minimal-residual polynomial
 *                  of degree 2, which keeps converging on spectra with complex
 *                  eigenvalue pairs where BiCGStab's degree-1 factors stall.
 *                  info.iters counts BiCG steps (2 per cycle, each 2
 *                  applications of the operator, as one BiCGStab iteration);
 *                  maxiter bounds the same count; FP64 only (inner_prec 64) */
typedef struct {
    double tol;
    int32_t maxiter;
    int32_t eo;
    int32_t inner_prec;
    int32_t inner_recon;
    int32_t nrhs;
    int32_t use_graph;
    double delta_reliable;
    int32_t check_every;
    int32_t stag_window;
    double tol_inner;
    int32_t max_stagnations;
    int32_t persistent;
    int32_t bicgstab_ell;
} lqcd_solve_params;

/* Filled by the solvers (one per right-hand side / system). */
typedef struct {
    int32_t status;            /* mirrors the return code */
    int32_t iters;             /* Krylov iterations (inner iterations for mixed precision) */
    int32_t reliable_updates;  /* FP64 residual replacements (mixed precision) */
    int32_t restarts;          /* restarts after a failed true-residual check (multi-shift:
                                  refinement passes of this shift) */
    double true_resid;         /* ||b - M x||_2 / ||b||_2 in FP64, full lattice */
    double seconds;            /* wall time of the call */
    double hops_outer;         /* Dslash applications at the outer (FP64) precision, in units
                                  of one even-odd hop over V/2 output sites */
    double hops_inner;         /* same, at the inner precision (mixed precision only) */
    int32_t outer_iters;       /* outer defect-correction steps (1 + steps ended by tol_inner) */
    int32_t stagnations;       /* stagnations of the inner solve detected */
    int32_t fallbacks;         /* 1: the FP16 inner solve continued at FP32 storage */
    int32_t persistent_launches; /* persistent launches of a batched solve (one per start) */
    double eo_resid;           /* even-odd solves (eo = 1): ||bhat - Mhat x_e||_2 / ||bhat||_2 in FP64,
                                  the even half of b - M x after the reconstruction of x_o;
                                  NaN for full-lattice and staggered solves */
} lqcd_solve_info;

/* Launch configuration of a kernel family (LQCD_KERNEL_DSLASH: the Wilson
 * hop on one right-hand side; LQCD_KERNEL_DSLASH_RHS: the Wilson hop on
 * several stacked right-hand sides, nrhs > 1; LQCD_KERNEL_STAG: the
 * staggered hop, which ignores rhs_tile and rhs_group; LQCD_KERNEL_BLAS: the
 * site-local kernels) at one storage precision:
 *   block   work-items per block (64, 128, 192 or 256; with order = 1 the
 *           requested size, the block then holds whole x-rows)
 *   swizzle 1: block indices are remapped so that each of the 8 XCDs works
 *           on a contiguous range of blocks
 *   order   hop kernels only.  0: blocks walk the sites in memory order;
 *           1: a block covers whole x-rows at one (z, t) and blocks run
 *           t fastest, then z, so neighbour spinors are reused from the
 *           XCD's L2 cache; k in 2..64: the same row blocks in z-slabs of
 *           T planes (T the largest divisor of Lz not above k), z fastest
 *           within a slab, then t, then the slab, which brings the z
 *           neighbours closer in the block order.
 *   rhs_tile Dslash only: right-hand sides one work-item applies each link
 *           to (1, 2 or 4; FP64 at most 2), so links are loaded once per tile.
 *   rhs_group Dslash only: 0, or G in 2..16: with several right-hand-side
 *           tiles, G tiles run back to back on each spatial block, so the
 *           links loaded for the first are re-read from L2 by the others.
 *   ygroup  hop kernels with order = 1: 0 or 1 (none), or G in 2..64: G
 *           neighbouring chunks of x-rows along y run right after t (then z),
 *           so the rows a chunk's y-hops read beyond its edge come from L2;
 *           the largest divisor of the chunk count not above G is used.
 *   rhs_lanes Dslash with rhs_tile = 1 only: 0 or 1 (none), or 2, 4, 8, 16:
 *           the right-hand sides of a site run in that many adjacent lanes of
 *           one wavefront (the next power of two of nrhs, at most this), whose
 *           link loads are one request: each link comes from memory once per
 *           hop for all of them.  Needs order = 1 (blocks of whole x-rows of
 *           sites, block = the site budget times the lanes); where no row
 *           tile fits, the launch uses tiles in registers instead.
 * Process-wide; the defaults come from measurements on MI355X. */
typedef struct {
    int32_t block;
    int32_t swizzle;
    int32_t order;
    int32_t rhs_tile;
    int32_t rhs_group;
    int32_t ygroup;
    int32_t rhs_lanes;
} lqcd_launch;

enum { LQCD_KERNEL_DSLASH = 0, LQCD_KERNEL_BLAS = 1, LQCD_KERNEL_STAG = 2, LQCD_KERNEL_DSLASH_RHS = 3 };

/* Message of the last error on this thread ("" if none). */
LQCD_API const char* lqcd_last_error(void);

/* Library version string. */
LQCD_API const char* lqcd_version(void);

/* The memory clock (kHz) and bus width (bits) the HIP runtime reports for
 * device (the inputs of a nominal HBM peak; the data rate per clock depends
 * on the memory type and is not reported).  EINVAL for NULL outputs, EHIP
 * for a runtime error (e.g. no such device). */
LQCD_API int lqcd_device_memory(int32_t device, int32_t* clock_khz, int32_t* bus_bits);

/* Bytes of one field in the internal layout.  kind: LQCD_FIELD_*; prec and
 * recon as in lqcd_op (recon ignored for spinors).  nrhs fields stacked are
 * nrhs times this size. */
LQCD_API int lqcd_field_bytes(const lqcd_geom* geom, int32_t kind, int32_t prec, int32_t recon, size_t* bytes);

/* Workspace bytes needed by dslash_* (params = NULL) or by a solver call
 * with these parameters. */
LQCD_API int lqcd_workspace_bytes(const lqcd_geom* geom, const lqcd_op* op, const lqcd_solve_params* params,
                         size_t* bytes);

/* Set / read the launch configuration of kernel family `kernel`
 * (LQCD_KERNEL_*) at storage precision prec (64, 32, 16).  Takes effect for
 * calls issued afterwards from any thread. */
LQCD_API int lqcd_set_launch(int32_t kernel, int32_t prec, const lqcd_launch* cfg);
LQCD_API int lqcd_get_launch(int32_t kernel, int32_t prec, lqcd_launch* cfg);

/* Autotune cache (the analogue of the paper's cache of compiled kernels,
 * section 4): launch shapes keyed by the device architecture (gcnArchName
 * without its feature suffix, e.g. "gfx950"), kernel family
 * (LQCD_KERNEL_DSLASH, _STAG or _DSLASH_RHS), storage precision, link
 * reconstruction, lattice extents and right-hand sides.  lqcd_autotune_dslash,
 * lqcd_autotune_dslash_rhs and lqcd_autotune_stag put their winner there
 * (besides the process-wide table of lqcd_set_launch); every later launch of
 * that family on a problem with that key uses the cached shape, which takes
 * precedence over the table (lqcd_autotune_batch tunes for a mix of lattices
 * and writes the table only).  The environment variable LQCD_TUNE_CACHE names
 * a file that is read on first use of the cache (a missing file is an empty
 * cache) and rewritten after every autotuner run.  File format: a JSON array,
 * one object per line, {"arch", "kernel", "prec", "recon", "L": [x, y, z, t],
 * "nrhs", "block", "swizzle", "order", "rhs_tile", "rhs_group", "ygroup",
 * "rhs_lanes", "us"} with "us" the tuned time of one launch.
 *   load : merge a file's entries (EINVAL naming the line for a malformed
 *          entry or an unreadable file; nothing is merged then);
 *   save : write every entry (to a temporary file beside path, then renamed
 *          over it);
 *   clear: drop every entry (and skip a later read of LQCD_TUNE_CACHE);
 *   put  : add or replace one entry (cfg validated as by lqcd_set_launch);
 *   get  : the shape a launch on this key uses: *found = 1 and the cached
 *          shape (and its time in *us, may be NULL), or *found = 0 and the
 *          table's shape.
 * All calls are thread-safe; none touches the device except for reading
 * the current device's architecture ("host" without a device). */
LQCD_API int lqcd_tune_cache_load(const char* path);
LQCD_API int lqcd_tune_cache_save(const char* path);
LQCD_API int lqcd_tune_cache_clear(void);
LQCD_API int lqcd_tune_cache_put(int32_t kernel, int32_t prec, int32_t recon, const lqcd_geom* geom, int32_t nrhs,
                                 const lqcd_launch* cfg, double us);
LQCD_API int lqcd_tune_cache_get(int32_t kernel, int32_t prec, int32_t recon, const lqcd_geom* geom, int32_t nrhs,
                                 lqcd_launch* cfg, double* us, int32_t* found);

/* Autotuner: time every Dslash launch configuration (block 64..256, XCD
 * remap on/off, memory or row-tile order) on this geometry with HIP events,
 * `reps` launches each after two warm-up launches, and install the fastest
 * as the process-wide setting for op->prec.  U, in, out are as for
 * dslash_eo_apply with op_kind = LQCD_OP_HOP, out_parity 0, nrhs 1 (in and out
 * are scratch; out is overwritten).  best / best_us (optional) receive the
 * choice and its mean launch time in microseconds.  Synchronises stream. */
LQCD_API int lqcd_autotune_dslash(const lqcd_geom* geom, const lqcd_op* op, const void* U, const void* in, void* out,
                                  int32_t reps, void* stream, lqcd_launch* best, double* best_us);

/* For several right-hand sides: with the XCD remap and block order of
 * LQCD_KERNEL_DSLASH_RHS at op->prec kept, times the even-odd hop on nrhs
 * (2..16) stacked parity fields for every block request (128, 192, 256),
 * right-hand-side tile compiled (1, 2, 4; FP64 1, 2) and group (0, 2, 4, 8,
 * 16), and tile 1 across 2, 4, 8, 16 lanes (up to the next power of two of
 * nrhs; with order >= 1), and installs the fastest as LQCD_KERNEL_DSLASH_RHS.
 * best_us: mean time of one launch over all nrhs.  Synchronises stream. */
LQCD_API int lqcd_autotune_dslash_rhs(const lqcd_geom* geom, const lqcd_op* op, const void* U, const void* in,
                                      void* out, int32_t nrhs, int32_t reps, void* stream, lqcd_launch* best,
                                      double* best_us);

/* Canonical complex128 gauge field (device) -> internal layout at prec/recon. */
LQCD_API int lqcd_pack_gauge(const lqcd_geom* geom, int32_t prec, int32_t recon, const void* U_canonical, void* U_out,
                    void* stream);

/* Canonical complex128 spinors (device, nrhs stacked) -> internal full-lattice
 * fields at prec, and back. */
LQCD_API int lqcd_pack_spinor(const lqcd_geom* geom, int32_t prec, int32_t nrhs, const void* psi_canonical, void* out,
                     void* stream);
LQCD_API int lqcd_unpack_spinor(const lqcd_geom* geom, int32_t prec, int32_t nrhs, const void* in, void* psi_canonical,
                       void* stream);

/* out = M in (dagger = 0) or M^+ in (dagger = 1) on the full lattice; in and
 * out are nrhs stacked full-lattice fields at op->prec, U at op->prec /
 * op->recon.  in and out must not overlap.
 * Paper: section 1 (the Dslash is the kernel the inversion repeats), section 3
 * (twisted-mass Wilson fermions), section 6 (Dslash bandwidth). */
LQCD_API int dslash_apply(const lqcd_geom* geom, const lqcd_op* op, const void* U, const void* in, void* out,
                 int32_t dagger, int32_t nrhs, void* ws, void* stream);

/* Even-odd pieces on parity fields (nrhs stacked):
 *   op = LQCD_OP_HOP  : out = H_{p,1-p} in, the pure hopping term onto
 *                       parity p = out_parity (in holds parity 1 - p);
 *   op = LQCD_OP_SCHUR: out = Mhat in (dagger: Mhat^+ in) on even sites;
 *                       out_parity must be 0; needs ws.
 * in and out must not overlap.
 * Paper: section 1 and section 6 (the Dslash and its bandwidth; the hop is the
 * kernel the section 6 measurement times), section 3 (twisted mass). */
LQCD_API int dslash_eo_apply(const lqcd_geom* geom, const lqcd_op* op, const void* U, const void* in, void* out,
                    int32_t out_parity, int32_t op_kind, int32_t dagger, int32_t nrhs, void* ws, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation and arguments as dslash_eo_apply, without ws.  LQCD_OP_SCHUR keeps
 * its odd-parity temporary (nrhs parity fields at op->prec) in one 64 MiB
 * array of device memory that the library holds per GPU until the process
 * ends; a request larger than that fails with LQCD_EINVAL before any device
 * work (FP64 fits nrhs * V/2 up to about 349,000 sites, e.g. 32^3 x 8 with two
 * right-hand sides; FP32 fits 48^3 x 12 with one).  The first call on a
 * device looks up that device's copy of the array.  Every call on one GPU
 * uses the same array: calls that overlap in time on one GPU (other streams
 * or threads) race and must be serialised by the caller.  No hipMalloc,
 * hipFree or other allocation. */
LQCD_API int dslash_eo_apply_noalloc(const lqcd_geom* geom, const lqcd_op* op, const void* U, const void* in,
                                     void* out, int32_t out_parity, int32_t op_kind, int32_t dagger, int32_t nrhs,
                                     void* stream);

/* Solve M x = b (nrhs stacked full-lattice FP64 fields, U internal FP64 at
 * op->recon; op->prec must be 64) by CG on the normal equations (CGNR),
 * tracking r = b - M x; stops on the FP64 true residual.  x is overwritten
 * (initial guess ignored).  info: nrhs entries.
 * Paper: section 1 (inversion of the fermion matrix by Krylov methods such as
 * CG dominates the cost), section 3 (standard inversion algorithms). */
LQCD_API int cg_solve(const lqcd_geom* geom, const lqcd_op* op, const void* U, const void* b, void* x,
             const lqcd_solve_params* params, lqcd_solve_info* info, void* ws, size_t ws_bytes, void* stream);

/* Same contract, BiCGStab on M (or on Mhat with eo = 1); BiCGStab(2) with
 * params->bicgstab_ell = 2 (workspace: 9 FP64 vectors per right-hand side
 * with eo, 7 without, against BiCGStab's 8 and 6).
 * Paper: section 3 (standard inversion algorithms). */
LQCD_API int bicgstab_solve(const lqcd_geom* geom, const lqcd_op* op, const void* U, const void* b, void* x,
                   const lqcd_solve_params* params, lqcd_solve_info* info, void* ws, size_t ws_bytes,
                   void* stream);

/* Batched CGNR over nsys independent systems (1..16), e.g. lattices of
 * different volumes with their own kappa, mu and links: system s is solved as
 * cg_solve would with geoms[s], ops[s], U[s], b[s], x[s] and the shared
 * params (nrhs right-hand sides each).  Every kernel of an iteration is
 * launched once for all systems (per-system arguments come from tables in
 * the workspace), and with params->use_graph the iterations are replayed from
 * a captured HIP graph; each system stops on its own FP64 true residual.
 * info: nsys * nrhs entries, system-major.  ws: lqcd_workspace_bytes_batch
 * bytes of device memory.  With params->persistent = 1 the whole iteration
 * loop is one cooperative launch per start (see lqcd_solve_params).
 * Paper: section 1 (finite-temperature studies scan many parameter sets and
 * volumes in parallel), section 4 (kernels specialised at run time). */
LQCD_API int lqcd_workspace_bytes_batch(int32_t nsys, const lqcd_geom* geoms, const lqcd_op* ops,
                                        const lqcd_solve_params* params, size_t* bytes);
LQCD_API int cg_solve_batch(int32_t nsys, const lqcd_geom* geoms, const lqcd_op* ops, const void* const* U,
                            const void* const* b, void* const* x, const lqcd_solve_params* params,
                            lqcd_solve_info* info, void* ws, size_t ws_bytes, void* stream);

/* Autotuner of a batch: times `iters` (1..1000) iterations of the batched
 * CGNR that cg_solve_batch runs on exactly these systems (batched launches,
 * no graph) for each candidate launch shape of the inner hop family
 * (LQCD_KERNEL_DSLASH_RHS at params->inner_prec when params->nrhs > 1: block
 * requests 128, 192, 256 x right-hand-side tile 1 or 2 x tile groups 0..8;
 * LQCD_KERNEL_DSLASH when nrhs = 1: block x memory order / row tiles x XCD
 * remap), keeps the fastest in the process-wide table for later solves and
 * returns it in *best with the time of one iteration in *best_us (either may
 * be NULL).  Arguments as for cg_solve_batch (params->persistent must be 0);
 * x and ws are scratch (x is overwritten).  Synchronises stream.  On an error
 * the table keeps its previous entry.
 * Paper: section 4 (kernels specialised at run time for the problem at hand). */
LQCD_API int lqcd_autotune_batch(int32_t nsys, const lqcd_geom* geoms, const lqcd_op* ops, const void* const* U,
                                 const void* const* b, void* const* x, const lqcd_solve_params* params, void* ws,
                                 size_t ws_bytes, int32_t iters, void* stream, lqcd_launch* best, double* best_us);

/* ------------------------------------------------------------------------
 * Staggered (Kogut-Susskind) fermions.
 *
 * The paper (section 3) adds the standard staggered formulation and
 * (section 1) counts its derivative part D_KS at 570 flops and 1584 bytes
 * per site.  Operator (one colour vector, 3 complex, per site; the same
 * gauge field, layout and boundary phases as the Wilson operator):
 *
 *   (D chi)(x) = 1/2 sum_mu eta_mu(x) [ f+ U_mu(x) chi(x + mu) - f- U_mu(x - mu)^+ chi(x - mu) ]
 *   eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y), eta_3 = (-1)^(x+y+z)
 *   M = m + D,  M^+ = m - D  (D is anti-Hermitian)
 *
 * Colour fields: canonical (V, 3) complex128 per right-hand side, site index
 * x + Lx (y + Ly (z + Lz t)); internal layout per parity (FP64: 3 planes of
 * double2; FP32: a plane of float4 and one of float2; FP16: one plane of 16
 * bytes holding 6 scaled halves and the FP32 scale); a full-lattice field is
 * the even parity followed by the odd one.  Sizes: lqcd_field_bytes with
 * LQCD_FIELD_COLOUR_PARITY / LQCD_FIELD_COLOUR_FULL. */
typedef struct {
    double mass;      /* bare mass m (lattice units); the solvers need m > 0 */
    int32_t prec;     /* 64, 32 or 16 (FP16 storage, FP32 arithmetic) */
    int32_t recon;    /* 18 or 12 (FP16: 12) */
} lqcd_stag_op;

/* Canonical <-> internal colour fields (nrhs stacked full-lattice fields). */
LQCD_API int lqcd_pack_colour(const lqcd_geom* geom, int32_t prec, int32_t nrhs, const void* chi_canonical, void* out,
                              void* stream);
LQCD_API int lqcd_unpack_colour(const lqcd_geom* geom, int32_t prec, int32_t nrhs, const void* in,
                                void* chi_canonical, void* stream);

/* out = M in (dagger = 0) or M^+ in (dagger = 1) on the full lattice, nrhs
 * stacked full-lattice colour fields at op->prec; in and out must not
 * overlap.  Enqueues only. */
LQCD_API int stag_apply(const lqcd_geom* geom, const lqcd_stag_op* op, const void* U, const void* in, void* out,
                        int32_t dagger, int32_t nrhs, void* stream);

/* Even-odd pieces on parity colour fields (nrhs stacked):
 *   op = LQCD_OP_HOP    : out = D_{p,1-p} in onto parity p = out_parity;
 *   op = LQCD_OP_NORMAL : out = (m^2 - D_eo D_oe) in on even sites, the even
 *                         block of M^+ M (Hermitian positive definite for
 *                         m > 0); out_parity must be 0; ws must hold
 *                         nrhs odd parity fields at op->prec.
 * in and out must not overlap. */
LQCD_API int stag_eo_apply(const lqcd_geom* geom, const lqcd_stag_op* op, const void* U, const void* in, void* out,
                           int32_t out_parity, int32_t op_kind, int32_t nrhs, void* ws, void* stream);

/* Times the staggered even-odd hop (LQCD_OP_HOP, out_parity 0, nrhs 1) in
 * the same 16 launch shapes as lqcd_autotune_dslash and keeps the fastest
 * for LQCD_KERNEL_STAG at op->prec; in and out are parity colour fields
 * (scratch; out is overwritten).  Synchronises stream. */
LQCD_API int lqcd_autotune_stag(const lqcd_geom* geom, const lqcd_stag_op* op, const void* U, const void* in,
                                void* out, int32_t reps, void* stream, lqcd_launch* best, double* best_us);

/* Device workspace (bytes) of stag_cg_solve (nshift = 0) or of
 * stag_multishift_solve with nshift shifts (1..32). */
LQCD_API int lqcd_workspace_bytes_stag(const lqcd_geom* geom, const lqcd_stag_op* op, int32_t nshift, size_t* bytes);

/* Staggered D_KS (paper: section 3, staggered fermions; section 6, the
 * D_KS kernel's bandwidth).
 * Solve M x = b for one full-lattice FP64 colour field b (U FP64 at
 * op->recon, op->prec = 64, op->mass > 0): CG on the even-site normal
 * operator N = m^2 - D_eo D_oe with right-hand side m b_e - D_eo b_o, then
 * x_o = (b_o - D_oe x_e) / m.  The CG residual r_e of N gives the full one,
 * ||b - M x|| = ||r_e|| / m, so CG stops at ||r_e|| <= tol m ||b||; the FP64
 * true residual of the full system is then checked and CG restarts from the
 * current x if it misses.  params: eo = 1, inner_prec = 64, nrhs = 1 (other
 * fields as for cg_solve).  x is overwritten.  info: one entry. */
LQCD_API int stag_cg_solve(const lqcd_geom* geom, const lqcd_stag_op* op, const void* U, const void* b, void* x,
                           const lqcd_solve_params* params, lqcd_solve_info* info, void* ws, size_t ws_bytes,
                           void* stream);

/* Multi-shift CG (the inversions a rational approximation needs): solve
 * (N + shifts[i]) x_i = b for every shift at once, b one even-parity FP64
 * colour field, x nshift even-parity fields stacked (x_i at byte offset
 * i * lqcd_field_bytes(COLOUR_PARITY, 64)), shifts >= 0 in any order (1..32
 * of them).  One Krylov space, the smallest shift as the base system; each
 * system leaves the shared recursion when its recursive residual
 * ||b - (N + shift_i) x_i|| falls to tol ||b||.  Its FP64 true residual is
 * then recomputed; a shift that misses tol (rounding of the shifted
 * recurrences) is refined by single-shift CG on N + shift_i started from x_i
 * (up to 4 passes, counted in info[i].restarts, its iterations added to
 * info[i].iters).  info[i].status is LQCD_OK only when info[i].true_resid <=
 * tol, else LQCD_ENOCONV (the call returns the first failing status).
 * params: tol, maxiter, use_graph, check_every as for cg_solve; eo = 1,
 * inner_prec = 64, nrhs = 1.
 * Paper: section 3 (RHMC for staggered fermions, whose rational
 * approximation needs these shifted inversions). */
LQCD_API int stag_multishift_solve(const lqcd_geom* geom, const lqcd_stag_op* op, const void* U, const void* b,
                                   void* x, const double* shifts, int32_t nshift, const lqcd_solve_params* params,
                                   lqcd_solve_info* info, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * N_f = 2 twisted-mass HMC, fermion part (the paper generates gauge fields
 * with HMC, §3, the determinant entering through pseudo-fermions that need
 * the inverse of M, §1).  Pseudo-fermion action S_f = ||M^-1 phi||^2; its
 * force along U_mu(y) -> exp(i w T^a) U_mu(y), T^a = lambda_a / 2, is
 * F_mu(y) = sum_a (dS_f / dw^a) T^a (3x3 Hermitian, traceless):
 *
 *   X = M^-1 phi,  Wf = M(-mu)^-1 gamma_5 X  (so Z = gamma_5 Wf = (M^+)^-1 X)
 *   W = f+ U_mu(y) A - f- B U_mu(y)^+
 *   A = sum_s [(1 - gamma_mu) X(y + mu)]_s Z_s(y)^+,  B = sum_s X_s(y) [(1 + gamma_mu) Z(y + mu)]_s^+
 *   F_mu(y) = (i kappa / 2) [(W - W^+) - tr(W - W^+) / 3]
 *
 * (f+- the boundary phases of the forward hop from y and of the backward hop
 * from y + mu). */

/* out = gamma_5 in (chiral basis: diag(1, 1, -1, -1) on spin), nrhs stacked
 * full-lattice FP64 spinor fields; in and out may be the same field. */
LQCD_API int lqcd_gamma5(const lqcd_geom* geom, int32_t nrhs, const void* in, void* out, void* stream);

/* F = scale * force (accumulate = 0) or F += scale * force (accumulate = 1);
 * X and Wf full-lattice FP64 spinor fields (internal layout), U FP64 at
 * op->recon (op->prec = 64), F device memory in the canonical layout
 * F[mu][site][3][3] complex128, site = x + Lx (y + Ly (z + Lz t)), caller
 * owned (4 * V * 144 bytes), not overlapping X, Wf or U.  EINVAL for a NULL
 * pointer, op->prec != 64, accumulate not 0 or 1, a non-finite scale, or a
 * lattice whose full-lattice FP64 spinor field or one direction of F would
 * reach 2 GiB (about 11 million sites; 64^3 x 32 fits).  Enqueues only. */
LQCD_API int tm_force(const lqcd_geom* geom, const lqcd_op* op, const void* U, const void* X, const void* Wf,
                      void* F, double scale, int32_t accumulate, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LQCD_H */
