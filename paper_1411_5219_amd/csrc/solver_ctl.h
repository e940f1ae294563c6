// The device-resident control block of one Krylov solve and the scalar step
// of each solver, run once the reductions of a kernel are summed.
//
// Plain C++: compiled into the library by hipcc (host and device) and, for
// the tests of the trigger logic, by a host compiler alone.  The solvers:
//   CGNR (Saad, the CGNR algorithm), optionally with an inner solve at low
//     precision and FP64 reliable updates (Sleijpen and van der Vorst 1996,
//     residual replacement), an outer defect correction, stagnation
//     detection and a fall back from FP16 to FP32 storage;
//   BiCGStab (van der Vorst 1992) and BiCGStab(2) (Sleijpen and Fokkema
//     1993, two BiCG steps and a minimal-residual polynomial of degree 2);
//   the multi-shift CG (Jegerlehner 1996, shift added to the operator).
// The paper names the inversion with Krylov methods as the dominant cost
// (section 1) and standard inversion algorithms (section 3); the solvers
// themselves are the textbook methods.
#pragma once

#include <stdint.h>

#include "lqcd.h"

#if defined(__HIPCC__)
#define LQCD_HD __host__ __device__
#else
#define LQCD_HD
#endif

namespace lqcd {

// What the finalize of a reduction does with its totals.
enum Fin {
    FIN_STORE = 0,        // copy totals to Ctl::red[]
    FIN_CG_ZZ = 1,        // zz = ||z||^2 (start of CGNR)
    FIN_CG_ALPHA = 2,     // ww = ||w||^2, alpha = zz / ww
    FIN_CG_RR = 3,        // rr = ||r||^2, iteration done: convergence / reliable-update / stagnation tests
    FIN_CG_BETA = 4,      // zz' = ||z'||^2, beta = zz' / zz (0 when the search direction restarts), zz = zz'
    FIN_TRUE_RR = 5,      // true_rr = ||b - M x||^2 (FP64)
    FIN_BI_ALPHA = 6,     // alpha = rho / <r0, v>
    FIN_BI_OMEGA = 7,     // omega = <t, s> / ||t||^2 (||t|| = 0: s is the exact residual of x + alpha p)
    FIN_BI_RHO = 8,       // rr, rho = <r0, r>, convergence / breakdown test
    FIN_BI_INIT = 9,      // rr and rho at the start of BiCGStab
    FIN_RU_RR = 10,       // reliable update: rr = ||r||^2 in FP64 after the update
    FIN_BB_E = 11,        // red[0] = ||b_e||^2 (first half of ||b||^2)
    FIN_BB = 12,          // bb = red[0] + ||b_o||^2, thresh = tol^2 * bb
    FIN_BB_FULL = 13,     // bb = ||b||^2 of a full-lattice field, thresh = tol^2 * bb
    FIN_RR_INIT = 14,     // rr = rr_max = ||r||^2 (start of a reliable-update solve)
    // multi-shift CG, run by the base system's finalize for every shift
    FIN_MS_INIT = 15,     // rr = ||b||^2 = bb of every shift, thresh = tol^2 bb, zeta = 1
    FIN_MS_INIT_KEEP = 16,// rr = ||r||^2, zeta = 1; bb and thresh already set
    FIN_MS_ALPHA = 17,    // alpha = rr / <p, A p>; zeta_{k+1}, alpha_i of every shift
    FIN_MS_BETA = 18,     // rr' = ||r||^2, beta, beta_i, zeta shift, per-shift convergence
    // BiCGStab(2): one cycle is two BiCG steps (u_1 = A u_0, r_1 = A r_0,
    // u_2 = A u_1, r_2 = A r_1) and the minimal residual over r_1, r_2
    FIN_BL_INIT = 19,     // rr = ||r_0||^2, <rt, r_0>: rho0 = 1, alpha = 0, omega = 1, first cycle's beta
    FIN_BL_ALPHA = 20,    // gamma = <rt, u_{j+1}>, alpha = rho0 / gamma
    FIN_BL_BETA = 21,     // rho1 = <rt, r_1>, beta = alpha rho1 / rho0, rho0 = rho1
    FIN_BL_TAU = 22,      // sigma1 = ||r_1||^2, tau = <r_1, r_2> / sigma1, gp1 = <r_1, r_0> / sigma1
    FIN_BL_OMEGA = 23,    // sigma2 = ||r_2'||^2 (r_2' = r_2 - tau r_1), gp2 = <r_2', r_0> / sigma2: omega, g1, g2
    FIN_BL_RES = 24,      // rr = ||r_0||^2, <rt, r_0>: convergence, next cycle's beta
    FIN_EO_RR = 25,       // eo_rr = ||(b - M x)_e||^2 = ||bhat - Mhat x_e||^2 once x_o is reconstructed
    FIN_BBHAT = 26,       // bbh = ||bhat||^2
};

// Status of a solve that handed control back to the host to continue at FP32
// storage (never returned to a caller: the host restarts the solve).
constexpr int kStatusFallback = 1;

// Device-resident control block of one solve (one per right-hand side).
// Kernels read their scalars from here, so no host round trip is needed
// inside an iteration.
struct Ctl {
    double bb;        // ||b||^2 of the full system (stopping reference)
    double thresh;    // tol^2 * bb
    double zz, ww, rr, alpha, beta;
    double rr_max;    // largest ||r_low||^2 since the last reliable update
    double delta2;    // reliable-update trigger: rr < delta2 * rr_max
    double tol2;      // tol^2
    double true_rr;
    double rho[2], rho_old[2], balpha[2], omega[2], r0v[2], ts[2], tt;
    double omega_step[2];  // omega of the current BiCGStab step (0 in the lucky case)
    double red[6];    // FIN_STORE totals
    // Multi-shift CG (one Ctl per shifted system, ms_n of them in a row; the
    // base system, the smallest shift, at index ms_base): this system's shift
    // minus the base shift and its residual ratios to the base residual,
    // zeta_{k-1}, zeta_k and, inside an iteration, zeta_{k+1}; the base also
    // keeps the base CG's alpha_{k-1} and beta_{k-1}.
    double sigma, zeta_prev, zeta, zeta_next, alpha_prev, beta_prev;
    // Mixed precision: FP64 ||r||^2 at the last reliable update and at the
    // start of the current outer (defect-correction) step, tol_inner^2.
    double rr_prev_upd, rr_outer, tol_inner2;
    // Even-odd solves: ||bhat - Mhat x_e||^2 at the end and ||bhat||^2.
    double eo_rr, bbh;
    // BiCGStab(2) (rho0, rho1, alpha and omega in rho_old, rho, balpha and
    // omega): beta, the Gram-Schmidt coefficient tau = <r_1, r_2> / ||r_1||^2,
    // the projections gp1, gp2 of r_0 on r_1, r_2', and the polynomial
    // coefficients g1, g2 in the basis r_1, r_2 (x += g1 r_0 + g2 r_1,
    // r_0 -= g1 r_1 + g2 r_2, u_0 -= g1 u_1 + g2 u_2)
    double bl_beta[2], bl_tau[2], bl_gp1[2], bl_gp2[2], bl_g1[2], bl_g2[2], bl_sigma1;
    int ms_index, ms_n, ms_base;
    int iter;         // completed iterations
    int done;         // 1 when converged (or failed): every kernel becomes a no-op
    int status;       // 0, a negative LQCD error code, or kStatusFallback
    int update;       // reliable update pending
    int nupdates;     // reliable updates performed
    int iter_limit;   // stop (done, status ENOCONV) at this many iterations
    int lucky;        // BiCGStab: ||t|| = 0 in the current step
    int last_upd_iter;// iteration of the last reliable update (or start)
    int stag_window;  // a stagnation after this many iterations without an update (0: off)
    int max_stag;     // stagnations before an FP16 inner solve falls back to FP32 (0: never)
    int nstag;        // stagnations detected
    int reset_p;      // the pending update discards the search direction
    int outer_req;    // the pending update ends an outer step (tol_inner reached)
    int nouter;       // outer steps ended by tol_inner
    int fallback_ok;  // the inner storage may fall back (FP16 inner)
    int bl_skip;      // BiCGStab(2): r_1 or r_2' vanished, the cycle takes no minimal-residual step
};

// Parameters of a control block at the start of a solve.
struct CtlInit {
    double tol;
    double delta;      // reliable-update threshold (0: plain solve)
    double tol_inner;  // outer step ends at ||r_low|| <= tol_inner ||r_outer|| (0: off)
    int iter_limit;
    int stag_window;
    int max_stag;
    int fallback_ok;
};

LQCD_HD inline Ctl ctl_make(const CtlInit& in)
{
    Ctl c = {};
    c.tol2 = in.tol * in.tol;
    c.delta2 = in.delta * in.delta;
    c.tol_inner2 = in.tol_inner * in.tol_inner;
    c.iter_limit = in.iter_limit;
    c.stag_window = in.stag_window;
    c.max_stag = in.max_stag;
    c.fallback_ok = in.fallback_ok;
    return c;
}

LQCD_HD inline bool finite(double v) { return __builtin_isfinite(v); }

LQCD_HD inline void cdiv(const double* a, const double* b, double* out)
{
    const double d = b[0] * b[0] + b[1] * b[1];
    const double re = (a[0] * b[0] + a[1] * b[1]) / d;
    const double im = (a[1] * b[0] - a[0] * b[1]) / d;
    out[0] = re;
    out[1] = im;
}

LQCD_HD inline void cmul(const double* a, const double* b, double* out)
{
    const double re = a[0] * b[0] - a[1] * b[1];
    const double im = a[0] * b[1] + a[1] * b[0];
    out[0] = re;
    out[1] = im;
}

LQCD_HD inline void fail(Ctl* c, int status)
{
    c->status = status;
    c->done = 1;
}

// A stagnation of the inner solve: the next reliable update restarts the
// search direction; with FP16 storage, max_stag of them hand the solve back
// to the host to continue at FP32 (decided at the update, see FIN_RU_RR).
LQCD_HD inline void stagnation(Ctl* c)
{
    c->nstag += 1;
    c->reset_p = 1;
}

// v holds the reduction totals, zero-padded to 6 entries.  Runs for one
// right-hand side (multi-shift: for every shift of the family) after the
// kernel that produced the partials.
LQCD_HD inline void finalize_totals(int fin, Ctl* c, const double* v)
{
    switch (fin) {
    case FIN_STORE:
        for (int j = 0; j < 6; ++j) c->red[j] = v[j];
        break;
    case FIN_CG_ZZ:
        c->zz = v[0];
        if (!finite(v[0])) fail(c, LQCD_ENONFINITE);
        else if (v[0] == 0.0) c->done = 1;  // r is exactly zero
        break;
    case FIN_CG_ALPHA:
        c->ww = v[0];
        if (!finite(v[0])) fail(c, LQCD_ENONFINITE);
        else if (v[0] == 0.0) c->done = 1;
        else c->alpha = c->zz / v[0];
        break;
    case FIN_CG_RR:
        c->rr = v[0];
        c->iter += 1;
        if (!finite(v[0])) { fail(c, LQCD_ENONFINITE); break; }
        if (c->delta2 > 0.0) {
            // mixed precision: never stop on the low-precision recursion;
            // request an FP64 reliable update instead
            if (v[0] <= c->thresh || v[0] < c->delta2 * c->rr_max) {
                c->update = 1;
            } else {
                if (v[0] > c->rr_max) c->rr_max = v[0];
                // no reduction by delta for stag_window iterations: stagnation
                if (c->stag_window > 0 && c->iter - c->last_upd_iter >= c->stag_window) {
                    c->update = 1;
                    stagnation(c);
                }
            }
            // the inner solve of this outer step reached tol_inner
            if (c->tol_inner2 > 0.0 && v[0] <= c->tol_inner2 * c->rr_outer) {
                c->update = 1;
                c->outer_req = 1;
                c->reset_p = 1;
            }
        } else if (v[0] <= c->thresh) {
            c->done = 1;
            break;
        }
        if (c->iter >= c->iter_limit && !c->update) fail(c, LQCD_ENOCONV);
        break;
    case FIN_CG_BETA:
        if (!finite(v[0])) { fail(c, LQCD_ENONFINITE); break; }
        c->beta = (c->reset_p || !(c->zz > 0.0)) ? 0.0 : v[0] / c->zz;
        c->reset_p = 0;
        c->zz = v[0];
        c->update = 0;
        if (c->iter >= c->iter_limit) fail(c, LQCD_ENOCONV);
        break;
    case FIN_RU_RR:
        c->rr = v[0];
        c->rr_max = v[0];
        c->nupdates += 1;
        c->last_upd_iter = c->iter;
        if (!finite(v[0])) { fail(c, LQCD_ENONFINITE); break; }
        if (v[0] <= c->thresh) { c->done = 1; break; }
        // the FP64 residual did not fall since the previous update: stagnation
        // (unless this update already restarts the search direction)
        if (!c->reset_p && c->rr_prev_upd > 0.0 && v[0] >= c->rr_prev_upd) stagnation(c);
        c->rr_prev_upd = v[0];
        if (c->outer_req) {
            c->nouter += 1;
            c->rr_outer = v[0];
            c->outer_req = 0;
        }
        if (c->fallback_ok && c->max_stag > 0 && c->nstag >= c->max_stag) {
            // x is up to date in FP64: continue from here at FP32 storage
            c->status = kStatusFallback;
            c->done = 1;
        }
        break;
    case FIN_RR_INIT:
        c->rr = v[0];
        c->rr_max = v[0];
        c->rr_prev_upd = v[0];
        c->rr_outer = v[0];
        c->last_upd_iter = c->iter;
        c->reset_p = 0;
        c->outer_req = 0;
        c->update = 0;
        if (!finite(v[0])) fail(c, LQCD_ENONFINITE);
        else if (v[0] <= c->thresh) c->done = 1;
        break;
    case FIN_TRUE_RR:
        c->true_rr = v[0];
        break;
    case FIN_EO_RR:
        c->eo_rr = v[0];
        break;
    case FIN_BBHAT:
        c->bbh = v[0];
        break;
    case FIN_BB_E:
        c->red[0] = v[0];
        break;
    case FIN_BB:
    case FIN_BB_FULL: {
        const double bb = fin == FIN_BB ? c->red[0] + v[0] : v[0];
        c->bb = bb;
        c->thresh = c->tol2 * bb;
        if (!finite(bb)) fail(c, LQCD_ENONFINITE);
        else if (bb == 0.0) c->done = 1;
        break;
    }
    case FIN_BI_INIT:
        c->rr = v[0];
        c->rho[0] = v[1];
        c->rho[1] = v[2];
        c->rho_old[0] = 1.0;
        c->rho_old[1] = 0.0;
        c->balpha[0] = 1.0;
        c->balpha[1] = 0.0;
        c->omega[0] = 1.0;
        c->omega[1] = 0.0;
        c->lucky = 0;
        if (!finite(v[0])) fail(c, LQCD_ENONFINITE);
        else if (v[0] <= c->thresh) c->done = 1;
        break;
    case FIN_BI_ALPHA:
        c->r0v[0] = v[0];
        c->r0v[1] = v[1];
        if (!finite(v[0]) || !finite(v[1])) fail(c, LQCD_ENONFINITE);
        else if (v[0] == 0.0 && v[1] == 0.0) fail(c, LQCD_EBREAKDOWN);
        else cdiv(c->rho, c->r0v, c->balpha);
        break;
    case FIN_BI_OMEGA:
        c->tt = v[0];
        c->ts[0] = v[1];
        c->ts[1] = v[2];
        if (!finite(v[0]) || !finite(v[1]) || !finite(v[2])) { fail(c, LQCD_ENONFINITE); break; }
        if (v[0] == 0.0) {
            // t = M s = 0: s is the exact residual of x + alpha p, which
            // this step takes without the stabilising half (omega = 0 for
            // the update only; rho and omega of the recursion are kept)
            c->lucky = 1;
            c->omega_step[0] = 0.0;
            c->omega_step[1] = 0.0;
        } else {
            c->lucky = 0;
            c->omega_step[0] = v[1] / v[0];
            c->omega_step[1] = v[2] / v[0];
        }
        break;
    case FIN_BI_RHO:
        c->rr = v[0];
        c->iter += 1;
        if (!finite(v[0]) || !finite(v[1]) || !finite(v[2])) { fail(c, LQCD_ENONFINITE); break; }
        if (v[0] <= c->thresh) { c->done = 1; break; }
        if (!c->lucky) {
            c->rho_old[0] = c->rho[0];
            c->rho_old[1] = c->rho[1];
            c->omega[0] = c->omega_step[0];
            c->omega[1] = c->omega_step[1];
        }
        c->rho[0] = v[1];
        c->rho[1] = v[2];
        if ((v[1] == 0.0 && v[2] == 0.0) || (c->omega[0] == 0.0 && c->omega[1] == 0.0)) {
            fail(c, LQCD_EBREAKDOWN);
            break;
        }
        if (c->iter >= c->iter_limit) fail(c, LQCD_ENOCONV);
        break;
    case FIN_BL_INIT:
    case FIN_BL_RES: {
        c->rr = v[0];
        if (fin == FIN_BL_INIT) {
            c->rho_old[0] = 1.0;
            c->rho_old[1] = 0.0;
            c->balpha[0] = 0.0;
            c->balpha[1] = 0.0;
            c->omega[0] = 1.0;
            c->omega[1] = 0.0;
            c->bl_g1[0] = c->bl_g1[1] = c->bl_g2[0] = c->bl_g2[1] = 0.0;
            c->bl_skip = 0;
        } else {
            c->iter += 2;
        }
        if (!finite(v[0]) || !finite(v[1]) || !finite(v[2])) { fail(c, LQCD_ENONFINITE); break; }
        if (v[0] <= c->thresh) { c->done = 1; break; }
        if (c->iter >= c->iter_limit) { fail(c, LQCD_ENOCONV); break; }
        // next cycle: rho0 = -omega rho0, then its first BiCG step's beta
        double r0n[2];
        cmul(c->omega, c->rho_old, r0n);
        r0n[0] = -r0n[0];
        r0n[1] = -r0n[1];
        if (r0n[0] == 0.0 && r0n[1] == 0.0) { fail(c, LQCD_EBREAKDOWN); break; }
        c->rho[0] = v[1];
        c->rho[1] = v[2];
        double q[2];
        cdiv(c->rho, r0n, q);
        cmul(c->balpha, q, c->bl_beta);
        c->rho_old[0] = v[1];
        c->rho_old[1] = v[2];
        break;
    }
    case FIN_BL_ALPHA: {
        const double g[2] = {v[0], v[1]};
        if (!finite(g[0]) || !finite(g[1])) { fail(c, LQCD_ENONFINITE); break; }
        if (g[0] == 0.0 && g[1] == 0.0) { fail(c, LQCD_EBREAKDOWN); break; }
        cdiv(c->rho_old, g, c->balpha);
        break;
    }
    case FIN_BL_BETA: {
        if (!finite(v[0]) || !finite(v[1])) { fail(c, LQCD_ENONFINITE); break; }
        if (c->rho_old[0] == 0.0 && c->rho_old[1] == 0.0) { fail(c, LQCD_EBREAKDOWN); break; }
        c->rho[0] = v[0];
        c->rho[1] = v[1];
        double q[2];
        cdiv(c->rho, c->rho_old, q);
        cmul(c->balpha, q, c->bl_beta);
        c->rho_old[0] = v[0];
        c->rho_old[1] = v[1];
        break;
    }
    case FIN_BL_TAU:
        for (int j = 0; j < 5; ++j)
            if (!finite(v[j])) fail(c, LQCD_ENONFINITE);
        if (c->done) break;
        c->bl_sigma1 = v[0];
        c->bl_skip = v[0] == 0.0;
        if (c->bl_skip) {
            c->bl_tau[0] = c->bl_tau[1] = c->bl_gp1[0] = c->bl_gp1[1] = 0.0;
        } else {
            c->bl_tau[0] = v[1] / v[0];
            c->bl_tau[1] = v[2] / v[0];
            c->bl_gp1[0] = v[3] / v[0];
            c->bl_gp1[1] = v[4] / v[0];
        }
        break;
    case FIN_BL_OMEGA:
        if (!finite(v[0]) || !finite(v[1]) || !finite(v[2])) { fail(c, LQCD_ENONFINITE); break; }
        if (c->bl_skip || v[0] == 0.0) {
            // r_1 = 0 or r_2' = 0: the cycle ends without the minimal residual
            // step (omega kept), as the published algorithm does
            c->bl_skip = 1;
            c->bl_gp1[0] = c->bl_gp1[1] = c->bl_gp2[0] = c->bl_gp2[1] = 0.0;
            c->bl_g1[0] = c->bl_g1[1] = c->bl_g2[0] = c->bl_g2[1] = 0.0;
            break;
        }
        c->bl_gp2[0] = v[1] / v[0];
        c->bl_gp2[1] = v[2] / v[0];
        c->bl_g2[0] = c->bl_gp2[0];
        c->bl_g2[1] = c->bl_gp2[1];
        c->omega[0] = c->bl_g2[0];
        c->omega[1] = c->bl_g2[1];
        {
            double tg[2];
            cmul(c->bl_tau, c->bl_g2, tg);
            c->bl_g1[0] = c->bl_gp1[0] - tg[0];
            c->bl_g1[1] = c->bl_gp1[1] - tg[1];
        }
        break;
    case FIN_MS_INIT:
    case FIN_MS_INIT_KEEP: {
        Ctl* c0 = c - c->ms_index;
        c->rr = v[0];
        c->alpha_prev = 1.0;
        c->beta_prev = 0.0;
        for (int i = 0; i < c->ms_n; ++i) {
            Ctl* ci = c0 + i;
            if (fin == FIN_MS_INIT) {
                ci->bb = v[0];
                ci->thresh = ci->tol2 * v[0];
            }
            ci->zeta_prev = 1.0;
            ci->zeta = 1.0;
            if (!finite(v[0])) fail(ci, LQCD_ENONFINITE);
            else if (v[0] <= ci->thresh) ci->done = 1;
        }
        break;
    }
    case FIN_MS_ALPHA: {
        // v[1] = Re <w, p> = <p, A p> of the base system
        Ctl* c0 = c - c->ms_index;
        const double pap = v[1];
        const bool bad = !finite(pap) || !(pap > 0.0);
        const double al = bad ? 0.0 : c->rr / pap;
        for (int i = 0; i < c->ms_n; ++i) {
            Ctl* ci = c0 + i;
            if (ci->done) continue;
            if (bad) { fail(ci, finite(pap) ? LQCD_EBREAKDOWN : LQCD_ENONFINITE); continue; }
            // zeta_{k+1} = zeta_k zeta_{k-1} alpha_{k-1}
            //   / (alpha_k beta_{k-1} (zeta_{k-1} - zeta_k) + zeta_{k-1} alpha_{k-1} (1 + sigma alpha_k))
            const double den = al * c->beta_prev * (ci->zeta_prev - ci->zeta) +
                               ci->zeta_prev * c->alpha_prev * (1.0 + ci->sigma * al);
            const double zn = ci->zeta * ci->zeta_prev * c->alpha_prev / den;
            if (!finite(zn) || ci->zeta == 0.0) { fail(ci, LQCD_ENONFINITE); continue; }
            ci->zeta_next = zn;
            ci->alpha = al * zn / ci->zeta;
        }
        c->alpha = al;  // the base system's alpha (its zeta is 1)
        break;
    }
    case FIN_MS_BETA: {
        Ctl* c0 = c - c->ms_index;
        const double rr = v[0];
        const double be = c->rr > 0.0 ? rr / c->rr : 0.0;
        const int it = c->iter + 1;
        for (int i = 0; i < c->ms_n; ++i) {
            Ctl* ci = c0 + i;
            if (ci->done) continue;
            if (!finite(rr)) { fail(ci, LQCD_ENONFINITE); continue; }
            const double q = ci->zeta_next / ci->zeta;
            ci->beta = be * q * q;
            ci->zeta_prev = ci->zeta;
            ci->zeta = ci->zeta_next;
            ci->iter = it;
            if (ci->zeta * ci->zeta * rr <= ci->thresh) ci->done = 1;
            else if (it >= ci->iter_limit) fail(ci, LQCD_ENOCONV);
        }
        c->iter = it;
        c->alpha_prev = c->alpha;
        c->beta_prev = be;
        c->rr = rr;
        break;
    }
    default:
        break;
    }
}

}  // namespace lqcd
