// Scalar steps of the Krylov solvers, run by one thread of the last block of
// a reduction kernel once the grand totals are known.  Keeping them on the
// device lets a whole iteration run without a host round trip.
#pragma once

#include "lqcd.h"
#include "lqcd_kernels.h"

namespace lqcd {

__device__ inline bool finite(double v) { return isfinite(v); }

__device__ inline void cdiv(const double* a, const double* b, double* out)
{
    const double d = b[0] * b[0] + b[1] * b[1];
    const double re = (a[0] * b[0] + a[1] * b[1]) / d;
    const double im = (a[1] * b[0] - a[0] * b[1]) / d;
    out[0] = re;
    out[1] = im;
}

__device__ inline void fail(Ctl* c, int status)
{
    c->status = status;
    c->done = 1;
}

// v holds the reduction totals, zero-padded to 6 entries.
__device__ inline void finalize_totals(int fin, Ctl* c, const double* v)
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
            if (v[0] <= c->thresh || v[0] < c->delta2 * c->rr_max) c->update = 1;
            else if (v[0] > c->rr_max) c->rr_max = v[0];
        } else if (v[0] <= c->thresh) {
            c->done = 1;
            break;
        }
        if (c->iter >= c->iter_limit && !c->update) fail(c, LQCD_ENOCONV);
        break;
    case FIN_CG_BETA:
        if (!finite(v[0])) { fail(c, LQCD_ENONFINITE); break; }
        c->beta = c->zz > 0.0 ? v[0] / c->zz : 0.0;
        c->zz = v[0];
        c->update = 0;
        if (c->iter >= c->iter_limit) fail(c, LQCD_ENOCONV);
        break;
    case FIN_RU_RR:
        c->rr = v[0];
        c->rr_max = v[0];
        c->nupdates += 1;
        if (!finite(v[0])) fail(c, LQCD_ENONFINITE);
        else if (v[0] <= c->thresh) c->done = 1;
        break;
    case FIN_RR_INIT:
        c->rr = v[0];
        c->rr_max = v[0];
        if (!finite(v[0])) fail(c, LQCD_ENONFINITE);
        else if (v[0] <= c->thresh) c->done = 1;
        break;
    case FIN_TRUE_RR:
        c->true_rr = v[0];
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
        if (!finite(v[0])) fail(c, LQCD_ENONFINITE);
        else if (v[0] == 0.0) { c->omega[0] = 0.0; c->omega[1] = 0.0; }
        else { c->omega[0] = v[1] / v[0]; c->omega[1] = v[2] / v[0]; }
        break;
    case FIN_BI_RHO:
        c->rr = v[0];
        c->iter += 1;
        if (!finite(v[0]) || !finite(v[1]) || !finite(v[2])) { fail(c, LQCD_ENONFINITE); break; }
        if (v[0] <= c->thresh) { c->done = 1; break; }
        c->rho_old[0] = c->rho[0];
        c->rho_old[1] = c->rho[1];
        c->rho[0] = v[1];
        c->rho[1] = v[2];
        if ((v[1] == 0.0 && v[2] == 0.0) || (c->omega[0] == 0.0 && c->omega[1] == 0.0)) {
            fail(c, LQCD_EBREAKDOWN);
            break;
        }
        if (c->iter >= c->iter_limit) fail(c, LQCD_ENOCONV);
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

template <int N>
__device__ inline void finalize(int fin, Ctl* c, const double (&v)[N])
{
    double t[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < N && j < 6; ++j) t[j] = v[j];
    finalize_totals(fin, c, t);
}

__device__ inline bool pred_skip(int pred, const Ctl* c)
{
    if (pred == PRED_ALWAYS || c == nullptr) return false;
    const int done = __hip_atomic_load(&c->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (done) return true;
    if (pred == PRED_UPDATE) return c->update == 0;
    if (pred == PRED_NO_UPDATE) return c->update != 0;
    return false;
}

}  // namespace lqcd
