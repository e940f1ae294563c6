/*
 * FP64 CPU oracle for the staggered (Kogut-Susskind) fermion matrix.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the tests, the smoke check and the CPU baseline of
 * the benchmark use it.  It shares no code with the GPU path.
 *
 * What it computes.  The paper (section 3) adds the standard staggered
 * formulation and (section 1) counts its derivative part D_KS at 570 flops
 * and 1584 bytes per site (eight neighbour colour vectors, eight links, one
 * output), but prints no formula.  The reading used here is the textbook
 * one-component operator:
 *
 *   (D phi)(x) = 1/2 sum_mu eta_mu(x) [ f+_mu(x) U_mu(x) phi(x + mu)
 *                                      - f-_mu(x) U_mu(x - mu)^+ phi(x - mu) ]
 *
 *   eta_0(x) = 1, eta_1(x) = (-1)^x0, eta_2(x) = (-1)^(x0 + x1),
 *   eta_3(x) = (-1)^(x0 + x1 + x2)
 *
 * with the boundary factors of the Wilson oracle: f+_mu(x) = exp(i theta_mu)
 * when x_mu = L_mu - 1, f-_mu(x) = exp(-i theta_mu) when x_mu = 0, else 1.
 * D is anti-Hermitian, so with the bare mass m
 *
 *   M = m + D,     M^+ = m - D.
 *
 * Written as plain site loops: the phases are recomputed from the
 * coordinates at every hop and every 3x3 product is spelled out.
 *
 * Layout (canonical, complex128): U[mu][site][a][b] (link from site to
 * site + mu), phi[site][colour], site = x + Lx*(y + Ly*(z + Lz*t)).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef double _Complex cplx;

static inline int64_t site_index(const int c[4], const int L[4])
{
    return (int64_t)c[0] + (int64_t)L[0] * ((int64_t)c[1] + (int64_t)L[1] * ((int64_t)c[2] + (int64_t)L[2] * c[3]));
}

static inline void site_coords(int64_t i, const int L[4], int c[4])
{
    c[0] = (int)(i % L[0]); i /= L[0];
    c[1] = (int)(i % L[1]); i /= L[1];
    c[2] = (int)(i % L[2]); i /= L[2];
    c[3] = (int)i;
}

/* eta_mu(x) = (-1)^(x_0 + ... + x_{mu-1}) */
static inline double eta(int mu, const int c[4])
{
    int s = 0;
    for (int nu = 0; nu < mu; ++nu) s += c[nu];
    return (s & 1) ? -1.0 : 1.0;
}

/* out = D in, full lattice. */
void stag_oracle_hop(const int *L, const double *theta, const double *Ud, const double *ind, double *outd)
{
    const cplx *U = (const cplx *)Ud;
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
    cplx ph[4];
    for (int mu = 0; mu < 4; ++mu) ph[mu] = cexp(I * theta[mu]);

#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < V; ++i) {
        int c[4];
        site_coords(i, L, c);
        cplx acc[3] = {0, 0, 0};
        for (int mu = 0; mu < 4; ++mu) {
            const double e = eta(mu, c);
            /* forward: + U_mu(x) phi(x + mu) */
            {
                int cn[4] = {c[0], c[1], c[2], c[3]};
                cn[mu] = (c[mu] + 1) % L[mu];
                const cplx f = c[mu] == L[mu] - 1 ? ph[mu] : 1.0;
                const cplx *u = U + ((int64_t)mu * V + i) * 9;
                const cplx *pn = in + site_index(cn, L) * 3;
                for (int a = 0; a < 3; ++a) {
                    cplx t = 0;
                    for (int b = 0; b < 3; ++b) t += u[3 * a + b] * pn[b];
                    acc[a] += 0.5 * e * f * t;
                }
            }
            /* backward: - U_mu(x - mu)^+ phi(x - mu) */
            {
                int cn[4] = {c[0], c[1], c[2], c[3]};
                cn[mu] = (c[mu] - 1 + L[mu]) % L[mu];
                const cplx f = c[mu] == 0 ? conj(ph[mu]) : 1.0;
                const int64_t j = site_index(cn, L);
                const cplx *u = U + ((int64_t)mu * V + j) * 9;
                const cplx *pn = in + j * 3;
                for (int a = 0; a < 3; ++a) {
                    cplx t = 0;
                    for (int b = 0; b < 3; ++b) t += conj(u[3 * b + a]) * pn[b];
                    acc[a] -= 0.5 * e * f * t;
                }
            }
        }
        for (int a = 0; a < 3; ++a) out[i * 3 + a] = acc[a];
    }
}

/* out = M in (dagger = 0) or M^+ in (dagger = 1), M = m + D. */
void stag_oracle_apply_M(const int *L, const double *theta, double mass, const double *Ud, const double *ind,
                         double *outd, int dagger)
{
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
    stag_oracle_hop(L, theta, Ud, ind, outd);
    const double sd = dagger ? -1.0 : 1.0;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < 3 * V; ++k) out[k] = mass * in[k] + sd * out[k];
}
