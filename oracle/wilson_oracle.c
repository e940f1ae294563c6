/*
 * FP64 CPU oracle for the Wilson / twisted-mass Wilson fermion matrix.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the tests, the smoke check and the CPU baseline of
 * the benchmark use it.  It shares no code with the GPU path.
 *
 * What it computes (readings of the paper, whose section 1 names the Wilson
 * "derivative part" of D and whose section 3 names twisted-mass Wilson
 * fermions, but which prints no formula):
 *
 *   (H psi)(x) = sum_mu [ (1 - s gamma_mu) U_mu(x)      f+_mu(x) psi(x + mu)
 *                       + (1 + s gamma_mu) U_mu(x - mu)^+ f-_mu(x) psi(x - mu) ]
 *
 * with s = +1 for H and s = -1 for its adjoint H^+ (the adjoint swaps the
 * projector signs), f+_mu(x) = exp(i theta_mu) when x_mu = L_mu - 1 (the hop
 * crosses the boundary forwards) and 1 otherwise, f-_mu(x) = exp(-i theta_mu)
 * when x_mu = 0 and 1 otherwise.  The twisted-mass matrix is
 *
 *   M = 1 + 2 i kappa mu gamma_5 - kappa H,     M^+ = 1 - 2 i kappa mu gamma_5 - kappa H^+.
 *
 * Gamma matrices: chiral basis, gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]
 * for k = 1, 2, 3 (directions x, y, z) and gamma_4 = [[0, 1], [1, 0]] (t);
 * gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 is computed, not typed in.
 *
 * Every spin projector is applied as a full 4x4 matrix to the colour-rotated
 * 4-spinor: slow and direct, on purpose.
 *
 * Layout (canonical, complex128): U[mu][site][a][b] (link from site to
 * site + mu), psi[site][spin][colour], site = x + Lx*(y + Ly*(z + Lz*t)).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef double _Complex cplx;

static void pauli(int k, cplx s[2][2])
{
    memset(s, 0, sizeof(cplx) * 4);
    if (k == 1) { s[0][1] = 1; s[1][0] = 1; }
    if (k == 2) { s[0][1] = -I; s[1][0] = I; }
    if (k == 3) { s[0][0] = 1; s[1][1] = -1; }
}

/* g[mu][row][col] for mu = 0..3 (x, y, z, t) and g5. */
static void build_gammas(cplx g[4][4][4], cplx g5[4][4])
{
    memset(g, 0, sizeof(cplx) * 64);
    for (int k = 1; k <= 3; ++k) {
        cplx s[2][2];
        pauli(k, s);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                g[k - 1][a][2 + b] = -I * s[a][b];
                g[k - 1][2 + a][b] = I * s[a][b];
            }
    }
    for (int a = 0; a < 2; ++a) {
        g[3][a][2 + a] = 1;
        g[3][2 + a][a] = 1;
    }
    cplx t1[4][4], t2[4][4];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            cplx v = 0;
            for (int c = 0; c < 4; ++c) v += g[0][a][c] * g[1][c][b];
            t1[a][b] = v;
        }
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            cplx v = 0;
            for (int c = 0; c < 4; ++c) v += t1[a][c] * g[2][c][b];
            t2[a][b] = v;
        }
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            cplx v = 0;
            for (int c = 0; c < 4; ++c) v += t2[a][c] * g[3][c][b];
            g5[a][b] = v;
        }
}

/* Export the matrices so the tests can check the Clifford algebra. */
void oracle_gammas(double *out /* 5*4*4 complex as re,im pairs */)
{
    cplx g[4][4][4], g5[4][4];
    build_gammas(g, g5);
    cplx *o = (cplx *)out;
    for (int m = 0; m < 4; ++m)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) o[(m * 4 + a) * 4 + b] = g[m][a][b];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) o[(4 * 4 + a) * 4 + b] = g5[a][b];
}

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

/* out = H in (dagger = 0) or H^+ in (dagger = 1), full lattice. */
void oracle_hop(const int *L, const double *theta, const double *Ud, const double *ind,
                double *outd, int dagger)
{
    const cplx *U = (const cplx *)Ud;
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
    cplx g[4][4][4], g5[4][4];
    build_gammas(g, g5);
    const double s = dagger ? -1.0 : 1.0;
    cplx ph[4];
    for (int mu = 0; mu < 4; ++mu) ph[mu] = cexp(I * theta[mu]);

#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < V; ++i) {
        int c[4];
        site_coords(i, L, c);
        cplx acc[4][3];
        memset(acc, 0, sizeof(acc));
        for (int mu = 0; mu < 4; ++mu) {
            for (int dir = 0; dir < 2; ++dir) {
                int cn[4] = {c[0], c[1], c[2], c[3]};
                cplx phase = 1;
                const cplx *link;
                if (dir == 0) { /* forward: U_mu(x) psi(x + mu) */
                    cn[mu] = (c[mu] + 1) % L[mu];
                    if (c[mu] == L[mu] - 1) phase = ph[mu];
                    link = U + ((int64_t)mu * V + i) * 9;
                } else {        /* backward: U_mu(x - mu)^+ psi(x - mu) */
                    cn[mu] = (c[mu] - 1 + L[mu]) % L[mu];
                    if (c[mu] == 0) phase = conj(ph[mu]);
                    link = U + ((int64_t)mu * V + site_index(cn, L)) * 9;
                }
                const cplx *pn = in + site_index(cn, L) * 12;
                cplx v[4][3];
                for (int sp = 0; sp < 4; ++sp)
                    for (int a = 0; a < 3; ++a) {
                        cplx t = 0;
                        for (int b = 0; b < 3; ++b) {
                            cplx u = dir == 0 ? link[3 * a + b] : conj(link[3 * b + a]);
                            t += u * pn[3 * sp + b];
                        }
                        v[sp][a] = phase * t;
                    }
                /* spin projector: (1 - s gamma) forwards, (1 + s gamma) backwards */
                const double sg = dir == 0 ? -s : s;
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) {
                        cplx coef = (a == b ? 1.0 : 0.0) + sg * g[mu][a][b];
                        if (coef == 0) continue;
                        for (int col = 0; col < 3; ++col) acc[a][col] += coef * v[b][col];
                    }
            }
        }
        cplx *o = out + i * 12;
        for (int a = 0; a < 4; ++a)
            for (int col = 0; col < 3; ++col) o[3 * a + col] = acc[a][col];
    }
}

/* out = M in or M^+ in with M = 1 + 2 i kappa mu gamma_5 - kappa H. */
void oracle_apply_M(const int *L, const double *theta, double kappa, double mu,
                    const double *Ud, const double *ind, double *outd, int dagger)
{
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
    cplx g[4][4][4], g5[4][4];
    build_gammas(g, g5);
    oracle_hop(L, theta, Ud, ind, outd, dagger);
    const cplx tw = (dagger ? -1.0 : 1.0) * 2.0 * I * kappa * mu;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < V; ++i) {
        const cplx *p = in + i * 12;
        cplx *o = out + i * 12;
        cplx r[12];
        for (int a = 0; a < 4; ++a)
            for (int col = 0; col < 3; ++col) {
                cplx g5p = 0;
                for (int b = 0; b < 4; ++b) g5p += g5[a][b] * p[3 * b + col];
                r[3 * a + col] = p[3 * a + col] + tw * g5p - kappa * o[3 * a + col];
            }
        memcpy(o, r, sizeof(r));
    }
}

int oracle_num_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}
