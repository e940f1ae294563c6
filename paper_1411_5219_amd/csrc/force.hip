// N_f = 2 twisted-mass pseudo-fermion force on gfx950.
//
// For S_f = ||M^-1 phi||^2, X = M^-1 phi and Z = (M^+)^-1 X, the derivative
// along U_mu(y) -> exp(i w T^a) U_mu(y) gathered over the generators is
//
//   F_mu(y) = (i kappa / 2) [ (W - W^+) - tr(W - W^+) / 3 ],
//   W = f+ U A - f- B U^+,
//   A = sum_t h-(X(y + mu))_t h-(Z(y))_t^+,   B = sum_t h+(X(y))_t h+(Z(y + mu))_t^+,
//
// where h-+ are the half spinors of the projectors (1 -+ gamma_mu) (the
// same 2x3 projections the Dslash uses: sum over the four spins of
// (1 -+ gamma) psi (x) chi^+ reduces to the two half-spinor outer products)
// and f+- the boundary phases of the forward hop from y and the backward hop
// from y + mu.  Z is not stored: the caller passes Wf with Z = gamma_5 Wf
// (Wf = M(-mu)^-1 gamma_5 X, since M(mu)^+ = gamma_5 M(-mu) gamma_5).
//
// One work-item per site of the full lattice (both parities in one launch),
// the four directions in turn; F is written in the canonical layout
// F[mu][site][3][3] (complex128) for the host side of the molecular dynamics.
#include "dslash_impl.h"

namespace lqcd {

struct ForceArgs {
    Geom g;
    const void* U;      // FP64 links, internal layout
    const char* X;      // full-lattice FP64 spinor fields, internal layout
    const char* Wf;
    double2* F;         // canonical (4, V, 3, 3)
    int64_t pb;         // bytes of one parity field
    double kappa;
    double scale;
    int accumulate;
};

template <int RECON, int MU>
__device__ __forceinline__ void force_one(const ForceArgs& a, const SiteGeo& geo, int p, int64_t site, int64_t V,
                                          const Spinor<double>& Xy, const Spinor<double>& Zy)
{
    using R = double;
    const int64_t S = a.g.S;
    const Nbr n = geo.template get<2 * MU>();  // forward hop from y: neighbour y + mu, link U_mu(y)
    const int64_t qoff = (int64_t)(1 - p) * a.pb;
    Spinor<R> Xf, Wn;
    SpinorIO<64>::load(a.X + qoff, S, n.nb, Xf);
    SpinorIO<64>::load(a.Wf + qoff, S, n.nb, Wn);
    Spinor<R> Zf;  // Z(y + mu) = gamma_5 Wf(y + mu)
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) Zf.s[s][c] = s < 2 ? Wn.s[s][c] : -Wn.s[s][c];
    Link<R> U;
    LinkIO<64, RECON>::template load<0>(a.U, S, n.lblk, n.lsite, U);

    cplx<R> hx[2][3], hz[2][3], gx[2][3], gz[2][3];
    project<R, MU, 1>(Xf, hx);   // (1 - gamma) X(y + mu)
    project<R, MU, 1>(Zy, hz);   // (1 - gamma) Z(y)
    project<R, MU, -1>(Xy, gx);  // (1 + gamma) X(y)
    project<R, MU, -1>(Zf, gz);  // (1 + gamma) Z(y + mu)

    // A = sum_t hx_t hz_t^+, B = sum_t gx_t gz_t^+
    cplx<R> A[3][3], B[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            A[i][j] = hx[0][i] * conj(hz[0][j]) + hx[1][i] * conj(hz[1][j]);
            B[i][j] = gx[0][i] * conj(gz[0][j]) + gx[1][i] * conj(gz[1][j]);
        }
    const bool cross = n.cross;
    const cplx<R> fp = cross ? cplx<R>{a.g.ph[MU][0], a.g.ph[MU][1]} : cplx<R>{1.0, 0.0};
    const cplx<R> fm = conj(fp);
    // W = f+ U A - f- B U^+
    cplx<R> Wm[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const cplx<R> ua = U.u[i][0] * A[0][j] + U.u[i][1] * A[1][j] + U.u[i][2] * A[2][j];
            const cplx<R> bu = B[i][0] * conj(U.u[j][0]) + B[i][1] * conj(U.u[j][1]) + B[i][2] * conj(U.u[j][2]);
            Wm[i][j] = fp * ua - fm * bu;
        }
    // F = (i kappa / 2) [(W - W^+) - tr(W - W^+) / 3]
    cplx<R> D[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) D[i][j] = Wm[i][j] - conj(Wm[j][i]);
    const cplx<R> tr3 = {(D[0][0].x + D[1][1].x + D[2][2].x) / 3.0, (D[0][0].y + D[1][1].y + D[2][2].y) / 3.0};
    const double k = 0.5 * a.kappa * a.scale;
    double2* out = a.F + ((int64_t)MU * V + site) * 9;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const cplx<R> d = i == j ? D[i][j] - tr3 : D[i][j];
            // i k d
            double2 v = make_double2(-k * d.y, k * d.x);
            if (a.accumulate) {
                const double2 o = out[i * 3 + j];
                v.x += o.x;
                v.y += o.y;
            }
            out[i * 3 + j] = v;
        }
}

template <int RECON>
__global__ void __launch_bounds__(256) k_tm_force(const ForceArgs a)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int Vh = a.g.Vh;
    if (gid >= 2 * (int64_t)Vh) return;
    const int p = (int)(gid / Vh);
    const int h = (int)(gid - (int64_t)p * Vh);
    const int Lxh = a.g.Lxh, Ly = a.g.L[1], Lz = a.g.L[2];
    SitePos sp;
    sp.h = h;
    sp.xh = h % Lxh;
    int r = h / Lxh;
    sp.y = r % Ly;
    r /= Ly;
    sp.z = r % Lz;
    sp.t = r / Lz;
    sp.x = 2 * sp.xh + ((sp.y + sp.z + sp.t + p) & 1);
    sp.valid = true;
    const SiteGeo geo = site_geo(a.g, sp, p);
    const int64_t V = 2 * (int64_t)Vh;
    const int64_t site = sp.x + (int64_t)a.g.L[0] * (sp.y + (int64_t)Ly * (sp.z + (int64_t)Lz * sp.t));
    const int64_t poff = (int64_t)p * a.pb;
    Spinor<double> Xy, Wy, Zy;
    SpinorIO<64>::load(a.X + poff, a.g.S, h, Xy);
    SpinorIO<64>::load(a.Wf + poff, a.g.S, h, Wy);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) Zy.s[s][c] = s < 2 ? Wy.s[s][c] : -Wy.s[s][c];
    force_one<RECON, 0>(a, geo, p, site, V, Xy, Zy);
    force_one<RECON, 1>(a, geo, p, site, V, Xy, Zy);
    force_one<RECON, 2>(a, geo, p, site, V, Xy, Zy);
    force_one<RECON, 3>(a, geo, p, site, V, Xy, Zy);
}

hipError_t launch_tm_force(int recon, const Geom& g, const void* U, const void* X, const void* Wf, void* F,
                           double kappa, double scale, int accumulate, hipStream_t s)
{
    ForceArgs a{};
    a.g = g;
    a.U = U;
    a.X = static_cast<const char*>(X);
    a.Wf = static_cast<const char*>(Wf);
    a.F = static_cast<double2*>(F);
    a.pb = spinor_parity_bytes(64, g.S);
    a.kappa = kappa;
    a.scale = scale;
    a.accumulate = accumulate;
    dim3 b(256), gr((unsigned)((2 * (int64_t)g.Vh + 255) / 256));
    if (recon == 18) hipLaunchKernelGGL(k_tm_force<18>, gr, b, 0, s, a);
    else if (recon == 12) hipLaunchKernelGGL(k_tm_force<12>, gr, b, 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace lqcd
