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
// (Wf = M(-mu)^-1 gamma_5 X, since M(mu)^+ = gamma_5 M(-mu) gamma_5), and
// with gamma_5 = diag(1, 1, -1, -1) the projection (1 -+ gamma) of Z is the
// projection (1 +- gamma) of Wf.
//
// Work split: a block of four waves covers 64 consecutive sites of the
// canonical order (both parities interleaved), wave w computing the link in
// direction w.  The direction is wave-uniform, so each wave runs one
// straight-line instance with no divergence, holds only one direction's
// state (the half spinors, A, B, the link and W), and the four waves of a
// block read X(y) and Wf(y) of the same sites, the later ones from the
// compute unit's cache.  F is written in the
// canonical layout F[mu][site][3][3] (complex128): the 64 lanes of a wave
// own 64 consecutive 144-byte matrices, one contiguous 9 KiB run, which the
// wave transposes through LDS so that each of its nine store instructions
// writes 1 KiB of consecutive bytes (stored straight from registers, each
// instruction would scatter 16-byte pieces 144 bytes apart).
#include "dslash_impl.h"

// Waves per SIMD the register allocation must allow: one direction's state
// needs about 170 VGPRs; at three waves the compiler spills a few of them,
// and two waves without spills measured slightly faster.
#ifndef LQCD_FORCE_WAVES
#define LQCD_FORCE_WAVES 2
#endif
#ifndef LQCD_FORCE_SWIZZLE
#define LQCD_FORCE_SWIZZLE 1
#endif
// Largest z slab of the block order (the launch takes the largest divisor
// of Lz not above it).
#ifndef LQCD_FORCE_ZTILE
#define LQCD_FORCE_ZTILE 2
#endif
// Cache policy of the link loads (each link is read once).
#ifndef LQCD_FORCE_LINK_AUX
#define LQCD_FORCE_LINK_AUX 2
#endif
// Cache policy of the F stores: streaming (the field is consumed by a later pass).
#ifndef LQCD_FORCE_OUT_AUX
#define LQCD_FORCE_OUT_AUX 2
#endif

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
    int ztile;          // z planes per slab of the block order (divides Lz)
};

// The lanes of a wave hold sites of both parities, so every field is read
// through one wave-uniform buffer resource spanning both parity halves, the
// parity going into the per-lane offset: a per-lane base address would turn
// each buffer load into a loop over the distinct bases.
__device__ __forceinline__ void load_spinor(rsrc_t r, int64_t S, uint32_t voff, Spinor<double>& v)
{
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const double2 d = bload<double2>(r, voff, (uint32_t)(k * S * 16));
        v.s[k / 3][k % 3] = {d.x, d.y};
    }
}

template <int RECON>
__device__ __forceinline__ void load_link(rsrc_t r, int64_t S, uint32_t voff, Link<double>& U)
{
    constexpr int NP = LinkIO<64, RECON>::kPlanes;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const double2 d = bload<double2, LQCD_FORCE_LINK_AUX>(r, voff, (uint32_t)(k * S * 16));
        U.u[k / 3][k % 3] = {d.x, d.y};
    }
    if constexpr (RECON == 12) reconstruct_row2(U);
}

// C = sum_t a_t b_t^+ over the two half-spinor components.
__device__ __forceinline__ void outer2(const cplx<double> (&a)[2][3], const cplx<double> (&b)[2][3],
                                       cplx<double> (&C)[3][3])
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) C[i][j] = a[0][i] * conj(b[0][j]) + a[1][i] * conj(b[1][j]);
}

template <int RECON, int MU>
__device__ __forceinline__ void force_link(const ForceArgs& a, const SiteGeo& geo, int p, double2 (&out)[9])
{
    using R = double;
    const int64_t S = a.g.S;
    const Nbr n = geo.template get<2 * MU>();  // forward hop from y: neighbour y + mu, link U_mu(y)
    const rsrc_t rX = make_rsrc(a.X, 2 * a.pb);
    const rsrc_t rW = make_rsrc(a.Wf, 2 * a.pb);
    const uint32_t oy = static_cast<uint32_t>(p * a.pb + (int64_t)geo.h * 16);        // y, parity p
    const uint32_t on = static_cast<uint32_t>((1 - p) * a.pb + (int64_t)n.nb * 16);   // y + mu, parity 1 - p

    // A = sum_t (1 - gamma) X(y + mu) (x) [(1 - gamma) Z(y)]^+
    cplx<R> A[3][3];
    {
        Spinor<R> s;
        cplx<R> hx[2][3], hz[2][3];
        load_spinor(rX, S, on, s);
        project<R, MU, 1>(s, hx);
        load_spinor(rW, S, oy, s);
        project<R, MU, -1>(s, hz);  // (1 - gamma) gamma_5 Wf = gamma_5 (1 + gamma) Wf: same half spinor
        outer2(hx, hz, A);
    }
    // U_mu(y): the two parity blocks of direction mu are adjacent
    constexpr int NP = LinkIO<64, RECON>::kPlanes;
    const int64_t lb = (int64_t)NP * S * 16;
    Link<R> U;
    load_link<RECON>(make_rsrc(static_cast<const char*>(a.U) + 2 * MU * lb, 2 * lb), S,
                     static_cast<uint32_t>(p * lb + (int64_t)n.lsite * 16), U);
    const cplx<R> fp = n.cross ? cplx<R>{a.g.ph[MU][0], a.g.ph[MU][1]} : cplx<R>{1.0, 0.0};
    const cplx<R> fm = conj(fp);
    // W = f+ U A (A is overwritten row by row through UA)
    cplx<R> Wm[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Wm[i][j] = fp * (U.u[i][0] * A[0][j] + U.u[i][1] * A[1][j] + U.u[i][2] * A[2][j]);
    // B = sum_t (1 + gamma) X(y) (x) [(1 + gamma) Z(y + mu)]^+; W -= f- B U^+
    {
        cplx<R> B[3][3];
        Spinor<R> s;
        cplx<R> gx[2][3], gz[2][3];
        load_spinor(rX, S, oy, s);
        project<R, MU, -1>(s, gx);
        load_spinor(rW, S, on, s);
        project<R, MU, 1>(s, gz);
        outer2(gx, gz, B);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                Wm[i][j] = Wm[i][j] -
                           fm * (B[i][0] * conj(U.u[j][0]) + B[i][1] * conj(U.u[j][1]) + B[i][2] * conj(U.u[j][2]));
    }
    // F = (i kappa / 2) [(W - W^+) - tr(W - W^+) / 3]; the diagonal of W - W^+ is 2 i Im W_ii
    const double tr3 = 2.0 * (Wm[0][0].y + Wm[1][1].y + Wm[2][2].y) / 3.0;
    const double k = 0.5 * a.kappa * a.scale;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cplx<R> d;
            if (i == j) d = {0.0, 2.0 * Wm[i][i].y - tr3};
            else d = Wm[i][j] - conj(Wm[j][i]);
            out[i * 3 + j] = make_double2(-k * d.y, k * d.x);  // i k d
        }
}

template <int RECON>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LQCD_FORCE_WAVES)))
k_tm_force(const ForceArgs a)
{
    __shared__ double2 stage[4][64 * 9];
    const int nb = (int)gridDim.x;
    const int bid = LQCD_FORCE_SWIZZLE ? xcd_swizzle((int)blockIdx.x, nb) : (int)blockIdx.x;
    const int lane = (int)threadIdx.x & 63;
    const int mu = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int Lx = a.g.L[0], Ly = a.g.L[1], Lz = a.g.L[2], Lt = a.g.L[3];
    const int64_t V = 2 * (int64_t)a.g.Vh;
    // Block order: t fastest, then z within a slab of a.ztile planes, then
    // the 64-site segment of the xy plane, then the slab.  The blocks that
    // read a site's spinors as neighbours in t, z and y then run within a
    // few dozen blocks of the one that reads them as its own sites, while
    // the lines are still in L2.
    const int plane = Lx * Ly;
    const int nseg = (plane + 63) >> 6;
    int rb = bid;
    const int t = rb % Lt;
    rb /= Lt;
    const int zl = rb % a.ztile;
    rb /= a.ztile;
    const int seg = rb % nseg;
    const int z = (rb / nseg) * a.ztile + zl;
    const int nvalid = min(64, plane - seg * 64);
    const int64_t base = (int64_t)seg * 64 + (int64_t)plane * (z + (int64_t)Lz * t);
    const int64_t site = base + lane;
    double2 out[9];
    if (lane < nvalid) {
        SitePos sp;
        const int q = seg * 64 + lane;
        sp.x = q % Lx;
        sp.y = q / Lx;
        sp.z = z;
        sp.t = t;
        sp.xh = sp.x >> 1;
        sp.h = (int)(site >> 1);  // Lx is even: the parity-local index is the canonical index halved
        sp.valid = true;
        const int p = (sp.x + sp.y + sp.z + sp.t) & 1;
        const SiteGeo geo = site_geo(a.g, sp, p);
        if (mu == 0) force_link<RECON, 0>(a, geo, p, out);
        else if (mu == 1) force_link<RECON, 1>(a, geo, p, out);
        else if (mu == 2) force_link<RECON, 2>(a, geo, p, out);
        else force_link<RECON, 3>(a, geo, p, out);
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) out[k] = make_double2(0.0, 0.0);
    }
    // Transpose through the wave's own LDS slice: lane l holds the matrix of
    // site base + l; after the exchange, store k of lane l writes entry
    // 64 k + l of the wave's 576 consecutive complex numbers.
    double2* st = stage[mu];
#pragma unroll
    for (int k = 0; k < 9; ++k) st[lane * 9 + k] = out[k];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const rsrc_t r = make_rsrc(a.F + (int64_t)mu * V * 9, V * 144);
    const uint32_t o0 = static_cast<uint32_t>(base) * 144u;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        if (k * 64 + lane >= nvalid * 9) break;  // a ragged last segment of the plane
        double2 v = st[k * 64 + lane];
        const uint32_t o = o0 + (uint32_t)(k * 64 + lane) * 16u;
        if (a.accumulate) {
            const double2 old = bload<double2>(r, o, 0u);
            v.x += old.x;
            v.y += old.y;
        }
        bstore<LQCD_FORCE_OUT_AUX>(r, o, 0u, v);
    }
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
    const int64_t V = 2 * (int64_t)g.Vh;
    // one buffer resource per field: both spinor parities, one direction of F
    if (2 * a.pb > INT32_MAX || V * 144 > INT32_MAX) return hipErrorInvalidValue;
    a.ztile = 1;
    for (int d = LQCD_FORCE_ZTILE; d > 1; --d)
        if (g.L[2] % d == 0) {
            a.ztile = d;
            break;
        }
    const int64_t nseg = ((int64_t)g.L[0] * g.L[1] + 63) / 64;
    dim3 b(256), gr((unsigned)(nseg * g.L[2] * g.L[3]));
    if (recon == 18) hipLaunchKernelGGL(k_tm_force<18>, gr, b, 0, s, a);
    else if (recon == 12) hipLaunchKernelGGL(k_tm_force<12>, gr, b, 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace lqcd
