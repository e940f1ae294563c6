// Even-odd Wilson / twisted-mass Dslash for gfx950.
//
// One work-item per output site of parity p.  For each of the 8 hops it
// loads the neighbour spinor of parity 1-p, projects it to a 2x3 half
// spinor with (1 -+ gamma_mu), multiplies by the link (or its adjoint),
// applies the boundary phase on hops that cross the boundary, and rebuilds
// the lower spin components from the upper ones.  The site-diagonal
// twisted-mass terms are fused into the store (out = add + a*site + c*hop)
// together with FP64 reductions, so a Schur-complement application or a
// residual never needs a separate vector pass.
//
// In the chiral basis gamma_mu = [[0, B_mu], [B_mu^+, 0]] with
//   B_x = -i sigma_1, B_y = -i sigma_2, B_z = -i sigma_3, B_t = 1,
// so (1 - s gamma_mu) psi = (h ; -s B_mu^+ h) with h = psi_up - s B_mu psi_lo;
// only h is multiplied by the link.
#include "lqcd.h"
#include "lqcd_device.h"
#include "lqcd_fin.h"
#include "lqcd_kernels.h"

namespace lqcd {

// h = u - SIG * B_MU l   (u = spins 0,1; l = spins 2,3)
template <class R, int MU, int SIG>
__device__ __forceinline__ void project(const Spinor<R>& p, cplx<R> (&h)[2][3])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cplx<R> u0 = p.s[0][c], u1 = p.s[1][c], l0 = p.s[2][c], l1 = p.s[3][c];
        cplx<R> b0, b1;
        if (MU == 0) { b0 = mti(l1); b1 = mti(l0); }        // -i sigma_1
        else if (MU == 1) { b0 = -l1; b1 = l0; }            // -i sigma_2
        else if (MU == 2) { b0 = mti(l0); b1 = ti(l1); }    // -i sigma_3
        else { b0 = l0; b1 = l1; }                          // 1
        if (SIG > 0) { h[0][c] = u0 - b0; h[1][c] = u1 - b1; }
        else { h[0][c] = u0 + b0; h[1][c] = u1 + b1; }
    }
}

// acc += (w ; -SIG * B_MU^+ w)
template <class R, int MU, int SIG>
__device__ __forceinline__ void accumulate(Spinor<R>& acc, const cplx<R> (&w)[2][3])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cplx<R> w0 = w[0][c], w1 = w[1][c];
        acc.s[0][c] = acc.s[0][c] + w0;
        acc.s[1][c] = acc.s[1][c] + w1;
        cplx<R> d0, d1;  // B^+ w
        if (MU == 0) { d0 = ti(w1); d1 = ti(w0); }          // i sigma_1
        else if (MU == 1) { d0 = w1; d1 = -w0; }            // i sigma_2
        else if (MU == 2) { d0 = ti(w0); d1 = mti(w1); }    // i sigma_3
        else { d0 = w0; d1 = w1; }
        if (SIG > 0) { acc.s[2][c] = acc.s[2][c] - d0; acc.s[3][c] = acc.s[3][c] - d1; }
        else { acc.s[2][c] = acc.s[2][c] + d0; acc.s[3][c] = acc.s[3][c] + d1; }
    }
}

// w = U h (ADJ = false) or U^+ h (ADJ = true), on both spin components.
template <class R, bool ADJ>
__device__ __forceinline__ void link_mul(const Link<R>& U, const cplx<R> (&h)[2][3], cplx<R> (&w)[2][3])
{
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cplx<R> t;
            if (!ADJ) t = U.u[a][0] * h[s][0] + U.u[a][1] * h[s][1] + U.u[a][2] * h[s][2];
            else t = cmulc(U.u[0][a], h[s][0]) + cmulc(U.u[1][a], h[s][1]) + cmulc(U.u[2][a], h[s][2]);
            w[s][a] = t;
        }
}

template <class R>
__device__ __forceinline__ void phase_mul(cplx<R> (&w)[2][3], cplx<R> ph)
{
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) w[s][a] = ph * w[s][a];
}

// One hop: neighbour spinor at eo index nb, link block lblk at eo site lsite.
template <int PREC, int RECON, int MU, bool FWD, int SIG>
__device__ __forceinline__ void hop(const void* in, const void* U, int64_t S, int64_t nb, int64_t lblk,
                                    int64_t lsite, bool cross, cplx<typename SpinorIO<PREC>::R> ph,
                                    Spinor<typename SpinorIO<PREC>::R>& acc)
{
    using R = typename SpinorIO<PREC>::R;
    Spinor<R> p;
    SpinorIO<PREC>::load(in, S, nb, p);
    cplx<R> h[2][3];
    project<R, MU, SIG>(p, h);
    Link<R> L;
    LinkIO<PREC, RECON>::load(U, S, lblk, lsite, L);
    cplx<R> w[2][3];
    link_mul<R, !FWD>(L, h, w);
    if (cross) phase_mul(w, FWD ? ph : conj(ph));
    accumulate<R, MU, SIG>(acc, w);
}

template <int RED>
struct RedN {
    static constexpr int N = RED == RED_NONE ? 1 : RED == RED_NORM ? 1 : RED == RED_DOT_AUX ? 2 : 3;
};

template <int PREC, int RECON, bool DAG, int RED>
__global__ void __launch_bounds__(256) k_dslash_eo(const DslashArgs a)
{
    using R = typename SpinorIO<PREC>::R;
    constexpr int N = RedN<RED>::N;
    const int rhs = blockIdx.y;
    Ctl* ctl = a.ctl ? a.ctl + rhs : nullptr;
    if (pred_skip(a.pred, ctl)) return;

    const int nb = gridDim.x;
    int bid = a.swizzle ? xcd_swizzle(blockIdx.x, nb) : (int)blockIdx.x;
    int p = a.parity;
    int64_t poff = 0, ioff = 0;  // parity offsets of output-side / neighbour fields
    if (a.full) {  // both parities in one launch: the first nb/2 blocks even, the rest odd
        const int nbh = nb >> 1;
        p = bid >= nbh;
        bid -= p * nbh;
        poff = p * a.par_bytes;
        ioff = (1 - p) * a.par_bytes;
    }
    const int Lx = a.g.L[0], Ly = a.g.L[1], Lz = a.g.L[2], Lt = a.g.L[3];
    const int Lxh = a.g.Lxh;
    int h, xh, y, z, t;
    bool valid;
    if (a.rows == 0) {
        h = bid * blockDim.x + threadIdx.x;
        valid = h < a.g.Vh;
        xh = h % Lxh;
        int r = h / Lxh;
        y = r % Ly;
        r /= Ly;
        z = r % Lz;
        t = r / Lz;
    } else {
        t = bid % Lt;
        const int r = bid / Lt;
        z = r % Lz;
        const int yc = r / Lz;
        const int yr = threadIdx.x / Lxh;
        xh = threadIdx.x - yr * Lxh;
        y = yc * a.rows + yr;
        valid = yr < a.rows && y < Ly;
        h = xh + Lxh * (y + Ly * (z + Lz * t));
    }
    const int64_t S = a.g.S;
    const int64_t r64 = rhs;

    double tot[3] = {0.0, 0.0, 0.0};

    if (valid) {
        const int x = 2 * xh + ((y + z + t + p) & 1);
        const int64_t hy = Lxh, hz = (int64_t)Lxh * Ly, ht = hz * Lz;
        const int64_t base = h - xh;

        const char* in = static_cast<const char*>(a.in) + r64 * a.st_in + ioff;
        constexpr int SF = DAG ? -1 : 1;  // projector sign of forward hops: (1 - SF gamma)
        Spinor<R> acc;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc.s[s][c] = {R(0), R(0)};

        const cplx<R> ph0 = {R(a.g.ph[0][0]), R(a.g.ph[0][1])};
        const cplx<R> ph1 = {R(a.g.ph[1][0]), R(a.g.ph[1][1])};
        const cplx<R> ph2 = {R(a.g.ph[2][0]), R(a.g.ph[2][1])};
        const cplx<R> ph3 = {R(a.g.ph[3][0]), R(a.g.ph[3][1])};
        const int q = 1 - p;
        // x
        {
            const int xp = x == Lx - 1 ? 0 : x + 1;
            const int xm = x == 0 ? Lx - 1 : x - 1;
            const int64_t nf = base + (xp >> 1), nbk = base + (xm >> 1);
            hop<PREC, RECON, 0, true, SF>(in, a.U, S, nf, 0 * 2 + p, h, x == Lx - 1, ph0, acc);
            hop<PREC, RECON, 0, false, -SF>(in, a.U, S, nbk, 0 * 2 + q, nbk, x == 0, ph0, acc);
        }
        // y
        {
            const int64_t nf = y == Ly - 1 ? h - (Ly - 1) * hy : h + hy;
            const int64_t nbk = y == 0 ? h + (Ly - 1) * hy : h - hy;
            hop<PREC, RECON, 1, true, SF>(in, a.U, S, nf, 1 * 2 + p, h, y == Ly - 1, ph1, acc);
            hop<PREC, RECON, 1, false, -SF>(in, a.U, S, nbk, 1 * 2 + q, nbk, y == 0, ph1, acc);
        }
        // z
        {
            const int64_t nf = z == Lz - 1 ? h - (Lz - 1) * hz : h + hz;
            const int64_t nbk = z == 0 ? h + (Lz - 1) * hz : h - hz;
            hop<PREC, RECON, 2, true, SF>(in, a.U, S, nf, 2 * 2 + p, h, z == Lz - 1, ph2, acc);
            hop<PREC, RECON, 2, false, -SF>(in, a.U, S, nbk, 2 * 2 + q, nbk, z == 0, ph2, acc);
        }
        // t
        {
            const int64_t nf = t == Lt - 1 ? h - (Lt - 1) * ht : h + ht;
            const int64_t nbk = t == 0 ? h + (Lt - 1) * ht : h - ht;
            hop<PREC, RECON, 3, true, SF>(in, a.U, S, nf, 3 * 2 + p, h, t == Lt - 1, ph3, acc);
            hop<PREC, RECON, 3, false, -SF>(in, a.U, S, nbk, 3 * 2 + q, nbk, t == 0, ph3, acc);
        }

        // epilogue: out = add + a * site + c * acc
        const cplx<R> cu = {R(a.c.up[0]), R(a.c.up[1])}, cl = {R(a.c.lo[0]), R(a.c.lo[1])};
        Spinor<R> o;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) o.s[s][c] = (s < 2 ? cu : cl) * acc.s[s][c];
        Spinor<R> st;
        if (a.site) {
            const cplx<R> au = {R(a.a.up[0]), R(a.a.up[1])}, al = {R(a.a.lo[0]), R(a.a.lo[1])};
            SpinorIO<PREC>::load(static_cast<const char*>(a.site) + r64 * a.st_site + poff, S, h, st);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int c = 0; c < 3; ++c) o.s[s][c] = o.s[s][c] + (s < 2 ? au : al) * st.s[s][c];
        }
        if (a.add) {
            Spinor<R> ad;
            SpinorIO<PREC>::load(static_cast<const char*>(a.add) + r64 * a.st_add + poff, S, h, ad);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int c = 0; c < 3; ++c) o.s[s][c] = o.s[s][c] + ad.s[s][c];
        }
        if (a.out) SpinorIO<PREC>::template store<LQCD_OUT_AUX>(static_cast<char*>(a.out) + r64 * a.st_out + poff, S, h, o);

        if (RED != RED_NONE) {
            // reduce what was stored (re-read rounding of low-precision storage is not modelled)
            if (RED == RED_NORM || RED == RED_NORM_DS || RED == RED_NORM_DA) {
                double n2 = 0.0;
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int c = 0; c < 3; ++c) n2 += (double)norm2(o.s[s][c]);
                tot[0] = n2;
            }
            if (RED == RED_NORM_DS) {  // <out, site>
                double re = 0.0, im = 0.0;
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const cplx<R> v = cmulc(o.s[s][c], st.s[s][c]);
                        re += (double)v.x;
                        im += (double)v.y;
                    }
                tot[1] = re;
                tot[2] = im;
            }
            if (RED == RED_DOT_AUX || RED == RED_NORM_DA) {  // <aux, out>
                Spinor<R> ax;
                SpinorIO<PREC>::load(static_cast<const char*>(a.aux) + r64 * a.st_aux + poff, S, h, ax);
                double re = 0.0, im = 0.0;
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const cplx<R> v = cmulc(ax.s[s][c], o.s[s][c]);
                        re += (double)v.x;
                        im += (double)v.y;
                    }
                tot[RED == RED_DOT_AUX ? 0 : 1] = re;
                tot[RED == RED_DOT_AUX ? 1 : 2] = im;
            }
        }
    }

    if (RED != RED_NONE) {
        double red[N];
#pragma unroll
        for (int j = 0; j < N; ++j) red[j] = tot[j];
        block_reduce_store<N>(red, a.r.partials + (int64_t)rhs * nb * N, blockIdx.x);
    }
}

template <int PREC, int RECON, bool DAG>
static hipError_t launch_red(int red, const DslashArgs& a, dim3 grid, dim3 block, hipStream_t s)
{
    switch (red) {
    case RED_NONE: hipLaunchKernelGGL((k_dslash_eo<PREC, RECON, DAG, RED_NONE>), grid, block, 0, s, a); break;
    case RED_NORM: hipLaunchKernelGGL((k_dslash_eo<PREC, RECON, DAG, RED_NORM>), grid, block, 0, s, a); break;
    case RED_NORM_DS: hipLaunchKernelGGL((k_dslash_eo<PREC, RECON, DAG, RED_NORM_DS>), grid, block, 0, s, a); break;
    case RED_DOT_AUX: hipLaunchKernelGGL((k_dslash_eo<PREC, RECON, DAG, RED_DOT_AUX>), grid, block, 0, s, a); break;
    case RED_NORM_DA: hipLaunchKernelGGL((k_dslash_eo<PREC, RECON, DAG, RED_NORM_DA>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int PREC, int RECON>
static hipError_t launch_dag(bool dag, int red, const DslashArgs& a, dim3 grid, dim3 block, hipStream_t s)
{
    return dag ? launch_red<PREC, RECON, true>(red, a, grid, block, s)
               : launch_red<PREC, RECON, false>(red, a, grid, block, s);
}

hipError_t launch_dslash(int prec, int recon, bool dagger, int red, const DslashArgs& args, int nrhs,
                         const Launch& cfg, hipStream_t s)
{
    DslashArgs a = args;
    a.swizzle = cfg.swizzle;
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
    dim3 block(blk);
    dim3 grid(nbh * (a.full ? 2u : 1u), nrhs);
    if (red != RED_NONE && (int)grid.x > a.r.capacity) return hipErrorInvalidValue;  // partials too small
    hipError_t e;
    if (prec == 64 && recon == 18) e = launch_dag<64, 18>(dagger, red, a, grid, block, s);
    else if (prec == 64 && recon == 12) e = launch_dag<64, 12>(dagger, red, a, grid, block, s);
    else if (prec == 32 && recon == 18) e = launch_dag<32, 18>(dagger, red, a, grid, block, s);
    else if (prec == 32 && recon == 12) e = launch_dag<32, 12>(dagger, red, a, grid, block, s);
    else if (prec == 16 && recon == 12) e = launch_dag<16, 12>(dagger, red, a, grid, block, s);
    else return hipErrorInvalidValue;
    if (e != hipSuccess || red == RED_NONE) return e;
    return launch_finalize((red == RED_NORM ? 1 : red == RED_DOT_AUX ? 2 : 3), a.r.partials,
                           (int)grid.x, a.r.fin, a.ctl, a.pred, nrhs, s);
}

}  // namespace lqcd
