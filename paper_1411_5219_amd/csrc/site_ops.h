// Site-local block routines shared by the standalone kernels (blas.hip) and
// the persistent batched solver (persist.hip): the fused BLAS-1 steps of the
// solvers with their FP64 block reductions, precision conversion, and the
// block-order sum of reduction partials.
#pragma once

#include "lqcd.h"
#include "lqcd_device.h"
#include "lqcd_fin.h"
#include "lqcd_kernels.h"

namespace lqcd {

template <int OP>
struct BlasRed {
    static constexpr int N = (OP == BLAS_CG_XR || OP == BLAS_NORM || OP == BLAS_AXMY_NORM) ? 1
                             : (OP == BLAS_BI_XR || OP == BLAS_NORM_DOT || OP == BLAS_BL_ORTH ||
                                OP == BLAS_BL_MR)                                          ? 3
                             : OP == BLAS_BL_GRAM                                          ? 5
                                                                                          : 0;
};

template <class R>
__device__ __forceinline__ cplx<R> cval(const double* d) { return {R(d[0]), R(d[1])}; }

// The work of block bx of nbx (x) and by (right-hand side) of a launch, on
// fields of kind KIND (spinors or colour vectors) stored at precision PREC.
template <int PREC, int KIND, int OP>
__device__ __forceinline__ void blas_block(const BlasArgs& a, int bx, int nbx, int by)
{
    using F = FieldIO<PREC, KIND>;
    using R = typename F::R;
    using Vec = typename F::Vec;
    constexpr int NC = F::NC;
    constexpr int N = BlasRed<OP>::N;
    constexpr int NN = N > 0 ? N : 1;
    const int rhs = by;
    Ctl* ctl = a.ctl ? a.ctl + rhs : nullptr;
    if (pred_skip(a.pred, ctl)) return;

    // each sub-field covers nbs whole blocks, so the sub-field is uniform per block
    const int nbs = nbx / a.nsub;
    const int sub = bx / nbs;
    const int64_t h = (int64_t)(bx - sub * nbs) * blockDim.x + threadIdx.x;
    const int64_t soff = (int64_t)sub * a.sub_stride;
    const int64_t r64 = rhs;
    const int64_t S = a.S;
    auto P = [&](void* base, int64_t st) { return static_cast<char*>(base) + r64 * st + soff; };

    double red[NN];
#pragma unroll
    for (int j = 0; j < NN; ++j) red[j] = 0.0;

    if (h < a.Vh) {
        if (OP == BLAS_CG_XR) {
            const R al = R(ctl->alpha);
            Vec x, p, r, w;
            F::load(P(a.x, a.st_x), S, h, x);
            F::load(P(a.y, a.st_y), S, h, p);
            F::load(P(a.z, a.st_z), S, h, r);
            F::load(P(a.w, a.st_w), S, h, w);
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                F::at(x, k) = F::at(x, k) + al * F::at(p, k);
                F::at(r, k) = F::at(r, k) - al * F::at(w, k);
                red[0] += (double)norm2(F::at(r, k));
            }
            F::store(P(a.x, a.st_x), S, h, x);
            F::store(P(a.z, a.st_z), S, h, r);
        } else if (OP == BLAS_CG_P) {
            const R be = R(ctl->beta);
            Vec p, z;
            F::load(P(a.y, a.st_y), S, h, p);
            F::load(P(a.z, a.st_z), S, h, z);
#pragma unroll
            for (int k = 0; k < NC; ++k) F::at(p, k) = F::at(z, k) + be * F::at(p, k);
            F::store(P(a.y, a.st_y), S, h, p);
        } else if (OP == BLAS_COPY) {
            Vec x;
            F::load(P(a.x, a.st_x), S, h, x);
            F::store(P(a.y, a.st_y), S, h, x);
        } else if (OP == BLAS_ZERO) {
            Vec x;
#pragma unroll
            for (int k = 0; k < NC; ++k) F::at(x, k) = {R(0), R(0)};
            F::store(P(a.y, a.st_y), S, h, x);
        } else if (OP == BLAS_SPIN_SCALE) {
            // spinors: coef.up on spins 0, 1 and coef.lo on spins 2, 3; colour vectors: coef.up
            const cplx<R> cu = cval<R>(a.coef.up), cl = cval<R>(a.coef.lo);
            Vec x;
            F::load(P(a.x, a.st_x), S, h, x);
#pragma unroll
            for (int k = 0; k < NC; ++k) F::at(x, k) = (KIND == KIND_COLOUR || k < 6 ? cu : cl) * F::at(x, k);
            F::store(P(a.y, a.st_y), S, h, x);
        } else if (OP == BLAS_NORM) {
            Vec x;
            F::load(P(a.x, a.st_x), S, h, x);
#pragma unroll
            for (int k = 0; k < NC; ++k) red[0] += (double)norm2(F::at(x, k));
        } else if (OP == BLAS_NORM_DOT) {
            Vec x, r0;
            F::load(P(a.x, a.st_x), S, h, x);
            F::load(static_cast<const char*>(a.r0) + r64 * a.st_r0 + soff, S, h, r0);
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                red[0] += (double)norm2(F::at(x, k));
                const cplx<R> d = cmulc(F::at(r0, k), F::at(x, k));
                red[1] += (double)d.x;
                red[2] += (double)d.y;
            }
        } else if (OP == BLAS_XPY) {
            Vec x, y;
            F::load(P(a.x, a.st_x), S, h, x);
            F::load(P(a.y, a.st_y), S, h, y);
#pragma unroll
            for (int k = 0; k < NC; ++k) F::at(y, k) = F::at(y, k) + F::at(x, k);
            F::store(P(a.y, a.st_y), S, h, y);
        } else if (OP == BLAS_BI_P) {
            // beta = (rho / rho_old) (alpha / omega), computed in FP64
            double t1[2], t2[2], be[2];
            cdiv(ctl->rho, ctl->rho_old, t1);
            cdiv(ctl->balpha, ctl->omega, t2);
            be[0] = t1[0] * t2[0] - t1[1] * t2[1];
            be[1] = t1[0] * t2[1] + t1[1] * t2[0];
            const cplx<R> b = cval<R>(be), om = cval<R>(ctl->omega);
            Vec p, r, v;
            F::load(P(a.y, a.st_y), S, h, p);
            F::load(P(a.z, a.st_z), S, h, r);
            F::load(P(a.v, a.st_v), S, h, v);
#pragma unroll
            for (int k = 0; k < NC; ++k) F::at(p, k) = F::at(r, k) + b * (F::at(p, k) - om * F::at(v, k));
            F::store(P(a.y, a.st_y), S, h, p);
        } else if (OP == BLAS_BI_S) {
            const cplx<R> al = cval<R>(ctl->balpha);
            Vec r, v;
            F::load(P(a.z, a.st_z), S, h, r);
            F::load(P(a.v, a.st_v), S, h, v);
#pragma unroll
            for (int k = 0; k < NC; ++k) F::at(r, k) = F::at(r, k) - al * F::at(v, k);
            F::store(P(a.w, a.st_w), S, h, r);
        } else if (OP == BLAS_BI_XR) {
            // omega of this step (0 when ||t|| = 0: x += alpha p, r = s)
            const cplx<R> al = cval<R>(ctl->balpha), om = cval<R>(ctl->omega_step);
            Vec x, p, sv, t, r0, r;
            F::load(P(a.x, a.st_x), S, h, x);
            F::load(P(a.y, a.st_y), S, h, p);
            F::load(P(a.w, a.st_w), S, h, sv);
            F::load(P(a.v, a.st_v), S, h, t);
            F::load(static_cast<const char*>(a.r0) + r64 * a.st_r0 + soff, S, h, r0);
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                F::at(x, k) = F::at(x, k) + al * F::at(p, k) + om * F::at(sv, k);
                F::at(r, k) = F::at(sv, k) - om * F::at(t, k);
                red[0] += (double)norm2(F::at(r, k));
                const cplx<R> d = cmulc(F::at(r0, k), F::at(r, k));
                red[1] += (double)d.x;
                red[2] += (double)d.y;
            }
            F::store(P(a.x, a.st_x), S, h, x);
            F::store(P(a.z, a.st_z), S, h, r);
        } else if (OP == BLAS_MS_AXPY) {
            // x_i += alpha_i p_i (alpha of this right-hand side's control block)
            const R al = R(ctl->alpha);
            Vec x, p;
            F::load(P(a.x, a.st_x), S, h, x);
            F::load(P(a.y, a.st_y), S, h, p);
#pragma unroll
            for (int k = 0; k < NC; ++k) F::at(x, k) = F::at(x, k) + al * F::at(p, k);
            F::store(P(a.x, a.st_x), S, h, x);
        } else if (OP == BLAS_MS_P) {
            // p_i = zeta_i z + beta_i p_i
            const R ze = R(ctl->zeta), be = R(ctl->beta);
            Vec p, z;
            F::load(P(a.y, a.st_y), S, h, p);
            F::load(P(a.z, a.st_z), S, h, z);
#pragma unroll
            for (int k = 0; k < NC; ++k) F::at(p, k) = ze * F::at(z, k) + be * F::at(p, k);
            F::store(P(a.y, a.st_y), S, h, p);
        } else if (OP == BLAS_BL_U0) {
            const cplx<R> be = cval<R>(ctl->bl_beta), g1 = cval<R>(ctl->bl_g1), g2 = cval<R>(ctl->bl_g2);
            Vec u0, r0v, u1, u2;
            F::load(P(a.y, a.st_y), S, h, u0);
            F::load(P(a.z, a.st_z), S, h, r0v);
            F::load(P(a.w, a.st_w), S, h, u1);
            F::load(P(a.v, a.st_v), S, h, u2);
#pragma unroll
            for (int k = 0; k < NC; ++k)
                F::at(u0, k) = F::at(r0v, k) - be * (F::at(u0, k) - g1 * F::at(u1, k) - g2 * F::at(u2, k));
            F::store(P(a.y, a.st_y), S, h, u0);
        } else if (OP == BLAS_BL_XR0) {
            const cplx<R> al = cval<R>(ctl->balpha);
            Vec x, u0, r0v, u1;
            F::load(P(a.x, a.st_x), S, h, x);
            F::load(P(a.y, a.st_y), S, h, u0);
            F::load(P(a.z, a.st_z), S, h, r0v);
            F::load(P(a.w, a.st_w), S, h, u1);
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                F::at(x, k) = F::at(x, k) + al * F::at(u0, k);
                F::at(r0v, k) = F::at(r0v, k) - al * F::at(u1, k);
            }
            F::store(P(a.x, a.st_x), S, h, x);
            F::store(P(a.z, a.st_z), S, h, r0v);
        } else if (OP == BLAS_BL_U01) {
            const cplx<R> be = cval<R>(ctl->bl_beta);
            Vec u0, r0v, u1, r1;
            F::load(P(a.y, a.st_y), S, h, u0);
            F::load(P(a.z, a.st_z), S, h, r0v);
            F::load(P(a.w, a.st_w), S, h, u1);
            F::load(P(a.v, a.st_v), S, h, r1);
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                F::at(u0, k) = F::at(r0v, k) - be * F::at(u0, k);
                F::at(u1, k) = F::at(r1, k) - be * F::at(u1, k);
            }
            F::store(P(a.y, a.st_y), S, h, u0);
            F::store(P(a.w, a.st_w), S, h, u1);
        } else if (OP == BLAS_BL_XR01) {
            const cplx<R> al = cval<R>(ctl->balpha);
            Vec x, u0, r0v, u1, r1, u2;
            F::load(P(a.x, a.st_x), S, h, x);
            F::load(P(a.y, a.st_y), S, h, u0);
            F::load(P(a.z, a.st_z), S, h, r0v);
            F::load(P(a.w, a.st_w), S, h, u1);
            F::load(P(a.v, a.st_v), S, h, r1);
            F::load(static_cast<const char*>(a.r0) + r64 * a.st_r0 + soff, S, h, u2);
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                F::at(x, k) = F::at(x, k) + al * F::at(u0, k);
                F::at(r0v, k) = F::at(r0v, k) - al * F::at(u1, k);
                F::at(r1, k) = F::at(r1, k) - al * F::at(u2, k);
            }
            F::store(P(a.x, a.st_x), S, h, x);
            F::store(P(a.z, a.st_z), S, h, r0v);
            F::store(P(a.v, a.st_v), S, h, r1);
        } else if (OP == BLAS_BL_GRAM) {
            Vec r0v, r1, r2;
            F::load(P(a.z, a.st_z), S, h, r0v);
            F::load(P(a.w, a.st_w), S, h, r1);
            F::load(P(a.v, a.st_v), S, h, r2);
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                red[0] += (double)norm2(F::at(r1, k));
                const cplx<R> d12 = cmulc(F::at(r1, k), F::at(r2, k));
                const cplx<R> d10 = cmulc(F::at(r1, k), F::at(r0v, k));
                red[1] += (double)d12.x;
                red[2] += (double)d12.y;
                red[3] += (double)d10.x;
                red[4] += (double)d10.y;
            }
        } else if (OP == BLAS_BL_ORTH) {
            const cplx<R> ta = cval<R>(ctl->bl_tau);
            Vec r0v, r1, r2;
            F::load(P(a.z, a.st_z), S, h, r0v);
            F::load(P(a.w, a.st_w), S, h, r1);
            F::load(P(a.v, a.st_v), S, h, r2);
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                F::at(r2, k) = F::at(r2, k) - ta * F::at(r1, k);
                red[0] += (double)norm2(F::at(r2, k));
                const cplx<R> d = cmulc(F::at(r2, k), F::at(r0v, k));
                red[1] += (double)d.x;
                red[2] += (double)d.y;
            }
            F::store(P(a.v, a.st_v), S, h, r2);
        } else if (OP == BLAS_BL_MR) {
            const cplx<R> g1 = cval<R>(ctl->bl_g1), g2 = cval<R>(ctl->bl_g2);
            const cplx<R> gp1 = cval<R>(ctl->bl_gp1), gp2 = cval<R>(ctl->bl_gp2);
            Vec x, r0v, r1, r2, rt;
            F::load(P(a.x, a.st_x), S, h, x);
            F::load(P(a.z, a.st_z), S, h, r0v);
            F::load(P(a.w, a.st_w), S, h, r1);
            F::load(P(a.v, a.st_v), S, h, r2);
            F::load(static_cast<const char*>(a.r0) + r64 * a.st_r0 + soff, S, h, rt);
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                F::at(x, k) = F::at(x, k) + g1 * F::at(r0v, k) + g2 * F::at(r1, k);
                F::at(r0v, k) = F::at(r0v, k) - gp1 * F::at(r1, k) - gp2 * F::at(r2, k);
                red[0] += (double)norm2(F::at(r0v, k));
                const cplx<R> d = cmulc(F::at(rt, k), F::at(r0v, k));
                red[1] += (double)d.x;
                red[2] += (double)d.y;
            }
            F::store(P(a.x, a.st_x), S, h, x);
            F::store(P(a.z, a.st_z), S, h, r0v);
        } else if (OP == BLAS_AXMY_NORM) {
            // z -= alpha w ; red ||z||^2
            const R al = R(ctl->alpha);
            Vec z, w;
            F::load(P(a.z, a.st_z), S, h, z);
            F::load(P(a.w, a.st_w), S, h, w);
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                F::at(z, k) = F::at(z, k) - al * F::at(w, k);
                red[0] += (double)norm2(F::at(z, k));
            }
            F::store(P(a.z, a.st_z), S, h, z);
        }
    }

    if (N > 0) block_reduce_store<NN>(red, a.r.partials + (int64_t)rhs * nbx * NN, bx);
}

template <int PD, int PS, bool ACC>
__device__ __forceinline__ void convert_block(const ConvertArgs& a, int bx, int nbx, int by)
{
    const int rhs = by;
    Ctl* ctl = a.ctl ? a.ctl + rhs : nullptr;
    if (pred_skip(a.pred, ctl)) return;
    const int nbs = nbx / a.nsub;
    const int sub = bx / nbs;
    const int64_t h = (int64_t)(bx - sub * nbs) * blockDim.x + threadIdx.x;
    if (h >= a.Vh) return;
    char* dst = static_cast<char*>(a.dst) + rhs * a.rhs_stride_dst + sub * a.sub_stride_dst;
    char* src = static_cast<char*>(a.src) + rhs * a.rhs_stride_src + sub * a.sub_stride_src;
    using RD = typename SpinorIO<PD>::R;
    using RS = typename SpinorIO<PS>::R;
    Spinor<RS> v;
    SpinorIO<PS>::load(src, a.S, h, v);
    Spinor<RD> d;
    if (ACC) SpinorIO<PD>::load(dst, a.S, h, d);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const cplx<RD> cv = {RD(v.s[s][c].x), RD(v.s[s][c].y)};
            d.s[s][c] = ACC ? d.s[s][c] + cv : cv;
        }
    SpinorIO<PD>::store(dst, a.S, h, d);
    if (a.zero_src) {
        Spinor<RS> z;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c) z.s[s][c] = {RS(0), RS(0)};
        SpinorIO<PS>::store(src, a.S, h, z);
    }
}

// Sum of one right-hand side's partials by one block of kFinThreads: each
// thread adds its strided share four blocks' partials at a time (the four
// loads issued together: the partials were just written on other XCDs and
// each round trip is long), then the block folds the threads' sums in a
// fixed order.
constexpr int kFinThreads = 1024;

template <int N>
__device__ __forceinline__ void sum_partials(const double* p, int nblocks, double (&v)[N])
{
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = 0.0;
    for (int b0 = threadIdx.x; b0 < nblocks; b0 += 4 * kFinThreads) {
        double t[4][N];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int b = b0 + u * kFinThreads;
#pragma unroll
            for (int j = 0; j < N; ++j) t[u][j] = b < nblocks ? p[(int64_t)b * N + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int j = 0; j < N; ++j) v[j] += t[u][j];
    }
}

}  // namespace lqcd
