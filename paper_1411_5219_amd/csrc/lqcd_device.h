// Device-side building blocks for the MI355X (gfx950) lattice kernels:
// complex arithmetic, the structure-of-arrays field layouts and their
// loads/stores in FP64, FP32 and FP16 storage, 12-real link reconstruction,
// and the deterministic FP64 block reduction.
//
// Layouts (all per parity; Vh = V/2 sites, S = Vh rounded up to 256):
//   spinor FP64 : 12 planes of double2, plane k = 3*spin + colour
//   spinor FP32 :  6 planes of float4, plane k holds complex 2k and 2k+1
//   spinor FP16 :  3 planes of 8 halves (complex 4k..4k+3, scaled) then one
//                  plane of float scales (max |real component| of the site)
//   links       : [mu][parity of the base site][plane][S]
//       FP64/18 : 9 planes double2 (row-major 3x3)
//       FP64/12 : 6 planes double2 (rows 0 and 1)
//       FP32/18 : 9 planes float2
//       FP32/12 : 3 planes float4 (complex pairs of rows 0 and 1)
//       FP16/12 : one plane of 8 halves (row 0, element (1,0)) and one
//                 plane of 4 halves (elements (1,1), (1,2))
//   colour vector (staggered fermions, 3 complex per site):
//       FP64    : 3 planes of double2
//       FP32    : one plane of float4 (colours 0, 1) and one of float2 (2)
//       FP16    : one plane of 16 bytes: 6 halves (scaled) and the FP32 scale
// A full-lattice field is the even-parity field followed by the odd one.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lqcd {

template <class R>
struct cplx {
    R x, y;
};

template <class R>
__device__ __forceinline__ cplx<R> mk(R x, R y) { return {x, y}; }
template <class R>
__device__ __forceinline__ cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <class R>
__device__ __forceinline__ cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <class R>
__device__ __forceinline__ cplx<R> operator-(cplx<R> a) { return {-a.x, -a.y}; }
template <class R>
__device__ __forceinline__ cplx<R> operator*(cplx<R> a, cplx<R> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class R>
__device__ __forceinline__ cplx<R> operator*(R s, cplx<R> a) { return {s * a.x, s * a.y}; }
// conj(a) * b
template <class R>
__device__ __forceinline__ cplx<R> cmulc(cplx<R> a, cplx<R> b)
{
    return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
template <class R>
__device__ __forceinline__ cplx<R> conj(cplx<R> a) { return {a.x, -a.y}; }

__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// sum_k U[a][k] v[k] (ADJ = false) or sum_k conj(U[k][a]) v[k] (ADJ = true):
// one row of an SU(3) matrix-vector product.  In FP32 each real part is a
// single chain of fused multiply-adds (1 multiply + 5 FMAs): summing three
// complex products as written compiles to 3 multiplies, 3 FMAs and 2 adds
// per real part (the sum of two FMA results is not contracted), and the FP32
// and FP16-storage hops are bound by their VALU issue.  FP64 keeps the
// written form: its hop is bound by memory, and the chains' longer live
// ranges push it past the register budget of two waves per SIMD.
template <class R, bool ADJ>
__device__ __forceinline__ cplx<R> su3_row(const cplx<R> (&U)[3][3], int a, const cplx<R> (&v)[3])
{
    if constexpr (sizeof(R) == 8) {
        if (!ADJ) return U[a][0] * v[0] + U[a][1] * v[1] + U[a][2] * v[2];
        return cmulc(U[0][a], v[0]) + cmulc(U[1][a], v[1]) + cmulc(U[2][a], v[2]);
    }
    R re, im;
    if (!ADJ) {
        re = U[a][0].x * v[0].x;
        im = U[a][0].x * v[0].y;
        re = fmar(-U[a][0].y, v[0].y, re);
        im = fmar(U[a][0].y, v[0].x, im);
#pragma unroll
        for (int k = 1; k < 3; ++k) {
            re = fmar(U[a][k].x, v[k].x, re);
            im = fmar(U[a][k].x, v[k].y, im);
            re = fmar(-U[a][k].y, v[k].y, re);
            im = fmar(U[a][k].y, v[k].x, im);
        }
    } else {
        re = U[0][a].x * v[0].x;
        im = U[0][a].x * v[0].y;
        re = fmar(U[0][a].y, v[0].y, re);
        im = fmar(-U[0][a].y, v[0].x, im);
#pragma unroll
        for (int k = 1; k < 3; ++k) {
            re = fmar(U[k][a].x, v[k].x, re);
            im = fmar(U[k][a].x, v[k].y, im);
            re = fmar(U[k][a].y, v[k].y, re);
            im = fmar(-U[k][a].y, v[k].x, im);
        }
    }
    return {re, im};
}
// i * a and -i * a
template <class R>
__device__ __forceinline__ cplx<R> ti(cplx<R> a) { return {-a.y, a.x}; }
template <class R>
__device__ __forceinline__ cplx<R> mti(cplx<R> a) { return {a.y, -a.x}; }
template <class R>
__device__ __forceinline__ R norm2(cplx<R> a) { return a.x * a.x + a.y * a.y; }

template <class R>
struct Spinor {
    cplx<R> s[4][3];
};

// ---------------------------------------------------------------------------
// Memory access through buffer resources.  A field (one parity of a spinor
// field, or one (mu, parity) block of links) is described by a buffer
// resource built from uniform kernel arguments, so it lives in scalar
// registers; the plane offset (uniform) goes in the scalar offset and one
// 32-bit per-lane byte offset per site is shared by all planes.  The
// resource carries the field size: an access outside the field returns zero
// (loads) or is dropped (stores) instead of touching other memory.

using rsrc_t = __amdgpu_buffer_rsrc_t;

// Buffer resource word 3 for raw (untyped, stride 0) buffers on gfx9-class
// hardware: 32-bit data format, no swizzling.
constexpr int kRsrcWord3 = 0x00020000;

// Cache-policy bits of link loads.  With one right-hand side a link is read
// once per application, so FP64 and FP32 links are loaded non-temporally
// (bit 1) to spare the cached neighbour spinors; FP16 links measured faster
// without the hint.  With several right-hand sides the links are re-read by
// the following blocks and are loaded normally (the kernel chooses).
#ifndef LQCD_LINK_AUX
#define LQCD_LINK_AUX 2
#endif
#ifndef LQCD_LINK16_AUX
#define LQCD_LINK16_AUX 0
#endif
// Cache-policy bits of the Dslash output stores: streaming (bit 1).  An L2
// line lives for about one hop's worth of a block's run time under this
// load, so output lines that stay in L2 push out neighbour spinors that
// other blocks are about to read; streamed stores cut the FP64 hop's reads
// from 1.15x to 1.11x of compulsory, and the following kernels that read
// the output lose nothing measurable.
#ifndef LQCD_OUT_AUX
#define LQCD_OUT_AUX 2
#endif

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, int64_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRsrcWord3);
}

template <class T, int AUX = 0>
__device__ __forceinline__ T bload(rsrc_t r, uint32_t voff, uint32_t soff)
{
    if constexpr (sizeof(T) == 16) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX));
    else if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
    else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
}

using u32x4 = __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t;
using u32x2 = __attribute__((__vector_size__(2 * sizeof(uint32_t)))) uint32_t;

template <int AUX = 0, class T>
__device__ __forceinline__ void bstore(rsrc_t r, uint32_t voff, uint32_t soff, const T& v)
{
    if constexpr (sizeof(T) == 16) __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, voff, soff, AUX);
    else if constexpr (sizeof(T) == 8) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, AUX);
    else __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, AUX);
}

// ---------------------------------------------------------------------------
// Spinor storage

template <int PREC>
struct SpinorIO;

// Every spinor access takes an optional per-lane byte offset xo (added to the
// site offset; the field of another right-hand side) and the bytes span the
// buffer resource covers from base (0: one field).
template <>
struct SpinorIO<64> {
    using R = double;
    static constexpr int kBytesPerSite = 192;
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t site, Spinor<R>& v,
                                                uint32_t xo = 0, int64_t span = 0)
    {
        const rsrc_t r = make_rsrc(base, span > 0 ? span : 192 * S);
        const uint32_t o = static_cast<uint32_t>(site) * 16u + xo;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const double2 d = bload<double2>(r, o, (uint32_t)(k * S * 16));
            v.s[k / 3][k % 3] = {d.x, d.y};
        }
    }
    template <int AUX = 0>
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t site, const Spinor<R>& v,
                                                 uint32_t xo = 0, int64_t span = 0)
    {
        const rsrc_t r = make_rsrc(base, span > 0 ? span : 192 * S);
        const uint32_t o = static_cast<uint32_t>(site) * 16u + xo;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const cplx<R> c = v.s[k / 3][k % 3];
            bstore<AUX>(r, o, (uint32_t)(k * S * 16), make_double2(c.x, c.y));
        }
    }
};

template <>
struct SpinorIO<32> {
    using R = float;
    static constexpr int kBytesPerSite = 96;
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t site, Spinor<R>& v,
                                                uint32_t xo = 0, int64_t span = 0)
    {
        const rsrc_t r = make_rsrc(base, span > 0 ? span : 96 * S);
        const uint32_t o = static_cast<uint32_t>(site) * 16u + xo;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const float4 d = bload<float4>(r, o, (uint32_t)(k * S * 16));
            v.s[(2 * k) / 3][(2 * k) % 3] = {d.x, d.y};
            v.s[(2 * k + 1) / 3][(2 * k + 1) % 3] = {d.z, d.w};
        }
    }
    template <int AUX = 0>
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t site, const Spinor<R>& v,
                                                 uint32_t xo = 0, int64_t span = 0)
    {
        const rsrc_t r = make_rsrc(base, span > 0 ? span : 96 * S);
        const uint32_t o = static_cast<uint32_t>(site) * 16u + xo;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const cplx<R> a = v.s[(2 * k) / 3][(2 * k) % 3];
            const cplx<R> c = v.s[(2 * k + 1) / 3][(2 * k + 1) % 3];
            bstore<AUX>(r, o, (uint32_t)(k * S * 16), make_float4(a.x, a.y, c.x, c.y));
        }
    }
};

// Scale of a site stored at FP16: its largest magnitude, or 0 (the site is
// stored as zero) when that is below the smallest normal FP32.  Such sites
// are rounding debris of cancellations that keep shrinking by kappa^2 per
// operator application (a point source on a large lattice reaches FP32
// denormals within a few applications), and the reciprocal of a denormal
// overflows to infinity.
__device__ __forceinline__ float fp16_site_scale(float m) { return m >= 1.17549435e-38f ? m : 0.f; }

// FP16 storage, FP32 arithmetic: the 24 reals of a site are stored as
// halves relative to one FP32 scale per site (the largest magnitude), so
// the stored values lie in [-1, 1] and the relative precision is per site.
template <>
struct SpinorIO<16> {
    using R = float;
    static constexpr int kBytesPerSite = 52;
    __device__ static __forceinline__ float h2f(uint32_t w, int hi)
    {
        __half_raw r;
        r.x = hi ? (unsigned short)(w >> 16) : (unsigned short)(w & 0xffffu);
        return __half2float(__half(r));
    }
    __device__ static __forceinline__ uint32_t f2h2(float a, float b)
    {
        __half_raw ra = __half(__float2half_rn(a));
        __half_raw rb = __half(__float2half_rn(b));
        return (uint32_t)ra.x | ((uint32_t)rb.x << 16);
    }
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t site, Spinor<R>& v,
                                                uint32_t xo = 0, int64_t span = 0)
    {
        const rsrc_t r = make_rsrc(base, span > 0 ? span : 52 * S);
        const uint32_t o = static_cast<uint32_t>(site) * 16u + xo;
        const float scale = bload<float>(r, static_cast<uint32_t>(site) * 4u + xo, (uint32_t)(3 * S * 16));
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const uint4 d = bload<uint4>(r, o, (uint32_t)(k * S * 16));
            const uint32_t w[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = 4 * k + j;
                v.s[c / 3][c % 3] = {scale * h2f(w[j], 0), scale * h2f(w[j], 1)};
            }
        }
    }
    template <int AUX = 0>
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t site, const Spinor<R>& v,
                                                 uint32_t xo = 0, int64_t span = 0)
    {
        float m = 0.f;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) m = fmaxf(m, fmaxf(fabsf(v.s[a][c].x), fabsf(v.s[a][c].y)));
        m = fp16_site_scale(m);
        const float inv = m > 0.f ? 1.0f / m : 0.f;
        const rsrc_t r = make_rsrc(base, span > 0 ? span : 52 * S);
        const uint32_t o = static_cast<uint32_t>(site) * 16u + xo;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint32_t w[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = 4 * k + j;
                w[j] = f2h2(v.s[c / 3][c % 3].x * inv, v.s[c / 3][c % 3].y * inv);
            }
            bstore<AUX>(r, o, (uint32_t)(k * S * 16), make_uint4(w[0], w[1], w[2], w[3]));
        }
        bstore<AUX>(r, static_cast<uint32_t>(site) * 4u + xo, (uint32_t)(3 * S * 16), m);
    }
};

// Bytes of one parity of a spinor field with stride S.
__host__ __device__ inline int64_t spinor_parity_bytes(int prec, int64_t S)
{
    return prec == 64 ? 192 * S : prec == 32 ? 96 * S : 52 * S;
}

// ---------------------------------------------------------------------------
// Colour-vector storage (staggered fermions)

template <class R>
struct Colour {
    cplx<R> c[3];
};

template <int PREC>
struct ColourIO;

template <>
struct ColourIO<64> {
    using R = double;
    static constexpr int kBytesPerSite = 48;
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t site, Colour<R>& v)
    {
        const rsrc_t r = make_rsrc(base, 48 * S);
        const uint32_t o = static_cast<uint32_t>(site) * 16u;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double2 d = bload<double2>(r, o, (uint32_t)(k * S * 16));
            v.c[k] = {d.x, d.y};
        }
    }
    template <int AUX = 0>
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t site, const Colour<R>& v)
    {
        const rsrc_t r = make_rsrc(base, 48 * S);
        const uint32_t o = static_cast<uint32_t>(site) * 16u;
#pragma unroll
        for (int k = 0; k < 3; ++k) bstore<AUX>(r, o, (uint32_t)(k * S * 16), make_double2(v.c[k].x, v.c[k].y));
    }
};

template <>
struct ColourIO<32> {
    using R = float;
    static constexpr int kBytesPerSite = 24;
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t site, Colour<R>& v)
    {
        const rsrc_t r = make_rsrc(base, 24 * S);
        const float4 a = bload<float4>(r, static_cast<uint32_t>(site) * 16u, 0u);
        const float2 b = bload<float2>(r, static_cast<uint32_t>(site) * 8u, (uint32_t)(16 * S));
        v.c[0] = {a.x, a.y};
        v.c[1] = {a.z, a.w};
        v.c[2] = {b.x, b.y};
    }
    template <int AUX = 0>
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t site, const Colour<R>& v)
    {
        const rsrc_t r = make_rsrc(base, 24 * S);
        bstore<AUX>(r, static_cast<uint32_t>(site) * 16u, 0u, make_float4(v.c[0].x, v.c[0].y, v.c[1].x, v.c[1].y));
        bstore<AUX>(r, static_cast<uint32_t>(site) * 8u, (uint32_t)(16 * S), make_float2(v.c[2].x, v.c[2].y));
    }
};

// FP16 storage, FP32 arithmetic: the 6 reals as halves relative to the
// site's largest magnitude, which is stored as an FP32 in the same 16 bytes.
template <>
struct ColourIO<16> {
    using R = float;
    static constexpr int kBytesPerSite = 16;
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t site, Colour<R>& v)
    {
        const rsrc_t r = make_rsrc(base, 16 * S);
        const uint4 d = bload<uint4>(r, static_cast<uint32_t>(site) * 16u, 0u);
        const float scale = __uint_as_float(d.w);
        const uint32_t w[3] = {d.x, d.y, d.z};
#pragma unroll
        for (int k = 0; k < 3; ++k) v.c[k] = {scale * SpinorIO<16>::h2f(w[k], 0), scale * SpinorIO<16>::h2f(w[k], 1)};
    }
    template <int AUX = 0>
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t site, const Colour<R>& v)
    {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) m = fmaxf(m, fmaxf(fabsf(v.c[k].x), fabsf(v.c[k].y)));
        m = fp16_site_scale(m);
        const float inv = m > 0.f ? 1.0f / m : 0.f;
        uint32_t w[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) w[k] = SpinorIO<16>::f2h2(v.c[k].x * inv, v.c[k].y * inv);
        const rsrc_t r = make_rsrc(base, 16 * S);
        bstore<AUX>(r, static_cast<uint32_t>(site) * 16u, 0u, make_uint4(w[0], w[1], w[2], __float_as_uint(m)));
    }
};

// Bytes of one parity of a colour-vector field with stride S.
__host__ __device__ inline int64_t colour_parity_bytes(int prec, int64_t S)
{
    return prec == 64 ? 48 * S : prec == 32 ? 24 * S : 16 * S;
}

// Site-local kernels (BLAS, conversion, packing) see a field as NC complex
// numbers per site: KIND 0 is a spinor (12), KIND 1 a colour vector (3).
enum FieldKind { KIND_SPINOR = 0, KIND_COLOUR = 1 };

template <int PREC, int KIND>
struct FieldIO;

template <int PREC>
struct FieldIO<PREC, KIND_SPINOR> {
    using IO = SpinorIO<PREC>;
    using R = typename IO::R;
    using Vec = Spinor<R>;
    static constexpr int NC = 12;
    __device__ static __forceinline__ cplx<R>& at(Vec& v, int k) { return v.s[k / 3][k % 3]; }
    __device__ static __forceinline__ void load(const void* b, int64_t S, int64_t h, Vec& v) { IO::load(b, S, h, v); }
    template <int AUX = 0>
    __device__ static __forceinline__ void store(void* b, int64_t S, int64_t h, const Vec& v)
    {
        IO::template store<AUX>(b, S, h, v);
    }
};

template <int PREC>
struct FieldIO<PREC, KIND_COLOUR> {
    using IO = ColourIO<PREC>;
    using R = typename IO::R;
    using Vec = Colour<R>;
    static constexpr int NC = 3;
    __device__ static __forceinline__ cplx<R>& at(Vec& v, int k) { return v.c[k]; }
    __device__ static __forceinline__ void load(const void* b, int64_t S, int64_t h, Vec& v) { IO::load(b, S, h, v); }
    template <int AUX = 0>
    __device__ static __forceinline__ void store(void* b, int64_t S, int64_t h, const Vec& v)
    {
        IO::template store<AUX>(b, S, h, v);
    }
};

__host__ __device__ inline int64_t field_parity_bytes(int kind, int prec, int64_t S)
{
    return kind == KIND_COLOUR ? colour_parity_bytes(prec, S) : spinor_parity_bytes(prec, S);
}

// ---------------------------------------------------------------------------
// Link storage

template <class R>
struct Link {
    cplx<R> u[3][3];
};

// Third row of an SU(3) matrix from the first two: row2 = conj(row0 x row1).
// conj(a b - c d), the entry of the third row of an SU(3) matrix rebuilt
// from the first two.  In FP32 each real part is one chain of fused
// multiply-adds (1 multiply + 3 FMAs; as written it compiles to 2
// multiplies, 2 FMAs and a subtract); FP64 keeps the written form, for the
// register budget of its hop (see su3_row).
template <class R>
__device__ __forceinline__ cplx<R> conj_cross(cplx<R> a, cplx<R> b, cplx<R> c, cplx<R> d)
{
    if constexpr (sizeof(R) == 8) return conj(a * b - c * d);
    R re = a.x * b.x;
    re = fmar(-a.y, b.y, re);
    re = fmar(-c.x, d.x, re);
    re = fmar(c.y, d.y, re);
    R im = -(a.x * b.y);
    im = fmar(-a.y, b.x, im);
    im = fmar(c.x, d.y, im);
    im = fmar(c.y, d.x, im);
    return {re, im};
}

template <class R>
__device__ __forceinline__ void reconstruct_row2(Link<R>& U)
{
    U.u[2][0] = conj_cross(U.u[0][1], U.u[1][2], U.u[0][2], U.u[1][1]);
    U.u[2][1] = conj_cross(U.u[0][2], U.u[1][0], U.u[0][0], U.u[1][2]);
    U.u[2][2] = conj_cross(U.u[0][0], U.u[1][1], U.u[0][1], U.u[1][0]);
}

template <int PREC, int RECON>
struct LinkIO;

// Generic plane-per-element link storage: kPlanes planes of W bytes per
// link block (mu, parity), each holding complex entries of the link.
template <>
struct LinkIO<64, 18> {
    using R = double;
    static constexpr int kPlanes = 9;
    static constexpr int kBytesPerLink = 144;
    template <int AUX = LQCD_LINK_AUX>
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t blk, int64_t site, Link<R>& U)
    {
        const rsrc_t r = make_rsrc(static_cast<const char*>(base) + blk * kPlanes * S * 16, kPlanes * S * 16);
        const uint32_t o = static_cast<uint32_t>(site) * 16u;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const double2 d = bload<double2, AUX>(r, o, (uint32_t)(k * S * 16));
            U.u[k / 3][k % 3] = {d.x, d.y};
        }
    }
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t blk, int64_t site, const Link<R>& U)
    {
        const rsrc_t r = make_rsrc(static_cast<char*>(base) + blk * kPlanes * S * 16, kPlanes * S * 16);
        const uint32_t o = static_cast<uint32_t>(site) * 16u;
#pragma unroll
        for (int k = 0; k < 9; ++k)
            bstore(r, o, (uint32_t)(k * S * 16), make_double2(U.u[k / 3][k % 3].x, U.u[k / 3][k % 3].y));
    }
};

template <>
struct LinkIO<64, 12> {
    using R = double;
    static constexpr int kPlanes = 6;
    static constexpr int kBytesPerLink = 96;
    template <int AUX = LQCD_LINK_AUX>
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t blk, int64_t site, Link<R>& U)
    {
        const rsrc_t r = make_rsrc(static_cast<const char*>(base) + blk * kPlanes * S * 16, kPlanes * S * 16);
        const uint32_t o = static_cast<uint32_t>(site) * 16u;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double2 d = bload<double2, AUX>(r, o, (uint32_t)(k * S * 16));
            U.u[k / 3][k % 3] = {d.x, d.y};
        }
        reconstruct_row2(U);
    }
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t blk, int64_t site, const Link<R>& U)
    {
        const rsrc_t r = make_rsrc(static_cast<char*>(base) + blk * kPlanes * S * 16, kPlanes * S * 16);
        const uint32_t o = static_cast<uint32_t>(site) * 16u;
#pragma unroll
        for (int k = 0; k < 6; ++k)
            bstore(r, o, (uint32_t)(k * S * 16), make_double2(U.u[k / 3][k % 3].x, U.u[k / 3][k % 3].y));
    }
};

template <>
struct LinkIO<32, 18> {
    using R = float;
    static constexpr int kPlanes = 9;
    static constexpr int kBytesPerLink = 72;
    template <int AUX = LQCD_LINK_AUX>
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t blk, int64_t site, Link<R>& U)
    {
        const rsrc_t r = make_rsrc(static_cast<const char*>(base) + blk * kPlanes * S * 8, kPlanes * S * 8);
        const uint32_t o = static_cast<uint32_t>(site) * 8u;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const float2 d = bload<float2, AUX>(r, o, (uint32_t)(k * S * 8));
            U.u[k / 3][k % 3] = {d.x, d.y};
        }
    }
    template <class Rin>
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t blk, int64_t site, const Link<Rin>& U)
    {
        const rsrc_t r = make_rsrc(static_cast<char*>(base) + blk * kPlanes * S * 8, kPlanes * S * 8);
        const uint32_t o = static_cast<uint32_t>(site) * 8u;
#pragma unroll
        for (int k = 0; k < 9; ++k)
            bstore(r, o, (uint32_t)(k * S * 8), make_float2((float)U.u[k / 3][k % 3].x, (float)U.u[k / 3][k % 3].y));
    }
};

template <>
struct LinkIO<32, 12> {
    using R = float;
    static constexpr int kPlanes = 3;
    static constexpr int kBytesPerLink = 48;
    template <int AUX = LQCD_LINK_AUX>
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t blk, int64_t site, Link<R>& U)
    {
        const rsrc_t r = make_rsrc(static_cast<const char*>(base) + blk * kPlanes * S * 16, kPlanes * S * 16);
        const uint32_t o = static_cast<uint32_t>(site) * 16u;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float4 d = bload<float4, AUX>(r, o, (uint32_t)(k * S * 16));
            U.u[(2 * k) / 3][(2 * k) % 3] = {d.x, d.y};
            U.u[(2 * k + 1) / 3][(2 * k + 1) % 3] = {d.z, d.w};
        }
        reconstruct_row2(U);
    }
    template <class Rin>
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t blk, int64_t site, const Link<Rin>& U)
    {
        const rsrc_t r = make_rsrc(static_cast<char*>(base) + blk * kPlanes * S * 16, kPlanes * S * 16);
        const uint32_t o = static_cast<uint32_t>(site) * 16u;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const auto a = U.u[(2 * k) / 3][(2 * k) % 3];
            const auto c = U.u[(2 * k + 1) / 3][(2 * k + 1) % 3];
            bstore(r, o, (uint32_t)(k * S * 16), make_float4((float)a.x, (float)a.y, (float)c.x, (float)c.y));
        }
    }
};

// FP16 links: SU(3) entries lie in [-1, 1], so no scale is needed.  A link
// block is 24*S bytes: a plane of 8 halves (16*S bytes: row 0 and element
// (1,0)) followed by a plane of 4 halves (8*S bytes: elements (1,1), (1,2)).
template <>
struct LinkIO<16, 12> {
    using R = float;
    static constexpr int kBytesPerLink = 24;
    template <int AUX = LQCD_LINK16_AUX>
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t blk, int64_t site, Link<R>& U)
    {
        const rsrc_t r = make_rsrc(static_cast<const char*>(base) + blk * 24 * S, 24 * S);
        const uint4 d = bload<uint4, AUX>(r, static_cast<uint32_t>(site) * 16u, 0u);
        const uint2 e = bload<uint2, AUX>(r, static_cast<uint32_t>(site) * 8u, (uint32_t)(16 * S));
        const uint32_t w[6] = {d.x, d.y, d.z, d.w, e.x, e.y};
#pragma unroll
        for (int k = 0; k < 6; ++k)
            U.u[k / 3][k % 3] = {SpinorIO<16>::h2f(w[k], 0), SpinorIO<16>::h2f(w[k], 1)};
        reconstruct_row2(U);
    }
    template <class Rin>
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t blk, int64_t site, const Link<Rin>& U)
    {
        const rsrc_t r = make_rsrc(static_cast<char*>(base) + blk * 24 * S, 24 * S);
        uint32_t w[6];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            w[k] = SpinorIO<16>::f2h2((float)U.u[k / 3][k % 3].x, (float)U.u[k / 3][k % 3].y);
        bstore(r, static_cast<uint32_t>(site) * 16u, 0u, make_uint4(w[0], w[1], w[2], w[3]));
        bstore(r, static_cast<uint32_t>(site) * 8u, (uint32_t)(16 * S), make_uint2(w[4], w[5]));
    }
};

__host__ __device__ inline int64_t link_bytes(int prec, int recon)
{
    if (prec == 64) return recon == 18 ? 144 : 96;
    if (prec == 32) return recon == 18 ? 72 : 48;
    return 24;
}

// ---------------------------------------------------------------------------
// Deterministic reductions.  Every thread holds N partial sums in FP64 and
// each block writes N partials; the totals are formed in a fixed order (see
// block_reduce_store), so they depend only on the grid shape.

template <int N>
__device__ __forceinline__ void wave_reduce(double (&v)[N])
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] += __shfl_xor(v[j], off, 64);
}

// Block-level part of a reduction: the wavefront folds its N sums with
// butterfly shuffles, the waves are combined in LDS in wave order, and
// thread 0 writes the block's N partial sums to partials[bid * N + j].
// A separate one-block-per-right-hand-side kernel (k_finalize) sums the
// partials in block order after the kernel boundary has made them visible,
// so totals depend only on the grid shape, never on scheduling, and no
// device-wide fence is needed.  Block size: a multiple of 64, <= 1024.
template <int N>
__device__ void block_reduce_store(double (&v)[N], double* partials, int bid)
{
    __shared__ double sm[N][16];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    wave_reduce<N>(v);
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < N; ++j) sm[j][wave] = v[j];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double s = 0.0;
            for (int w = 0; w < nwaves; ++w) s += sm[j][w];
            partials[(int64_t)bid * N + j] = s;
        }
    }
}

// Block index remap that hands each XCD a contiguous range of logical
// blocks.  Workgroups are dispatched round-robin over the 8 XCDs, so
// hardware block b runs on XCD b % 8; giving that XCD logical blocks
// [start(b%8), start(b%8) + count) keeps neighbouring sites in one L2.
__device__ __forceinline__ int xcd_swizzle(int b, int nb)
{
    const int q = nb >> 3, rem = nb & 7;
    const int xcd = b & 7, k = b >> 3;
    const int start = xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q;
    return start + k;
}

}  // namespace lqcd
