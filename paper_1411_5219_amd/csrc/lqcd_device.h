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
// Spinor storage

template <int PREC>
struct SpinorIO;

template <>
struct SpinorIO<64> {
    using R = double;
    static constexpr int kBytesPerSite = 192;
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t site, Spinor<R>& v)
    {
        const double2* p = static_cast<const double2*>(base) + site;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            double2 d = p[k * S];
            v.s[k / 3][k % 3] = {d.x, d.y};
        }
    }
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t site, const Spinor<R>& v)
    {
        double2* p = static_cast<double2*>(base) + site;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const cplx<R> c = v.s[k / 3][k % 3];
            p[k * S] = make_double2(c.x, c.y);
        }
    }
};

template <>
struct SpinorIO<32> {
    using R = float;
    static constexpr int kBytesPerSite = 96;
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t site, Spinor<R>& v)
    {
        const float4* p = static_cast<const float4*>(base) + site;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            float4 d = p[k * S];
            v.s[(2 * k) / 3][(2 * k) % 3] = {d.x, d.y};
            v.s[(2 * k + 1) / 3][(2 * k + 1) % 3] = {d.z, d.w};
        }
    }
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t site, const Spinor<R>& v)
    {
        float4* p = static_cast<float4*>(base) + site;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const cplx<R> a = v.s[(2 * k) / 3][(2 * k) % 3];
            const cplx<R> b = v.s[(2 * k + 1) / 3][(2 * k + 1) % 3];
            p[k * S] = make_float4(a.x, a.y, b.x, b.y);
        }
    }
};

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
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t site, Spinor<R>& v)
    {
        const uint4* p = static_cast<const uint4*>(base) + site;
        const float scale = reinterpret_cast<const float*>(static_cast<const uint4*>(base) + 3 * S)[site];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint4 d = p[k * S];
            uint32_t w[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = 4 * k + j;
                v.s[c / 3][c % 3] = {scale * h2f(w[j], 0), scale * h2f(w[j], 1)};
            }
        }
    }
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t site, const Spinor<R>& v)
    {
        float m = 0.f;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) m = fmaxf(m, fmaxf(fabsf(v.s[a][c].x), fabsf(v.s[a][c].y)));
        const float inv = m > 0.f ? 1.0f / m : 0.f;
        uint4* p = static_cast<uint4*>(base) + site;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint32_t w[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = 4 * k + j;
                w[j] = f2h2(v.s[c / 3][c % 3].x * inv, v.s[c / 3][c % 3].y * inv);
            }
            p[k * S] = make_uint4(w[0], w[1], w[2], w[3]);
        }
        reinterpret_cast<float*>(static_cast<uint4*>(base) + 3 * S)[site] = m;
    }
};

// Bytes of one parity of a spinor field with stride S.
__host__ __device__ inline int64_t spinor_parity_bytes(int prec, int64_t S)
{
    return prec == 64 ? 192 * S : prec == 32 ? 96 * S : 52 * S;
}

// ---------------------------------------------------------------------------
// Link storage

template <class R>
struct Link {
    cplx<R> u[3][3];
};

// Third row of an SU(3) matrix from the first two: row2 = conj(row0 x row1).
template <class R>
__device__ __forceinline__ void reconstruct_row2(Link<R>& U)
{
    U.u[2][0] = conj(U.u[0][1] * U.u[1][2] - U.u[0][2] * U.u[1][1]);
    U.u[2][1] = conj(U.u[0][2] * U.u[1][0] - U.u[0][0] * U.u[1][2]);
    U.u[2][2] = conj(U.u[0][0] * U.u[1][1] - U.u[0][1] * U.u[1][0]);
}

template <int PREC, int RECON>
struct LinkIO;

template <>
struct LinkIO<64, 18> {
    using R = double;
    static constexpr int kPlanes = 9;
    static constexpr int kPlaneBytes = 16;
    static constexpr int kBytesPerLink = 144;
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t blk, int64_t site, Link<R>& U)
    {
        const double2* p = static_cast<const double2*>(base) + blk * kPlanes * S + site;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            double2 d = p[k * S];
            U.u[k / 3][k % 3] = {d.x, d.y};
        }
    }
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t blk, int64_t site, const Link<R>& U)
    {
        double2* p = static_cast<double2*>(base) + blk * kPlanes * S + site;
#pragma unroll
        for (int k = 0; k < 9; ++k) p[k * S] = make_double2(U.u[k / 3][k % 3].x, U.u[k / 3][k % 3].y);
    }
};

template <>
struct LinkIO<64, 12> {
    using R = double;
    static constexpr int kPlanes = 6;
    static constexpr int kPlaneBytes = 16;
    static constexpr int kBytesPerLink = 96;
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t blk, int64_t site, Link<R>& U)
    {
        const double2* p = static_cast<const double2*>(base) + blk * kPlanes * S + site;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            double2 d = p[k * S];
            U.u[k / 3][k % 3] = {d.x, d.y};
        }
        reconstruct_row2(U);
    }
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t blk, int64_t site, const Link<R>& U)
    {
        double2* p = static_cast<double2*>(base) + blk * kPlanes * S + site;
#pragma unroll
        for (int k = 0; k < 6; ++k) p[k * S] = make_double2(U.u[k / 3][k % 3].x, U.u[k / 3][k % 3].y);
    }
};

template <>
struct LinkIO<32, 18> {
    using R = float;
    static constexpr int kPlanes = 9;
    static constexpr int kPlaneBytes = 8;
    static constexpr int kBytesPerLink = 72;
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t blk, int64_t site, Link<R>& U)
    {
        const float2* p = static_cast<const float2*>(base) + blk * kPlanes * S + site;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            float2 d = p[k * S];
            U.u[k / 3][k % 3] = {d.x, d.y};
        }
    }
    template <class Rin>
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t blk, int64_t site, const Link<Rin>& U)
    {
        float2* p = static_cast<float2*>(base) + blk * kPlanes * S + site;
#pragma unroll
        for (int k = 0; k < 9; ++k) p[k * S] = make_float2((float)U.u[k / 3][k % 3].x, (float)U.u[k / 3][k % 3].y);
    }
};

template <>
struct LinkIO<32, 12> {
    using R = float;
    static constexpr int kPlanes = 3;
    static constexpr int kPlaneBytes = 16;
    static constexpr int kBytesPerLink = 48;
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t blk, int64_t site, Link<R>& U)
    {
        const float4* p = static_cast<const float4*>(base) + blk * kPlanes * S + site;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float4 d = p[k * S];
            U.u[(2 * k) / 3][(2 * k) % 3] = {d.x, d.y};
            U.u[(2 * k + 1) / 3][(2 * k + 1) % 3] = {d.z, d.w};
        }
        reconstruct_row2(U);
    }
    template <class Rin>
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t blk, int64_t site, const Link<Rin>& U)
    {
        float4* p = static_cast<float4*>(base) + blk * kPlanes * S + site;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const auto a = U.u[(2 * k) / 3][(2 * k) % 3];
            const auto b = U.u[(2 * k + 1) / 3][(2 * k + 1) % 3];
            p[k * S] = make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
        }
    }
};

// FP16 links: SU(3) entries lie in [-1, 1], so no scale is needed.
template <>
struct LinkIO<16, 12> {
    using R = float;
    static constexpr int kPlanes = 0;  // mixed plane widths, see offsets below
    static constexpr int kBytesPerLink = 24;
    // block blk occupies 24*S bytes: 16*S (uint4 plane) then 8*S (uint2 plane)
    __device__ static __forceinline__ void load(const void* base, int64_t S, int64_t blk, int64_t site, Link<R>& U)
    {
        const char* b = static_cast<const char*>(base) + blk * 24 * S;
        const uint4 d = reinterpret_cast<const uint4*>(b)[site];
        const uint2 e = reinterpret_cast<const uint2*>(b + 16 * S)[site];
        const uint32_t w[6] = {d.x, d.y, d.z, d.w, e.x, e.y};
#pragma unroll
        for (int k = 0; k < 6; ++k)
            U.u[k / 3][k % 3] = {SpinorIO<16>::h2f(w[k], 0), SpinorIO<16>::h2f(w[k], 1)};
        reconstruct_row2(U);
    }
    template <class Rin>
    __device__ static __forceinline__ void store(void* base, int64_t S, int64_t blk, int64_t site, const Link<Rin>& U)
    {
        char* b = static_cast<char*>(base) + blk * 24 * S;
        uint32_t w[6];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            w[k] = SpinorIO<16>::f2h2((float)U.u[k / 3][k % 3].x, (float)U.u[k / 3][k % 3].y);
        reinterpret_cast<uint4*>(b)[site] = make_uint4(w[0], w[1], w[2], w[3]);
        reinterpret_cast<uint2*>(b + 16 * S)[site] = make_uint2(w[4], w[5]);
    }
};

__host__ __device__ inline int64_t link_bytes(int prec, int recon)
{
    if (prec == 64) return recon == 18 ? 144 : 96;
    if (prec == 32) return recon == 18 ? 72 : 48;
    return 24;
}

// ---------------------------------------------------------------------------
// Deterministic reductions.  Every thread holds N partial sums in FP64; the
// wavefront folds them with butterfly shuffles, waves are combined in LDS in
// wave order, and each block writes its N partials.  The last block to
// arrive (device-scope counter) sums the block partials in block order, so
// the result depends only on the grid shape, never on scheduling.

template <int N>
__device__ __forceinline__ void wave_reduce(double (&v)[N])
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] += __shfl_xor(v[j], off, 64);
}

// Returns true in the (single) last block; on return in that block, thread 0
// holds the grand totals in v.  Block size must be a multiple of 64, <= 1024.
template <int N>
__device__ bool block_reduce_last(double (&v)[N], double* partials, unsigned int* counter, int nblocks, int bid)
{
    __shared__ double sm[N][16];
    __shared__ int am_last;
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
            __hip_atomic_store(&partials[(int64_t)bid * N + j], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __threadfence();
        const unsigned int prev = atomicAdd(counter, 1u);
        am_last = (prev == (unsigned int)(nblocks - 1));
    }
    __syncthreads();
    if (!am_last) return false;
    __threadfence();
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
#pragma unroll
        for (int j = 0; j < N; ++j)
            v[j] += __hip_atomic_load(&partials[(int64_t)b * N + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    wave_reduce<N>(v);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < N; ++j) sm[j][wave] = v[j];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double s = 0.0;
            for (int w = 0; w < nwaves; ++w) s += sm[j][w];
            v[j] = s;
        }
        *counter = 0u;  // ready for the next launch (stream order)
    }
    return true;
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
