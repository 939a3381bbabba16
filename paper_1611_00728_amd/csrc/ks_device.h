// Device-side types and load/store helpers for the three storage precisions.
#pragma once

#include "ks_common.h"

namespace ks {

template <class R>
struct cx {
    R r, i;
};

template <class R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b)
{
    return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}

// acc += a * b
template <class R>
__device__ __forceinline__ void cfma(cx<R>& acc, cx<R> a, cx<R> b)
{
    acc.r = fma(a.r, b.r, acc.r);
    acc.r = fma(-a.i, b.i, acc.r);
    acc.i = fma(a.r, b.i, acc.i);
    acc.i = fma(a.i, b.r, acc.i);
}

// conj(a) * b
template <class R>
__device__ __forceinline__ cx<R> cconjmul(cx<R> a, cx<R> b)
{
    return {a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r};
}

// Storage traits: P = KS_F64 / KS_F32 / KS_F16.  R is the arithmetic type.
template <int P>
struct St;
template <>
struct St<KS_F64> {
    using R = double;
};
template <>
struct St<KS_F32> {
    using R = float;
};
template <>
struct St<KS_F16> {
    using R = float;
};

// ---------------------------------------------------------------- link entries

// bytes of one stored complex link entry
template <int P>
struct EntrySize {
    static constexpr size_t value = P == KS_F64 ? 16 : P == KS_F32 ? 8 : 4;
};

// start of plane `plane` ([plane][Vh] layout); uniform across the wave
template <int P>
__device__ __forceinline__ const void* plane_ptr(const void* base, int plane, int vh)
{
    return static_cast<const char*>(base) + (size_t)plane * (size_t)vh * EntrySize<P>::value;
}

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
typedef unsigned uvec2 __attribute__((ext_vector_type(2)));
typedef unsigned uvec4 __attribute__((ext_vector_type(4)));

// binary16 pair (round to nearest even, directly from FP64) packed into 32 bits
__device__ __forceinline__ unsigned pack_half2_from_double(double a, double b)
{
    const _Float16 ha = (_Float16)a, hb = (_Float16)b;
    unsigned short ua, ub;
    __builtin_memcpy(&ua, &ha, 2);
    __builtin_memcpy(&ub, &hb, 2);
    return (unsigned)ua | ((unsigned)ub << 16);
}

__device__ __forceinline__ cx<float> half2_to_cx(unsigned u)
{
    __half2 h;
    __builtin_memcpy(&h, &u, 4);
    const float2 f = __half22float2(h);
    return {f.x, f.y};
}

// Packed link planes.  Per slot, the N complex entries of a link occupy N * ES * lp bytes (lp
// the link pitch of the geometry, >= Vh): N / W "vector planes" of 16 bytes per site (W = 16 / ES
// entries each, site-major), then one plane holding the remaining N % W entries per site.  Every lane of a wave reads 16 bytes (or
// the remainder) of consecutive sites, so each load is one contiguous, fully used segment.
template <int P, int N>
struct LinkPack {
    static constexpr int ES = (int)EntrySize<P>::value;
    static constexpr int W = 16 / ES;
    static constexpr int NF = N / W;
    static constexpr int NR = N % W;
    // byte offset of entry e of `slot` at site h, planes of lp sites
    __host__ __device__ static size_t offset(int slot, int e, int lp, int h)
    {
        const size_t sb = (size_t)slot * N * ES * lp;
        const int j = e / W, t = e % W;
        if (j < NF) return sb + (size_t)j * 16 * lp + (size_t)h * 16 + t * ES;
        return sb + (size_t)NF * 16 * lp + (size_t)h * NR * ES + t * ES;
    }
};

// the N entries of link `slot` at site h from planes of lp sites
template <int P, int N>
__device__ __forceinline__ void load_link(const void* base, int slot, int lp, int h,
                                          cx<typename St<P>::R> m[9])
{
    using LP = LinkPack<P, N>;
    const char* sb = static_cast<const char*>(base) + (size_t)slot * N * LP::ES * lp;
#pragma unroll
    for (int j = 0; j < LP::NF; ++j) {
        const char* pl = sb + (size_t)j * 16 * lp;
        if constexpr (P == KS_F64) {
            const dvec2 v = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(pl) + h);
            m[j] = {v.x, v.y};
        } else if constexpr (P == KS_F32) {
            const fvec4 v = __builtin_nontemporal_load(reinterpret_cast<const fvec4*>(pl) + h);
            m[2 * j] = {v.x, v.y};
            m[2 * j + 1] = {v.z, v.w};
        } else {
            const uvec4 v = __builtin_nontemporal_load(reinterpret_cast<const uvec4*>(pl) + h);
            m[4 * j] = half2_to_cx(v.x);
            m[4 * j + 1] = half2_to_cx(v.y);
            m[4 * j + 2] = half2_to_cx(v.z);
            m[4 * j + 3] = half2_to_cx(v.w);
        }
    }
    if constexpr (LP::NR > 0) {
        const char* pl = sb + (size_t)LP::NF * 16 * lp;
        constexpr int o = LP::NF * LP::W;
        if constexpr (P == KS_F32) {
            const fvec2 v = __builtin_nontemporal_load(reinterpret_cast<const fvec2*>(pl) + h);
            m[o] = {v.x, v.y};
        } else if constexpr (P == KS_F16 && LP::NR == 1) {
            const unsigned v = __builtin_nontemporal_load(reinterpret_cast<const unsigned*>(pl) + h);
            m[o] = half2_to_cx(v);
        } else if constexpr (P == KS_F16 && LP::NR == 2) {
            const uvec2 v = __builtin_nontemporal_load(reinterpret_cast<const uvec2*>(pl) + h);
            m[o] = half2_to_cx(v.x);
            m[o + 1] = half2_to_cx(v.y);
        } else {
            static_assert(P == KS_F16 && LP::NR <= 2, "unsupported link packing");
        }
    }
}

// ---------------------------------------------------------------- colour vectors

// FP64: three site-major complex planes [3][Vh].  FP16: one 16-byte record per site,
// {FP32 scale n, half2 c0, half2 c1, half2 c2}, value = n * half.
template <int P>
struct Spinor;

template <>
struct Spinor<KS_F64> {
    using R = double;
    __device__ static __forceinline__ void load(const void* b, int vh, int h, cx<R> v[3])
    {
        const double2* p = static_cast<const double2*>(b);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double2 t = (p + (size_t)k * vh)[h];
            v[k] = {t.x, t.y};
        }
    }
    // v as it reads back after a store (no rounding at FP64)
    __device__ static __forceinline__ void round(cx<R>[3]) {}
    __device__ static __forceinline__ void store(void* b, int vh, int h, const cx<R> v[3])
    {
        double2* p = static_cast<double2*>(b);
#pragma unroll
        for (int k = 0; k < 3; ++k) (p + (size_t)k * vh)[h] = make_double2(v[k].r, v[k].i);
    }
};

// FP32: plane A of float4 (colours 0, 1) then plane B of float2 (colour 2), site-major.
template <>
struct Spinor<KS_F32> {
    using R = float;
    __device__ static __forceinline__ void load(const void* b, int vh, int h, cx<R> v[3])
    {
        const float4 a = static_cast<const float4*>(b)[h];
        const float2 c = reinterpret_cast<const float2*>(static_cast<const float4*>(b) + vh)[h];
        v[0] = {a.x, a.y};
        v[1] = {a.z, a.w};
        v[2] = {c.x, c.y};
    }
    __device__ static __forceinline__ void round(cx<R>[3]) {}
    __device__ static __forceinline__ void store(void* b, int vh, int h, const cx<R> v[3])
    {
        static_cast<float4*>(b)[h] = make_float4(v[0].r, v[0].i, v[1].r, v[1].i);
        reinterpret_cast<float2*>(static_cast<float4*>(b) + vh)[h] = make_float2(v[2].r, v[2].i);
    }
};

__device__ __forceinline__ unsigned pack_half2(float a, float b)
{
    const __half2 h = __floats2half2_rn(a, b);
    unsigned u;
    __builtin_memcpy(&u, &h, 4);
    return u;
}

__device__ __forceinline__ float2 unpack_half2(unsigned u)
{
    __half2 h;
    __builtin_memcpy(&h, &u, 4);
    return __half22float2(h);
}

template <>
struct Spinor<KS_F16> {
    using R = float;
    // replaces v by the values its 16-byte record decodes to
    __device__ static __forceinline__ void round(cx<R> v[3])
    {
        float n = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) n = fmaxf(n, fmaxf(fabsf(v[k].r), fabsf(v[k].i)));
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (n > 0.f) {
                const float2 a = unpack_half2(pack_half2(v[k].r / n, v[k].i / n));
                v[k] = {n * a.x, n * a.y};
            } else {
                v[k] = {0.f, 0.f};
            }
        }
    }
    __device__ static __forceinline__ void load(const void* b, int, int h, cx<R> v[3])
    {
        const uint4 rec = static_cast<const uint4*>(b)[h];
        const float n = __uint_as_float(rec.x);
        const float2 a = unpack_half2(rec.y), c = unpack_half2(rec.z), d = unpack_half2(rec.w);
        v[0] = {n * a.x, n * a.y};
        v[1] = {n * c.x, n * c.y};
        v[2] = {n * d.x, n * d.y};
    }
    __device__ static __forceinline__ void store(void* b, int, int h, const cx<R> v[3])
    {
        float n = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) n = fmaxf(n, fmaxf(fabsf(v[k].r), fabsf(v[k].i)));
        uint4 rec;
        rec.x = __float_as_uint(n);
        if (n > 0.f) {
            rec.y = pack_half2(v[0].r / n, v[0].i / n);
            rec.z = pack_half2(v[1].r / n, v[1].i / n);
            rec.w = pack_half2(v[2].r / n, v[2].i / n);
        } else {
            rec.y = rec.z = rec.w = 0u;
        }
        static_cast<uint4*>(b)[h] = rec;
    }
};

}  // namespace ks
