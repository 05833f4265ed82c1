// Device helpers: 16-byte spinor vector loads/stores in every storage
// precision, conversions, and the XCD-aware workgroup remap.
#pragma once

#include <hip/hip_runtime.h>

#include "dwf_common.h"

namespace dwf {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// ---- bf16 <-> f32 (round to nearest even; NaN stays NaN) -------------------
__device__ __host__ inline unsigned short f32_to_bf16_bits(float f) {
    const unsigned int u = __builtin_bit_cast(unsigned int, f);
    const unsigned int rounded = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    const unsigned int quiet = (u >> 16) | 0x40u;  // NaN stays NaN (quiet bit set)
    return (unsigned short)((u & 0x7fffffffu) > 0x7f800000u ? quiet : rounded);
}
__device__ __host__ inline float bf16_bits_to_f32(unsigned short b) {
    return __builtin_bit_cast(float, (unsigned int)b << 16);
}
__device__ inline unsigned short f32_to_f16_bits(float f) {
    _Float16 h = (_Float16)f;
    return __builtin_bit_cast(unsigned short, h);
}
__device__ inline float f16_bits_to_f32(unsigned short b) { return (float)__builtin_bit_cast(_Float16, b); }

// ---- unpack one 16-byte vector into 2G reals of the arithmetic type ---------
template <int P> __device__ inline void unpack16(const u32x4 &r, typename PT<P>::A *v);
template <> __device__ inline void unpack16<DWF_F64>(const u32x4 &r, double *v) {
    unsigned long long a = ((unsigned long long)r.y << 32) | r.x;
    unsigned long long b = ((unsigned long long)r.w << 32) | r.z;
    v[0] = __builtin_bit_cast(double, a);
    v[1] = __builtin_bit_cast(double, b);
}
template <> __device__ inline void unpack16<DWF_F32>(const u32x4 &r, float *v) {
    // copy the lanes to scalars first: bit-casting a vector-element lvalue
    // directly reads element 0 with this compiler
    const unsigned x = r.x, y = r.y, z = r.z, w = r.w;
    v[0] = __builtin_bit_cast(float, x);
    v[1] = __builtin_bit_cast(float, y);
    v[2] = __builtin_bit_cast(float, z);
    v[3] = __builtin_bit_cast(float, w);
}
template <> __device__ inline void unpack16<DWF_F16>(const u32x4 &r, float *v) {
    unsigned int w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[2 * k] = f16_bits_to_f32((unsigned short)(w[k] & 0xffffu));
        v[2 * k + 1] = f16_bits_to_f32((unsigned short)(w[k] >> 16));
    }
}
template <> __device__ inline void unpack16<DWF_BF16>(const u32x4 &r, float *v) {
    unsigned int w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[2 * k] = bf16_bits_to_f32((unsigned short)(w[k] & 0xffffu));
        v[2 * k + 1] = bf16_bits_to_f32((unsigned short)(w[k] >> 16));
    }
}

template <int P> __device__ inline u32x4 pack16(const typename PT<P>::A *v);
template <> __device__ inline u32x4 pack16<DWF_F64>(const double *v) {
    unsigned long long a = __builtin_bit_cast(unsigned long long, v[0]);
    unsigned long long b = __builtin_bit_cast(unsigned long long, v[1]);
    return u32x4{(unsigned)a, (unsigned)(a >> 32), (unsigned)b, (unsigned)(b >> 32)};
}
template <> __device__ inline u32x4 pack16<DWF_F32>(const float *v) {
    return u32x4{__builtin_bit_cast(unsigned, v[0]), __builtin_bit_cast(unsigned, v[1]),
                 __builtin_bit_cast(unsigned, v[2]), __builtin_bit_cast(unsigned, v[3])};
}
template <> __device__ inline u32x4 pack16<DWF_F16>(const float *v) {
    unsigned w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        w[k] = (unsigned)f32_to_f16_bits(v[2 * k]) | ((unsigned)f32_to_f16_bits(v[2 * k + 1]) << 16);
    return u32x4{w[0], w[1], w[2], w[3]};
}
template <> __device__ inline u32x4 pack16<DWF_BF16>(const float *v) {
    unsigned w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        w[k] = (unsigned)f32_to_bf16_bits(v[2 * k]) | ((unsigned)f32_to_bf16_bits(v[2 * k + 1]) << 16);
    return u32x4{w[0], w[1], w[2], w[3]};
}

// ---- whole spinor (24 reals, component k = spin*3 + colour) ----------------
// base points at the field's first 16-byte vector; c = checkerboard row.
template <int P, typename T>
__device__ inline void load_spinor(const u32x4 *__restrict__ base, long c, int Ls, int s, T *v) {
    constexpr int G = PT<P>::G, NG = 12 / G;
    const u32x4 *p = base + (c * NG) * Ls + s;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        typename PT<P>::A t[2 * G];
        unpack16<P>(p[(long)g * Ls], t);
#pragma unroll
        for (int j = 0; j < 2 * G; ++j) v[g * 2 * G + j] = (T)t[j];
    }
}

template <int P, typename T>
__device__ inline void store_spinor(u32x4 *__restrict__ base, long c, int Ls, int s, const T *v) {
    constexpr int G = PT<P>::G, NG = 12 / G;
    u32x4 *p = base + (c * NG) * Ls + s;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        typename PT<P>::A t[2 * G];
#pragma unroll
        for (int j = 0; j < 2 * G; ++j) t[j] = (typename PT<P>::A)v[g * 2 * G + j];
        p[(long)g * Ls] = pack16<P>(t);
    }
}

// ---- links: 9 complex per direction, storage precision --------------------
template <int P> __device__ inline void load_link(const void *links, long c, int dir, typename PT<P>::A *w);
template <> __device__ inline void load_link<DWF_F64>(const void *links, long c, int dir, double *w) {
    const u32x4 *p = (const u32x4 *)links + (c * 8 + dir) * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) unpack16<DWF_F64>(p[k], w + 2 * k);
}
template <> __device__ inline void load_link<DWF_F32>(const void *links, long c, int dir, float *w) {
    const u32x2 *p = (const u32x2 *)links + (c * 8 + dir) * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const u32x2 r = p[k];
        const unsigned re = r.x, im = r.y;
        w[2 * k] = __builtin_bit_cast(float, re);
        w[2 * k + 1] = __builtin_bit_cast(float, im);
    }
}
template <> __device__ inline void load_link<DWF_F16>(const void *links, long c, int dir, float *w) {
    const unsigned *p = (const unsigned *)links + (c * 8 + dir) * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        unsigned r = p[k];
        w[2 * k] = f16_bits_to_f32((unsigned short)(r & 0xffffu));
        w[2 * k + 1] = f16_bits_to_f32((unsigned short)(r >> 16));
    }
}
template <> __device__ inline void load_link<DWF_BF16>(const void *links, long c, int dir, float *w) {
    const unsigned *p = (const unsigned *)links + (c * 8 + dir) * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        unsigned r = p[k];
        w[2 * k] = bf16_bits_to_f32((unsigned short)(r & 0xffffu));
        w[2 * k + 1] = bf16_bits_to_f32((unsigned short)(r >> 16));
    }
}

// ---- XCD-aware workgroup remap ----------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Remapping gives each XCD one contiguous range of logical tiles, so
// neighbouring tiles, which share input spinors, hit the same L2.
__device__ inline long xcd_remap(long b, long nb) {
    constexpr long X = 8;
    long q = nb / X, r = nb % X;
    long xcd = b % X, k = b / X;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

}  // namespace dwf
