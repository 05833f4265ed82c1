// Hopping-term core shared by the single-field and the batched kernels: the
// 8-direction stencil of one lane = (output checkerboard row c, slice s).
//
// LS > 0 fixes Ls at compile time, so the six (FP32) or twelve (FP64) 16-byte
// vectors of a neighbour spinor sit at immediate offsets from one address and
// the lane -> (site, s) split is a constant division.  O32 selects 32-bit byte
// offsets from the field's base (fields below 4 GiB).
#pragma once

#include "dwf_device.h"
#include "dwf_spin.h"

namespace dwf {

// n / d for n < 2^24 and d >= 1, from a float reciprocal plus one correction.
__device__ __forceinline__ unsigned fdiv(unsigned n, unsigned d, float inv) {
    unsigned q = (unsigned)((float)n * inv);
    const int r = (int)n - (int)(q * d);
    q = r >= (int)d ? q + 1 : (r < 0 ? q - 1 : q);
    return q;
}

struct Lat {
    unsigned L0h, L1, L2, L3;
    float inv0h, inv1, inv2;
};

template <int P, typename T, typename Off>
__device__ __forceinline__ void load_spinor_off(const char *__restrict__ base, Off off, int gstride, T *v) {
    constexpr int G = PT<P>::G, NG = 12 / G;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        typename PT<P>::A t[2 * G];
        unpack16<P>(*(const u32x4 *)(base + off + (Off)(g * gstride)), t);
#pragma unroll
        for (int j = 0; j < 2 * G; ++j) v[g * 2 * G + j] = (T)t[j];
    }
}

template <int P, typename T, typename Off>
__device__ __forceinline__ void store_spinor_off(char *__restrict__ base, Off off, int gstride, const T *v,
                                                 bool nontemporal) {
    constexpr int G = PT<P>::G, NG = 12 / G;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        typename PT<P>::A t[2 * G];
#pragma unroll
        for (int j = 0; j < 2 * G; ++j) t[j] = (typename PT<P>::A)v[g * 2 * G + j];
        u32x4 *dst = (u32x4 *)(base + off + (Off)(g * gstride));
        if (nontemporal) __builtin_nontemporal_store(pack16<P>(t), dst);
        else *dst = pack16<P>(t);
    }
}

// Byte offset of vector (row, group 0, s) in a field with NG groups per row.
template <int P, typename Off>
__device__ __forceinline__ Off spinor_off(long row, int Ls, int s) {
    constexpr int NG = 12 / PT<P>::G;
    return (Off)(((Off)row * (Off)(NG * Ls) + (Off)s) * (Off)16);
}

// Spin projection of one (site, s) from its NG 16-byte vectors.  FP16 storage
// projects straight from the packed halves (project_f16); the others unpack first.
template <int PI, int MU, int TAU>
__device__ __forceinline__ void project_vecs(const u32x4 *v, typename PT<PI>::A *h) {
    if constexpr (PI == DWF_F16) {
        unsigned w[12];
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            w[4 * g] = v[g].x;
            w[4 * g + 1] = v[g].y;
            w[4 * g + 2] = v[g].z;
            w[4 * g + 3] = v[g].w;
        }
        project_f16<MU, TAU>(w, h);
    } else {
        constexpr int R2 = 2 * PT<PI>::G, NG = 12 / PT<PI>::G;
        typename PT<PI>::A p[24];
#pragma unroll
        for (int g = 0; g < NG; ++g) unpack16<PI>(v[g], p + R2 * g);
        project<MU, TAU>(p, h);
    }
}

template <int PI, int DIR, int MU, int TAU, typename Off>
__device__ __forceinline__ void hop(const char *links, const char *in, int Ls, long c, long nb, int s,
                                    typename PT<PI>::A *acc) {
    using A = typename PT<PI>::A;
    constexpr int NG = 12 / PT<PI>::G;
    A w[18], h[12];
    load_link<PI>(links, c, DIR, w);
    u32x4 v[NG];
    const Off off = spinor_off<PI, Off>(nb, Ls, s);
#pragma unroll
    for (int g = 0; g < NG; ++g) v[g] = *(const u32x4 *)(in + off + (Off)(g * Ls * 16));
    project_vecs<PI, MU, TAU>(v, h);
    mul_reconstruct<MU, TAU>(w, h, acc);
}

// acc = (D_h psi)(c, s) (DAG: D_h^dag) for output row c of parity `parity`.
template <int PI, int DAG, typename Off>
__device__ __forceinline__ void dhop_site(const char *links, const char *in, const Lat &g, int Ls, int parity, long c,
                                          int s, typename PT<PI>::A *acc) {
    const unsigned L0 = 2 * g.L0h;
    const unsigned uc = (unsigned)c;
    const unsigned rest = fdiv(uc, g.L0h, g.inv0h);
    const unsigned xh = uc - rest * g.L0h;
    const unsigned r2 = fdiv(rest, g.L1, g.inv1);
    const unsigned x1 = rest - r2 * g.L1;
    const unsigned x3 = fdiv(r2, g.L2, g.inv2);
    const unsigned x2 = r2 - x3 * g.L2;
    const unsigned x0 = 2 * xh + ((parity + x1 + x2 + x3) & 1);
    const long s2 = g.L1, s3 = (long)g.L1 * g.L2;
    const long lrest = rest;
    const long nb0 = lrest * g.L0h + ((x0 + 1 == L0 ? 0 : x0 + 1) >> 1);
    const long nb4 = lrest * g.L0h + ((x0 == 0 ? L0 - 1 : x0 - 1) >> 1);
    const long nb1 = (lrest + (x1 + 1 == g.L1 ? -(long)(g.L1 - 1) : 1)) * g.L0h + xh;
    const long nb5 = (lrest + (x1 == 0 ? (long)(g.L1 - 1) : -1)) * g.L0h + xh;
    const long nb2 = (lrest + (x2 + 1 == g.L2 ? -(long)(g.L2 - 1) * s2 : s2)) * g.L0h + xh;
    const long nb6 = (lrest + (x2 == 0 ? (long)(g.L2 - 1) * s2 : -s2)) * g.L0h + xh;
    const long nb3 = (lrest + (x3 + 1 == g.L3 ? -(long)(g.L3 - 1) * s3 : s3)) * g.L0h + xh;
    const long nb7 = (lrest + (x3 == 0 ? (long)(g.L3 - 1) * s3 : -s3)) * g.L0h + xh;
    constexpr int SG = DAG ? 1 : -1;
    hop<PI, 0, 0, SG, Off>(links, in, Ls, c, nb0, s, acc);
    hop<PI, 1, 1, SG, Off>(links, in, Ls, c, nb1, s, acc);
    hop<PI, 2, 2, SG, Off>(links, in, Ls, c, nb2, s, acc);
    hop<PI, 3, 3, SG, Off>(links, in, Ls, c, nb3, s, acc);
    hop<PI, 4, 0, -SG, Off>(links, in, Ls, c, nb4, s, acc);
    hop<PI, 5, 1, -SG, Off>(links, in, Ls, c, nb5, s, acc);
    hop<PI, 6, 2, -SG, Off>(links, in, Ls, c, nb6, s, acc);
    hop<PI, 7, 3, -SG, Off>(links, in, Ls, c, nb7, s, acc);
}

inline Lat make_lat(const int *L) {
    Lat g;
    g.L0h = (unsigned)(L[0] / 2);
    g.L1 = (unsigned)L[1];
    g.L2 = (unsigned)L[2];
    g.L3 = (unsigned)L[3];
    g.inv0h = 1.0f / (float)g.L0h;
    g.inv1 = 1.0f / (float)g.L1;
    g.inv2 = 1.0f / (float)g.L2;
    return g;
}

}  // namespace dwf
