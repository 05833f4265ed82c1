// Spin projection / reconstruction in the chiral gamma basis.
//
// gamma_mu = [[0, e_mu], [e_mu^dag, 0]] over the spin pairs (0,1) and (2,3),
// with e_0 = -i sigma_1, e_1 = -i sigma_2, e_2 = -i sigma_3, e_3 = 1.  For
// psi = (u, l):  (1 + tau gamma_mu) psi = (h, tau e_mu^dag h),  h = u + tau e_mu l,
// so a hop needs only the 6-complex half spinor h; multiplying by e_mu or
// e_mu^dag is a permutation with phases +-1, +-i.
#pragma once

#include <hip/hip_runtime.h>

namespace dwf {

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// h = u + TAU * e_MU l for the 3 colours; p holds 24 reals (k = spin*3+colour).
template <int MU, int TAU, typename A>
__device__ __forceinline__ void project(const A *__restrict__ p, A *__restrict__ h) {
#pragma unroll
    for (int col = 0; col < 3; ++col) {
        const A u0r = p[2 * col], u0i = p[2 * col + 1];
        const A u1r = p[2 * (3 + col)], u1i = p[2 * (3 + col) + 1];
        const A l0r = p[2 * (6 + col)], l0i = p[2 * (6 + col) + 1];
        const A l1r = p[2 * (9 + col)], l1i = p[2 * (9 + col) + 1];
        A e0r, e0i, e1r, e1i;
        if constexpr (MU == 0) {  // e l = (-i l1, -i l0)
            e0r = l1i; e0i = -l1r; e1r = l0i; e1i = -l0r;
        } else if constexpr (MU == 1) {  // (-l1, l0)
            e0r = -l1r; e0i = -l1i; e1r = l0r; e1i = l0i;
        } else if constexpr (MU == 2) {  // (-i l0, i l1)
            e0r = l0i; e0i = -l0r; e1r = -l1i; e1i = l1r;
        } else {  // (l0, l1)
            e0r = l0r; e0i = l0i; e1r = l1r; e1i = l1i;
        }
        h[2 * col] = u0r + TAU * e0r;
        h[2 * col + 1] = u0i + TAU * e0i;
        h[2 * (3 + col)] = u1r + TAU * e1r;
        h[2 * (3 + col) + 1] = u1i + TAU * e1i;
    }
}

// FP16 storage: one half-spinor component u + S * l straight from the packed
// words (complex = re in the low half, im in the high half), as one v_fma_mix_f32
// (f16 operands, f32 result, one rounding).  Bit for bit the FP32 sum of the
// converted halves, without the two conversions.  LH / UH select the high half.
template <int LH, int UH, int S>
__device__ __forceinline__ float mix_add(unsigned l, unsigned u) {
    float r;
#define DWF_MIX(LS, US, C) \
    asm("v_fma_mix_f32 %0, %1, " C ", %2 op_sel:[" #LS ",0," #US "] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(l), "v"(u))
    if constexpr (S > 0) {
        if constexpr (LH == 0 && UH == 0) DWF_MIX(0, 0, "1.0");
        else if constexpr (LH == 0 && UH == 1) DWF_MIX(0, 1, "1.0");
        else if constexpr (LH == 1 && UH == 0) DWF_MIX(1, 0, "1.0");
        else DWF_MIX(1, 1, "1.0");
    } else {
        if constexpr (LH == 0 && UH == 0) DWF_MIX(0, 0, "-1.0");
        else if constexpr (LH == 0 && UH == 1) DWF_MIX(0, 1, "-1.0");
        else if constexpr (LH == 1 && UH == 0) DWF_MIX(1, 0, "-1.0");
        else DWF_MIX(1, 1, "-1.0");
    }
#undef DWF_MIX
    return r;
}

// project<MU, TAU> for FP16 storage from the 12 packed words of a spinor
// (word k = spin * 3 + colour); same identities as project.
template <int MU, int TAU>
__device__ __forceinline__ void project_f16(const unsigned *__restrict__ w, float *__restrict__ h) {
#pragma unroll
    for (int col = 0; col < 3; ++col) {
        const unsigned u0 = w[col], u1 = w[3 + col], l0 = w[6 + col], l1 = w[9 + col];
        if constexpr (MU == 0) {  // e l = (-i l1, -i l0)
            h[2 * col] = mix_add<1, 0, TAU>(l1, u0);
            h[2 * col + 1] = mix_add<0, 1, -TAU>(l1, u0);
            h[2 * (3 + col)] = mix_add<1, 0, TAU>(l0, u1);
            h[2 * (3 + col) + 1] = mix_add<0, 1, -TAU>(l0, u1);
        } else if constexpr (MU == 1) {  // (-l1, l0)
            h[2 * col] = mix_add<0, 0, -TAU>(l1, u0);
            h[2 * col + 1] = mix_add<1, 1, -TAU>(l1, u0);
            h[2 * (3 + col)] = mix_add<0, 0, TAU>(l0, u1);
            h[2 * (3 + col) + 1] = mix_add<1, 1, TAU>(l0, u1);
        } else if constexpr (MU == 2) {  // (-i l0, i l1)
            h[2 * col] = mix_add<1, 0, TAU>(l0, u0);
            h[2 * col + 1] = mix_add<0, 1, -TAU>(l0, u0);
            h[2 * (3 + col)] = mix_add<1, 0, -TAU>(l1, u1);
            h[2 * (3 + col) + 1] = mix_add<0, 1, TAU>(l1, u1);
        } else {  // (l0, l1)
            h[2 * col] = mix_add<0, 0, TAU>(l0, u0);
            h[2 * col + 1] = mix_add<1, 1, TAU>(l0, u0);
            h[2 * (3 + col)] = mix_add<0, 0, TAU>(l1, u1);
            h[2 * (3 + col) + 1] = mix_add<1, 1, TAU>(l1, u1);
        }
    }
}

// acc += (chi, TAU * e_MU^dag chi) for chi = W h (both spin components).
template <int MU, int TAU, typename A>
__device__ __forceinline__ void mul_reconstruct(const A *__restrict__ w, const A *__restrict__ h,
                                                A *__restrict__ acc) {
    A chi[12];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            A re = 0, im = 0;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const A wr = w[2 * (3 * a + b)], wi = w[2 * (3 * a + b) + 1];
                const A hr = h[2 * (3 * k + b)], hi = h[2 * (3 * k + b) + 1];
                // explicit fused multiply-adds: the library is built with -ffp-contract=off,
                // so every kernel variant rounds identically and launch shapes agree bitwise
                re = fma_(wr, hr, re);
                re = fma_(-wi, hi, re);
                im = fma_(wr, hi, im);
                im = fma_(wi, hr, im);
            }
            chi[2 * (3 * k + a)] = re;
            chi[2 * (3 * k + a) + 1] = im;
        }
#pragma unroll
    for (int col = 0; col < 3; ++col) {
        const A c0r = chi[2 * col], c0i = chi[2 * col + 1];
        const A c1r = chi[2 * (3 + col)], c1i = chi[2 * (3 + col) + 1];
        acc[2 * col] += c0r;
        acc[2 * col + 1] += c0i;
        acc[2 * (3 + col)] += c1r;
        acc[2 * (3 + col) + 1] += c1i;
        A d0r, d0i, d1r, d1i;
        if constexpr (MU == 0) {  // e^dag chi = (i c1, i c0)
            d0r = -c1i; d0i = c1r; d1r = -c0i; d1i = c0r;
        } else if constexpr (MU == 1) {  // (c1, -c0)
            d0r = c1r; d0i = c1i; d1r = -c0r; d1i = -c0i;
        } else if constexpr (MU == 2) {  // (i c0, -i c1)
            d0r = -c0i; d0i = c0r; d1r = c1i; d1i = -c1r;
        } else {
            d0r = c0r; d0i = c0i; d1r = c1r; d1i = c1i;
        }
        acc[2 * (6 + col)] += TAU * d0r;
        acc[2 * (6 + col) + 1] += TAU * d0i;
        acc[2 * (9 + col)] += TAU * d1r;
        acc[2 * (9 + col) + 1] += TAU * d1i;
    }
}

}  // namespace dwf
