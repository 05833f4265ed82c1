// Inverse of the site-local fifth-dimension term, Mooee^-1 (Shamir: M5op^-1), applied to the
// Ls-vectors of the sites a workgroup holds, through LDS.
//
// Per chirality Mooee = d - e K with the twisted shift K: lower spins couple s to s+1, upper
// spins s to s-1 (the adjoint swaps the two), and the hop across the wall carries -mf.  The
// system (d - e K) y = v is a first-order recurrence along s; for the lower spins
//     y(s) = (v(s) + e y(s+1)) / d               for s < Ls-1,
// closed at the wall by the one value the geometric series of the inverse gives directly,
//     y(Ls-1) = sum_n coef[n] (K^n v)(Ls-1) = coef[0] v(Ls-1) - mf sum_{n>=1} coef[n] v(n-1),
// coef[n] = (e/d)^n / (d (1 + mf (e/d)^Ls)); the upper spins run the mirror image from s = 0.
// One lane solves one colour-spin component of one site (the site's Ls lanes share its 24
// components), so a component costs O(Ls) instead of the O(Ls^2) of the dense series.
//
// With the Moebius Schur factor the result is Mooee^-1 (b + c K) v = f y + g v, f = b + c d/e,
// g = -c/e (b + c K differs from Mooee by a multiple of the identity).
#pragma once

#include <hip/hip_runtime.h>

#include "dwf_common.h"
#include "dwf_spin.h"

namespace dwf {

struct M5InvCoef {
    double coef[kMaxLs];  // coef[n] of the series, n < Ls
    double mf;            // wall factor
    double id, ed;        // 1/d and e/d of the recurrence
    double f, g;          // Schur factor y -> f y + g v (used when schur != 0)
    int schur;
};

// Host side: the coefficients of Mooee^-1 for g (and of the Moebius Schur factor when schur).
void m5inv_setup(const Geom &geom, M5InvCoef &m, bool schur);

// v (24 reals of lane (site j, slice s)) <- Mooee^-1 v, or Mooee^-dag v when DAG.  lds holds
// at least (j + 1) * Ls * 25 reals for every site j of the workgroup.  Every lane of the
// workgroup calls it (two barriers); lanes without a site pass zeros.
template <int DAG, typename A>
__device__ __forceinline__ void m5inv_lds(const M5InvCoef &m, int Ls, A *lds, int j, int s, A *v) {
    A *site = lds + j * Ls * 25;
    A *mine = site + s * 25;
#pragma unroll
    for (int k = 0; k < 24; ++k) mine[k] = v[k];
    __syncthreads();
    const A id = (A)m.id, ed = (A)m.ed, mfn = (A)(-m.mf), f = (A)m.f, g = (A)m.g;
    for (int k = s; k < 24; k += Ls) {
        // forward components couple s to s+1: they start at the top of the site (s = Ls-1)
        const bool fwd = (k >= 12) != (DAG != 0);
        A *col = site + k;
        const int s0 = fwd ? Ls - 1 : 0;
        A y = (A)m.coef[0] * col[s0 * 25];
        for (int n = 1; n < Ls; ++n) {
            const int sn = fwd ? n - 1 : Ls - n;  // (K^n v)(s0) is -mf v(sn)
            y = fma_(mfn * (A)m.coef[n], col[sn * 25], y);
        }
        const int step = fwd ? -25 : 25;
        A *p = col + s0 * 25;
        A vv = *p;
        *p = m.schur ? fma_(f, y, g * vv) : y;
        for (int u = 1; u < Ls; ++u) {
            p += step;
            vv = *p;
            y = fma_(ed, y, id * vv);
            *p = m.schur ? fma_(f, y, g * vv) : y;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = mine[k];
}

}  // namespace dwf
