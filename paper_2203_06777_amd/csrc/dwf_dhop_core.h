// Hopping-term core shared by the single-field and the batched kernels:
// the 8-direction stencil of one output lane (checkerboard row c, slice s).
#pragma once

#include "dwf_device.h"
#include "dwf_spin.h"

namespace dwf {

template <int PI, int DIR, int MU, int TAU>
__device__ __forceinline__ void hop(const void *links, const u32x4 *in, int Ls, long c, long nb, int s,
                                    typename PT<PI>::A *acc) {
    using A = typename PT<PI>::A;
    A w[18], p[24], h[12];
    load_link<PI>(links, c, DIR, w);
    load_spinor<PI>(in, nb, Ls, s, p);
    project<MU, TAU>(p, h);
    mul_reconstruct<MU, TAU>(w, h, acc);
}

// acc = (D_h psi)(c, s) (DAG: D_h^dag) for output row c of parity `parity`.
template <int PI, int DAG>
__device__ __forceinline__ void dhop_site(const void *links, const u32x4 *in, int L0h, int L1, int L2, int L3,
                                          int Ls, int parity, long c, int s, typename PT<PI>::A *acc) {
    const int L0 = 2 * L0h;
    const int xh = (int)(c % L0h);
    const long rest = c / L0h;
    const int x1 = (int)(rest % L1);
    const long r2 = rest / L1;
    const int x2 = (int)(r2 % L2);
    const int x3 = (int)(r2 / L2);
    const int x0 = 2 * xh + ((parity + x1 + x2 + x3) & 1);
    const long s2 = L1, s3 = (long)L1 * L2;
    const long nb0 = rest * L0h + ((x0 + 1 == L0 ? 0 : x0 + 1) >> 1);
    const long nb4 = rest * L0h + ((x0 == 0 ? L0 - 1 : x0 - 1) >> 1);
    const long nb1 = (rest + (x1 + 1 == L1 ? -(long)(L1 - 1) : 1)) * L0h + xh;
    const long nb5 = (rest + (x1 == 0 ? (long)(L1 - 1) : -1)) * L0h + xh;
    const long nb2 = (rest + (x2 + 1 == L2 ? -(long)(L2 - 1) * s2 : s2)) * L0h + xh;
    const long nb6 = (rest + (x2 == 0 ? (long)(L2 - 1) * s2 : -s2)) * L0h + xh;
    const long nb3 = (rest + (x3 + 1 == L3 ? -(long)(L3 - 1) * s3 : s3)) * L0h + xh;
    const long nb7 = (rest + (x3 == 0 ? (long)(L3 - 1) * s3 : -s3)) * L0h + xh;
    constexpr int SG = DAG ? 1 : -1;
    hop<PI, 0, 0, SG>(links, in, Ls, c, nb0, s, acc);
    hop<PI, 1, 1, SG>(links, in, Ls, c, nb1, s, acc);
    hop<PI, 2, 2, SG>(links, in, Ls, c, nb2, s, acc);
    hop<PI, 3, 3, SG>(links, in, Ls, c, nb3, s, acc);
    hop<PI, 4, 0, -SG>(links, in, Ls, c, nb4, s, acc);
    hop<PI, 5, 1, -SG>(links, in, Ls, c, nb5, s, acc);
    hop<PI, 6, 2, -SG>(links, in, Ls, c, nb6, s, acc);
    hop<PI, 7, 3, -SG>(links, in, Ls, c, nb7, s, acc);
}

}  // namespace dwf
