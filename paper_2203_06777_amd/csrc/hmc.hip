// Link update of the hybrid Monte Carlo molecular dynamics: U <- exp(i eps P) U
// for every link, with P traceless Hermitian (the su(3) momenta) in the
// canonical gauge layout [V][4][3][3] (complex FP64).
//
// exp(A), A = i eps P, by scaling and squaring: B = A / 2^k with |B|_F <= 1/2,
// the degree-14 Taylor polynomial of exp(B) in Horner form
// (T = 1 + B/n (1 + B/(n-1) (...)), truncation error below 1e-17 |B|^15 / 15!),
// then k squarings.  One lane per link; a pass over P and U.
#include <cmath>

#include "dwf_common.h"

namespace dwf {

// c = a b for 3x3 complex matrices (row-major, re/im interleaved).
__device__ inline void mul33(const double *a, const double *b, double *c) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double re = 0, im = 0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double ar = a[2 * (3 * i + k)], ai = a[2 * (3 * i + k) + 1];
                const double br = b[2 * (3 * k + j)], bi = b[2 * (3 * k + j) + 1];
                re += ar * br - ai * bi;
                im += ar * bi + ai * br;
            }
            c[2 * (3 * i + j)] = re;
            c[2 * (3 * i + j) + 1] = im;
        }
}

constexpr int kTaylorDegree = 14;

__global__ void __launch_bounds__(256) k_expi_links(double *U, const double *P, double eps, long nlinks) {
    const long l = (long)blockIdx.x * 256 + threadIdx.x;
    if (l >= nlinks) return;
    const double *p = P + l * 18;
    double b[18], nrm = 0;
    // B = i eps P (re <- -eps Im P, im <- eps Re P)
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        b[2 * k] = -eps * p[2 * k + 1];
        b[2 * k + 1] = eps * p[2 * k];
        nrm += b[2 * k] * b[2 * k] + b[2 * k + 1] * b[2 * k + 1];
    }
    nrm = sqrt(nrm);
    int sq = 0;
    double scale = 1.0;
    while (nrm * scale > 0.5 && sq < 60) {
        scale *= 0.5;
        ++sq;
    }
#pragma unroll
    for (int k = 0; k < 18; ++k) b[k] *= scale;
    // Horner: T = 1 + B/n T
    double t[18], w[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) t[k] = (k == 0 || k == 8 || k == 16) ? 1.0 : 0.0;
    for (int n = kTaylorDegree; n >= 1; --n) {
        mul33(b, t, w);
        const double inv = 1.0 / n;
#pragma unroll
        for (int k = 0; k < 18; ++k) t[k] = w[k] * inv + ((k == 0 || k == 8 || k == 16) ? 1.0 : 0.0);
    }
    for (int i = 0; i < sq; ++i) {
        mul33(t, t, w);
#pragma unroll
        for (int k = 0; k < 18; ++k) t[k] = w[k];
    }
    double *u = U + l * 18;
    double uo[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) uo[k] = u[k];
    mul33(t, uo, w);
#pragma unroll
    for (int k = 0; k < 18; ++k) u[k] = w[k];
}

int launch_expi_links(const Geom &g, double *U, const double *P, double eps, hipStream_t st) {
    const long n = g.vol * 4;
    hipLaunchKernelGGL(k_expi_links, (unsigned)((n + 255) / 256), 256, 0, st, U, P, eps, n);
    DWF_HIP(hipGetLastError());
    return DWF_OK;
}

}  // namespace dwf
