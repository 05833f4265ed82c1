// Fermion force: the derivative of Re(Y^dag D_h X) with respect to the links.
//
// For the link U_mu(x) the hopping term contributes
//   Y(x)^dag (1-gamma_mu) eta U X(x+mu) + Y(x+mu)^dag (1+gamma_mu) eta U^dag X(x),
// so with the spin traces taken through the half-spinor projection,
//   M_mu(x)_{ba} = sum_s sum_k h_k(b) conj(g_k(a)),  h = P^- X(x+mu,s), g = P^- Y(x,s)
//   N_mu(x)_{ba} = sum_s sum_k h_k(b) conj(g_k(a)),  h = P^+ X(x,s),    g = P^+ Y(x+mu,s)
// where P^-+ takes the two-spin projection u -+ e_mu l of (1 -+ gamma_mu).
// kind 0 writes eta (M^dag + N), the Euclidean gradient; kind 1 writes the
// traceless Hermitian part of (i/2)(G - G^dag), G = eta (U M - N U^dag).
// One lane per (site, mu); a bandwidth pass over X, Y and the links.
#include "dwf_device.h"
#include "dwf_spin.h"

namespace dwf {

template <int MU>
__device__ inline void accum_outer(const double *xa, const double *ya, const double *xb, const double *yb, double *m,
                                   double *n) {
    double h[12], g[12];
    project<MU, -1>(xa, h);
    project<MU, -1>(ya, g);
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const double hr = h[2 * (3 * k + b)], hi = h[2 * (3 * k + b) + 1];
                const double gr = g[2 * (3 * k + a)], gi = g[2 * (3 * k + a) + 1];
                m[2 * (3 * b + a)] += hr * gr + hi * gi;
                m[2 * (3 * b + a) + 1] += hi * gr - hr * gi;
            }
    project<MU, 1>(xb, h);
    project<MU, 1>(yb, g);
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const double hr = h[2 * (3 * k + b)], hi = h[2 * (3 * k + b) + 1];
                const double gr = g[2 * (3 * k + a)], gi = g[2 * (3 * k + a) + 1];
                n[2 * (3 * b + a)] += hr * gr + hi * gi;
                n[2 * (3 * b + a) + 1] += hi * gr - hr * gi;
            }
}

// c = a * b for 3x3 complex (row-major, re/im interleaved); bdag: use b^dag.
__device__ inline void mat_mul(const double *a, const double *b, double *c, bool adag, bool bdag) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double re = 0, im = 0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int ia = adag ? (3 * k + i) : (3 * i + k);
                const int ib = bdag ? (3 * j + k) : (3 * k + j);
                const double ar = a[2 * ia], ai = adag ? -a[2 * ia + 1] : a[2 * ia + 1];
                const double br = b[2 * ib], bi = bdag ? -b[2 * ib + 1] : b[2 * ib + 1];
                re += ar * br - ai * bi;
                im += ar * bi + ai * br;
            }
            c[2 * (3 * i + j)] = re;
            c[2 * (3 * i + j) + 1] = im;
        }
}

struct ForceArgs {
    double *F;
    const u32x4 *X, *Y;
    const double *links[2];  // FP64 gathered links per parity (eta U in dir mu)
    long vol, cbv;           // 4D volume; 16-byte vectors per checkerboard field
    int L0, L1, L2, L3, Ls, kind, antiperiodic;
    double scale;
};

__global__ void __launch_bounds__(256) k_force(const ForceArgs a) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= a.vol * 4) return;
    const long i = t >> 2;
    const int mu = (int)(t & 3);
    int x[4];
    x[0] = (int)(i % a.L0);
    long r = i / a.L0;
    x[1] = (int)(r % a.L1);
    r /= a.L1;
    x[2] = (int)(r % a.L2);
    x[3] = (int)(r / a.L2);
    const int par = (x[0] + x[1] + x[2] + x[3]) & 1;
    const int L[4] = {a.L0, a.L1, a.L2, a.L3};
    int y[4] = {x[0], x[1], x[2], x[3]};
    y[mu] = (x[mu] + 1) % L[mu];
    const long cx = i >> 1;
    const long cy = (y[0] + (long)a.L0 * (y[1] + (long)a.L1 * (y[2] + (long)a.L2 * y[3]))) >> 1;
    const u32x4 *Xx = a.X + par * a.cbv, *Xy = a.X + (1 - par) * a.cbv;
    const u32x4 *Yx = a.Y + par * a.cbv, *Yy = a.Y + (1 - par) * a.cbv;
    double m[18], n[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) m[k] = n[k] = 0;
    for (int s = 0; s < a.Ls; ++s) {
        double xa[24], ya[24], xb[24], yb[24];
        load_spinor<DWF_F64>(Xy, cy, a.Ls, s, xa);  // X(x+mu)
        load_spinor<DWF_F64>(Yx, cx, a.Ls, s, ya);  // Y(x)
        load_spinor<DWF_F64>(Xx, cx, a.Ls, s, xb);  // X(x)
        load_spinor<DWF_F64>(Yy, cy, a.Ls, s, yb);  // Y(x+mu)
        switch (mu) {
            case 0: accum_outer<0>(xa, ya, xb, yb, m, n); break;
            case 1: accum_outer<1>(xa, ya, xb, yb, m, n); break;
            case 2: accum_outer<2>(xa, ya, xb, yb, m, n); break;
            default: accum_outer<3>(xa, ya, xb, yb, m, n); break;
        }
    }
    double out[18];
    if (a.kind == 0) {
        const double eta = (a.antiperiodic && mu == 3 && x[3] == a.L3 - 1) ? -1.0 : 1.0;
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                out[2 * (3 * p + q)] = eta * (m[2 * (3 * q + p)] + n[2 * (3 * p + q)]);
                out[2 * (3 * p + q) + 1] = eta * (-m[2 * (3 * q + p) + 1] + n[2 * (3 * p + q) + 1]);
            }
    } else {
        const double *w = a.links[par] + (cx * 8 + mu) * 18;  // eta_mu(x) U_mu(x)
        double wl[18], g1[18], g2[18];
#pragma unroll
        for (int k = 0; k < 18; ++k) wl[k] = w[k];
        mat_mul(wl, m, g1, false, false);  // W M
        mat_mul(n, wl, g2, false, true);   // N W^dag
        double g[18];
#pragma unroll
        for (int k = 0; k < 18; ++k) g[k] = g1[k] - g2[k];
        // K = (i/2)(G - G^dag): K_pq = (i/2)(G_pq - conj(G_qp))
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const double dr = g[2 * (3 * p + q)] - g[2 * (3 * q + p)];
                const double di = g[2 * (3 * p + q) + 1] + g[2 * (3 * q + p) + 1];
                out[2 * (3 * p + q)] = -0.5 * di;
                out[2 * (3 * p + q) + 1] = 0.5 * dr;
            }
        const double tr = (out[0] + out[8] + out[16]) / 3.0;  // real part of the trace / 3
        const double tri = (out[1] + out[9] + out[17]) / 3.0;
        out[0] -= tr;
        out[8] -= tr;
        out[16] -= tr;
        out[1] -= tri;
        out[9] -= tri;
        out[17] -= tri;
    }
    double *f = a.F + t * 18;
#pragma unroll
    for (int k = 0; k < 18; ++k) f[k] = a.scale * out[k];
}

int launch_force(dwf_ctx ctx, double *F, const void *X, const void *Y, int kind, double scale, hipStream_t st) {
    const Geom &g = ctx->g;
    ForceArgs a;
    a.F = F;
    a.X = (const u32x4 *)X;
    a.Y = (const u32x4 *)Y;
    a.links[0] = (const double *)ctx->links[DWF_F64][0];
    a.links[1] = (const double *)ctx->links[DWF_F64][1];
    a.vol = g.vol;
    a.cbv = (long)(cb_bytes(g, DWF_F64) / 16);
    a.L0 = g.L[0];
    a.L1 = g.L[1];
    a.L2 = g.L[2];
    a.L3 = g.L[3];
    a.Ls = g.Ls;
    a.kind = kind;
    a.antiperiodic = g.antiperiodic;
    a.scale = scale;
    const unsigned nb = (unsigned)((g.vol * 4 + 255) / 256);
    hipLaunchKernelGGL(k_force, nb, 256, 0, st, a);
    DWF_HIP(hipGetLastError());
    return DWF_OK;
}

}  // namespace dwf
