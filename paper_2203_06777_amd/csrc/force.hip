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
#include <algorithm>

#include "dwf_device.h"
#include "dwf_spin.h"

namespace dwf {

// acc_{ba} += sum_k h_k(b) conj(g_k(a)) with h, g the two-spin projections
// (two colour vectors each, re/im interleaved).
__device__ inline void accum_outer(const double *h, const double *g, double *acc) {
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const double hr = h[2 * (3 * k + b)], hi = h[2 * (3 * k + b) + 1];
                const double gr = g[2 * (3 * k + a)], gi = g[2 * (3 * k + a) + 1];
                acc[2 * (3 * b + a)] += hr * gr + hi * gi;
                acc[2 * (3 * b + a) + 1] += hi * gr - hr * gi;
            }
}

// h = u + tau e_MU l with tau = +-1 held in a register (same values as the
// compile-time projection: tau * e is exact, so the fma rounds once).
template <int MU>
__device__ inline void project_tau(const double *p, double tau, double *h) {
#pragma unroll
    for (int col = 0; col < 3; ++col) {
        const double u0r = p[2 * col], u0i = p[2 * col + 1];
        const double u1r = p[2 * (3 + col)], u1i = p[2 * (3 + col) + 1];
        const double l0r = p[2 * (6 + col)], l0i = p[2 * (6 + col) + 1];
        const double l1r = p[2 * (9 + col)], l1i = p[2 * (9 + col) + 1];
        double e0r, e0i, e1r, e1i;
        if constexpr (MU == 0) {  // e l = (-i l1, -i l0)
            e0r = l1i; e0i = -l1r; e1r = l0i; e1i = -l0r;
        } else if constexpr (MU == 1) {  // (-l1, l0)
            e0r = -l1r; e0i = -l1i; e1r = l0r; e1i = l0i;
        } else if constexpr (MU == 2) {  // (-i l0, i l1)
            e0r = l0i; e0i = -l0r; e1r = -l1i; e1i = l1r;
        } else {  // (l0, l1)
            e0r = l0r; e0i = l0i; e1r = l1r; e1i = l1i;
        }
        h[2 * col] = fma_(tau, e0r, u0r);
        h[2 * col + 1] = fma_(tau, e0i, u0i);
        h[2 * (3 + col)] = fma_(tau, e1r, u1r);
        h[2 * (3 + col) + 1] = fma_(tau, e1i, u1i);
    }
}

// G_ab = (W M)_ab - (N W^dag)_ab for 3x3 complex matrices (row-major, re/im
// interleaved); w in global memory, m and n in LDS.
__device__ inline void g_entry(const double *w, const double *m, const double *n, int a, int b, double &re,
                               double &im) {
    re = 0;
    im = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double wr = w[2 * (3 * a + k)], wi = w[2 * (3 * a + k) + 1];
        const double mr = m[2 * (3 * k + b)], mi = m[2 * (3 * k + b) + 1];
        re += wr * mr - wi * mi;
        im += wr * mi + wi * mr;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double nr = n[2 * (3 * a + k)], ni = n[2 * (3 * a + k) + 1];
        const double vr = w[2 * (3 * b + k)], vi = -w[2 * (3 * b + k) + 1];
        re -= nr * vr - ni * vi;
        im -= nr * vi + ni * vr;
    }
}

struct ForceArgs {
    double *F;
    const u32x4 *X, *Y;
    const double *links[2];  // FP64 gathered links per parity (eta U in dir mu)
    long cbv;                // 16-byte vectors per checkerboard field
    unsigned vol, L0, L1, L2, L3;
    unsigned ty, tz;         // (y, z) tile of the visiting order
    unsigned ns, nblk;       // sites per workgroup, workgroups
    int Ls, kind, antiperiodic;
    double scale;
};

// Visiting order of the sites: x fastest, then t, then y and z inside a
// ty x tz tile, then the tiles.  Returns the lexicographic index of the o-th
// site and its coordinates.  A site is then read as the +t neighbour L0 sites
// before it is read as own data, as the +y neighbour L0 Lt sites before and as
// the +z neighbour L0 Lt ty sites before, so those re-reads hit L2.
__device__ inline unsigned visit_site(const ForceArgs &a, unsigned o, unsigned *x) {
    x[0] = o % a.L0;
    unsigned q = o / a.L0;
    x[3] = q % a.L3;
    q /= a.L3;
    const unsigned ly = q % a.ty;
    q /= a.ty;
    const unsigned lz = q % a.tz;
    q /= a.tz;
    const unsigned nty = a.L1 / a.ty;
    x[1] = (q % nty) * a.ty + ly;
    x[2] = (q / nty) * a.tz + lz;
    return x[0] + a.L0 * (x[1] + a.L1 * (x[2] + a.L2 * x[3]));
}

// A workgroup takes ns consecutive sites of the visiting order and all their
// links; each XCD takes one contiguous part of the workgroups.  Lane
// ((mu * 2 + term) * ns + site) * Ls + s computes the slice-s outer product of
// one term: term 0 builds M from P^- X(x+mu) and P^- Y(x), term 1 builds N from
// P^+ X(x) and P^+ Y(x+mu).  The Ls lanes of a (mu, term, site) are adjacent,
// so every spinor read is Ls consecutive 16-byte vectors, and mu is uniform
// over a wavefront whenever 2 ns Ls is a multiple of 64.  The products are
// summed over s in LDS in a fixed order (bitwise reproducible); then nine
// lanes per link form the nine colour entries of the force.
constexpr int kForceMaxThreads = 512;
constexpr int kForceMaxSites = 32;  // ns = max(1, 256 / 8 Ls) <= 32

__global__ void __launch_bounds__(kForceMaxThreads) k_force(const ForceArgs a) {
    extern __shared__ double red[];  // [mu][term][site][s][18]
    const unsigned nxcd = 8, per = (a.nblk + nxcd - 1) / nxcd;
    const unsigned lb = (blockIdx.x % nxcd) * per + blockIdx.x / nxcd;
    if (lb >= a.nblk) return;  // whole workgroup
    const int Ls = a.Ls;
    const unsigned ns = a.ns;
    const int t = threadIdx.x;
    const unsigned grp = (unsigned)t / (unsigned)Ls;
    const int s = t - (int)grp * Ls;
    const unsigned sl = grp % ns, mt = grp / ns;
    const int mu = (int)(mt >> 1), term = (int)(mt & 1);
    // the workgroup's sites: lexicographic index and coordinates, computed once
    __shared__ unsigned site_tab[kForceMaxSites][5];
    if ((unsigned)t < ns) {
        unsigned x[4] = {0, 0, 0, 0}, i = 0;
        if (lb * ns + t < a.vol) i = visit_site(a, lb * ns + t, x);
        site_tab[t][0] = i;
        for (int k = 0; k < 4; ++k) site_tab[t][1 + k] = x[k];
    }
    __syncthreads();
    const unsigned o = lb * ns + sl;
    double acc[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) acc[k] = 0;
    if (o < a.vol) {
        const unsigned i = site_tab[sl][0];
        const unsigned x[4] = {site_tab[sl][1], site_tab[sl][2], site_tab[sl][3], site_tab[sl][4]};
        const int par = (int)((x[0] + x[1] + x[2] + x[3]) & 1);
        const unsigned xm = mu == 0 ? x[0] : (mu == 1 ? x[1] : (mu == 2 ? x[2] : x[3]));
        const unsigned Lm = mu == 0 ? a.L0 : (mu == 1 ? a.L1 : (mu == 2 ? a.L2 : a.L3));
        const unsigned st = mu == 0 ? 1u : (mu == 1 ? a.L0 : (mu == 2 ? a.L0 * a.L1 : a.L0 * a.L1 * a.L2));
        const unsigned iy = xm + 1 == Lm ? i - (Lm - 1) * st : i + st;  // x + mu
        const long cx = i >> 1, cy = iy >> 1;
        const u32x4 *xs = term ? a.X + par * a.cbv : a.X + (1 - par) * a.cbv;
        const u32x4 *ys = term ? a.Y + (1 - par) * a.cbv : a.Y + par * a.cbv;
        double xv[24], yv[24], h[12], g[12];
        load_spinor<DWF_F64>(xs, term ? cx : cy, Ls, s, xv);
        load_spinor<DWF_F64>(ys, term ? cy : cx, Ls, s, yv);
        const double tau = term ? 1.0 : -1.0;
        switch (mu) {
            case 0: project_tau<0>(xv, tau, h); project_tau<0>(yv, tau, g); break;
            case 1: project_tau<1>(xv, tau, h); project_tau<1>(yv, tau, g); break;
            case 2: project_tau<2>(xv, tau, h); project_tau<2>(yv, tau, g); break;
            default: project_tau<3>(xv, tau, h); project_tau<3>(yv, tau, g); break;
        }
        accum_outer(h, g, acc);
    }
    double *mine = red + (long)t * 18;
#pragma unroll
    for (int k = 0; k < 18; ++k) mine[k] = acc[k];
    __syncthreads();
    // Lane s of a group sums components s, s + Ls, ... over the Ls slices into
    // the group's slot 0; each component has exactly one such lane.
    double *gp = red + (long)grp * Ls * 18;
    for (int k = s; k < 18; k += Ls) {
        double sum = 0;
        for (int q = 0; q < Ls; ++q) sum += gp[q * 18 + k];
        gp[k] = sum;
    }
    __syncthreads();
    for (unsigned task = t; task < ns * 36; task += blockDim.x) {
        const unsigned jl = task / 9;  // local link: site * 4 + mu
        const int e = (int)(task - jl * 9), p = e / 3, q = e - 3 * (e / 3);
        const unsigned esl = jl >> 2;
        const int emu = (int)(jl & 3);
        const unsigned eo = lb * ns + esl;
        if (eo >= a.vol) continue;
        const double *m = red + (long)((emu * 2) * ns + esl) * Ls * 18;
        const double *n = red + (long)((emu * 2 + 1) * ns + esl) * Ls * 18;
        const unsigned ei = site_tab[esl][0];
        const unsigned x[4] = {site_tab[esl][1], site_tab[esl][2], site_tab[esl][3], site_tab[esl][4]};
        double ore, oim;
        if (a.kind == 0) {  // eta (M^dag + N)
            const double eta = (a.antiperiodic && emu == 3 && x[3] == a.L3 - 1) ? -1.0 : 1.0;
            ore = eta * (m[2 * (3 * q + p)] + n[2 * (3 * p + q)]);
            oim = eta * (-m[2 * (3 * q + p) + 1] + n[2 * (3 * p + q) + 1]);
        } else {  // traceless part of (i/2)(G - G^dag), G = W M - N W^dag, W = eta U
            const int par = (int)((x[0] + x[1] + x[2] + x[3]) & 1);
            const double *w = a.links[par] + ((long)(ei >> 1) * 8 + emu) * 18;
            double gpr, gpi, gqr, gqi;
            g_entry(w, m, n, p, q, gpr, gpi);
            g_entry(w, m, n, q, p, gqr, gqi);
            ore = -0.5 * (gpi + gqi);
            oim = 0.5 * (gpr - gqr);
            if (p == q) {
                double tr = 0;
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    double grr, gri;
                    g_entry(w, m, n, r, r, grr, gri);
                    tr += -0.5 * (gri + gri);
                }
                ore -= tr / 3.0;
            }
        }
        double *f = a.F + ((long)ei * 4 + emu) * 18 + 2 * e;
        f[0] = a.scale * ore;
        f[1] = a.scale * oim;
    }
}

int launch_force(dwf_ctx ctx, double *F, const void *X, const void *Y, int kind, double scale, hipStream_t st) {
    const Geom &g = ctx->g;
    if (g.vol * 4 > 0xffffffffL) return fail(DWF_EINVAL, "dwf_force: more than 2^32 links");
    ForceArgs a;
    a.F = F;
    a.X = (const u32x4 *)X;
    a.Y = (const u32x4 *)Y;
    a.links[0] = (const double *)ctx->links[DWF_F64][0];
    a.links[1] = (const double *)ctx->links[DWF_F64][1];
    a.cbv = (long)(cb_bytes(g, DWF_F64) / 16);
    a.vol = (unsigned)g.vol;
    a.L0 = g.L[0];
    a.L1 = g.L[1];
    a.L2 = g.L[2];
    a.L3 = g.L[3];
    a.Ls = g.Ls;
    a.kind = kind;
    a.antiperiodic = g.antiperiodic;
    a.scale = scale;
    // y tile: the +z re-read distance L0 Lt ty sites of X and Y within ~2 MB
    const long site_bytes = 2L * 24 * 8 * g.Ls;
    a.ty = 1;
    for (int t : {8, 4, 2})
        if (g.L[1] % t == 0 && (long)g.L[0] * g.L[3] * t * site_bytes <= (2L << 20)) {
            a.ty = t;
            break;
        }
    a.tz = g.L[2] % 4 == 0 ? 4 : (g.L[2] % 2 == 0 ? 2 : 1);
    a.ns = (unsigned)std::max(1, 256 / (8 * g.Ls));  // 8 Ls lanes per site (<= 512 for Ls <= 64)
    a.nblk = (a.vol + a.ns - 1) / a.ns;
    const unsigned threads = a.ns * 8 * g.Ls;
    const unsigned grid = (a.nblk + 7) / 8 * 8;
    const size_t shm = (size_t)threads * 18 * sizeof(double);
    hipLaunchKernelGGL(k_force, grid, threads, shm, st, a);
    DWF_HIP(hipGetLastError());
    return DWF_OK;
}

}  // namespace dwf
