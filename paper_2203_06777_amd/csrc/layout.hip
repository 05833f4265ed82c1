// Canonical <-> internal layout conversion, link gathering and precision
// conversion.  These run once per gauge / field load and are not on the
// timed path of the operator.
#include "dwf_device.h"

namespace dwf {

// Canonical checkerboard field [V/2][Ls][4][3] or full field [V][Ls][4][3]
// (lex order) <-> internal.  One lane per (site, s).
template <int P, int TO_INTERNAL>
__global__ void k_layout(u32x4 *internal, double *canonical, long nsites, int Ls, int full, int L0, int L1, int L2,
                         long cb_vec16) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nsites * Ls) return;
    const long i = t / Ls;
    const int s = (int)(t - i * Ls);
    long c = i;
    u32x4 *base = internal;
    if (full) {
        const long x0 = i % L0, r = i / L0;
        const long x1 = r % L1, r2 = r / L1;
        const long x2 = r2 % L2, x3 = r2 / L2;
        const int par = (int)((x0 + x1 + x2 + x3) & 1);
        c = i >> 1;
        base = internal + par * cb_vec16;
    }
    double *cp = canonical + (i * Ls + s) * 24;
    double v[24];
    if (TO_INTERNAL) {
#pragma unroll
        for (int k = 0; k < 24; ++k) v[k] = cp[k];
        store_spinor<P>(base, c, Ls, s, v);
    } else {
        load_spinor<P>(base, c, Ls, s, v);
#pragma unroll
        for (int k = 0; k < 24; ++k) cp[k] = v[k];
    }
}

template <int P> __device__ inline void store_cplx(void *base, long idx, double re, double im);
template <> __device__ inline void store_cplx<DWF_F64>(void *base, long idx, double re, double im) {
    ((double *)base)[2 * idx] = re;
    ((double *)base)[2 * idx + 1] = im;
}
template <> __device__ inline void store_cplx<DWF_F32>(void *base, long idx, double re, double im) {
    ((float *)base)[2 * idx] = (float)re;
    ((float *)base)[2 * idx + 1] = (float)im;
}
template <> __device__ inline void store_cplx<DWF_F16>(void *base, long idx, double re, double im) {
    ((unsigned short *)base)[2 * idx] = f32_to_f16_bits((float)re);
    ((unsigned short *)base)[2 * idx + 1] = f32_to_f16_bits((float)im);
}
template <> __device__ inline void store_cplx<DWF_BF16>(void *base, long idx, double re, double im) {
    ((unsigned short *)base)[2 * idx] = f32_to_bf16_bits((float)re);
    ((unsigned short *)base)[2 * idx + 1] = f32_to_bf16_bits((float)im);
}

// links[c][dir][a][b]: dir = mu: eta_mu(x) U_mu(x); dir = 4+mu: (eta_mu(x-mu) U_mu(x-mu))^dag.
template <int P>
__global__ void k_gather_links(void *links, const double *U, long half, int L0, int L1, int L2, int L3, int parity,
                               int antiperiodic) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= half * 8) return;
    const long c = t >> 3;
    const int dir = (int)(t & 7);
    const int mu = dir & 3;
    const long xh = c % (L0 / 2), rest = c / (L0 / 2);
    int x[4];
    x[1] = (int)(rest % L1);
    x[2] = (int)((rest / L1) % L2);
    x[3] = (int)(rest / ((long)L1 * L2));
    x[0] = (int)(2 * xh + ((parity + x[1] + x[2] + x[3]) & 1));
    const int L[4] = {L0, L1, L2, L3};
    if (dir >= 4) x[mu] = (x[mu] + L[mu] - 1) % L[mu];
    const double eta = (antiperiodic && mu == 3 && x[3] == L3 - 1) ? -1.0 : 1.0;
    const long lex = x[0] + (long)L0 * (x[1] + (long)L1 * (x[2] + (long)L2 * x[3]));
    const double *u = U + (lex * 4 + mu) * 18;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double re, im;
            if (dir < 4) {
                re = u[2 * (3 * a + b)];
                im = u[2 * (3 * a + b) + 1];
            } else {
                re = u[2 * (3 * b + a)];
                im = -u[2 * (3 * b + a) + 1];
            }
            store_cplx<P>(links, (c * 8 + dir) * 9 + 3 * a + b, eta * re, eta * im);
        }
}

template <int PI, int PO>
__global__ void k_convert(u32x4 *out, const u32x4 *in, long nrows, int Ls) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows * Ls) return;
    const long c = t / Ls;
    const int s = (int)(t - c * Ls);
    double v[24];
    load_spinor<PI>(in, c, Ls, s, v);
    store_spinor<PO>(out, c, Ls, s, v);
}

static inline unsigned nblk(long n, int th) { return (unsigned)((n + th - 1) / th); }

template <int TO>
static int layout_dispatch(const Geom &g, void *internal, double *canonical, int parity, int prec, hipStream_t st) {
    const long nsites = parity == 2 ? g.vol : g.half;
    const int full = parity == 2;
    const long cbv = (long)(cb_bytes(g, prec) / 16);
    const int th = 256;
    const unsigned nb = nblk(nsites * g.Ls, th);
    u32x4 *in = (u32x4 *)internal;
    switch (prec) {
        case DWF_F64:
            hipLaunchKernelGGL((k_layout<DWF_F64, TO>), nb, th, 0, st, in, canonical, nsites, g.Ls, full, g.L[0], g.L[1],
                               g.L[2], cbv);
            break;
        case DWF_F32:
            hipLaunchKernelGGL((k_layout<DWF_F32, TO>), nb, th, 0, st, in, canonical, nsites, g.Ls, full, g.L[0], g.L[1],
                               g.L[2], cbv);
            break;
        case DWF_F16:
            hipLaunchKernelGGL((k_layout<DWF_F16, TO>), nb, th, 0, st, in, canonical, nsites, g.Ls, full, g.L[0], g.L[1],
                               g.L[2], cbv);
            break;
        default:
            hipLaunchKernelGGL((k_layout<DWF_BF16, TO>), nb, th, 0, st, in, canonical, nsites, g.Ls, full, g.L[0],
                               g.L[1], g.L[2], cbv);
            break;
    }
    DWF_HIP(hipGetLastError());
    return DWF_OK;
}

int launch_pack(const Geom &g, void *internal, const double *canonical, int parity, int prec, hipStream_t st) {
    return layout_dispatch<1>(g, internal, const_cast<double *>(canonical), parity, prec, st);
}

int launch_unpack(const Geom &g, double *canonical, const void *internal, int parity, int prec, hipStream_t st) {
    return layout_dispatch<0>(g, const_cast<void *>(internal), canonical, parity, prec, st);
}

int launch_gather_links(const Geom &g, void *links, const double *U, int p, int prec, hipStream_t st) {
    const int th = 256;
    const unsigned nb = nblk(g.half * 8, th);
    switch (prec) {
        case DWF_F64:
            hipLaunchKernelGGL(k_gather_links<DWF_F64>, nb, th, 0, st, links, U, g.half, g.L[0], g.L[1], g.L[2], g.L[3],
                               p, g.antiperiodic);
            break;
        case DWF_F32:
            hipLaunchKernelGGL(k_gather_links<DWF_F32>, nb, th, 0, st, links, U, g.half, g.L[0], g.L[1], g.L[2], g.L[3],
                               p, g.antiperiodic);
            break;
        case DWF_F16:
            hipLaunchKernelGGL(k_gather_links<DWF_F16>, nb, th, 0, st, links, U, g.half, g.L[0], g.L[1], g.L[2], g.L[3],
                               p, g.antiperiodic);
            break;
        default:
            hipLaunchKernelGGL(k_gather_links<DWF_BF16>, nb, th, 0, st, links, U, g.half, g.L[0], g.L[1], g.L[2],
                               g.L[3], p, g.antiperiodic);
            break;
    }
    DWF_HIP(hipGetLastError());
    return DWF_OK;
}

template <int PI>
static int convert_from(u32x4 *out, int po, const u32x4 *in, long nrows, int Ls, hipStream_t st) {
    const int th = 256;
    const unsigned nb = nblk(nrows * Ls, th);
    switch (po) {
        case DWF_F64: hipLaunchKernelGGL((k_convert<PI, DWF_F64>), nb, th, 0, st, out, in, nrows, Ls); break;
        case DWF_F32: hipLaunchKernelGGL((k_convert<PI, DWF_F32>), nb, th, 0, st, out, in, nrows, Ls); break;
        case DWF_F16: hipLaunchKernelGGL((k_convert<PI, DWF_F16>), nb, th, 0, st, out, in, nrows, Ls); break;
        default: hipLaunchKernelGGL((k_convert<PI, DWF_BF16>), nb, th, 0, st, out, in, nrows, Ls); break;
    }
    DWF_HIP(hipGetLastError());
    return DWF_OK;
}

int launch_convert(const Geom &g, void *out, int po, const void *in, int pi, long ncb, hipStream_t st) {
    const long nrows = g.half * ncb;  // a full field is two checkerboards back to back
    u32x4 *o = (u32x4 *)out;
    const u32x4 *i = (const u32x4 *)in;
    switch (pi) {
        case DWF_F64: return convert_from<DWF_F64>(o, po, i, nrows, g.Ls, st);
        case DWF_F32: return convert_from<DWF_F32>(o, po, i, nrows, g.Ls, st);
        case DWF_F16: return convert_from<DWF_F16>(o, po, i, nrows, g.Ls, st);
        default: return convert_from<DWF_BF16>(o, po, i, nrows, g.Ls, st);
    }
}

}  // namespace dwf
