// Fifth-dimension term on its own: Mooee = d - e K and its adjoint and inverse
// (Shamir: d = 5 - M5, e = 1, i.e. M5op), and the general site-local
// combination (d x + db z) - K (e x + eb z) the Moebius operator needs.
//
// One lane per (4D site, s); the Ls lanes of a site exchange their spinors
// through LDS, so the kernel reads and writes each field once and out may
// alias an input.  K couples s to s +- 1 (P_- to s+1, P_+ to s-1, with -mf on
// the wraps); the inverse solves, per chirality and component, the first-order
// recurrence along s closed at the wall (dwf_m5inv.h).
#include "dwf_device.h"
#include "dwf_m5inv.h"

namespace dwf {

struct M5Args {
    const u32x4 *in, *in2;  // x, z (z may be null)
    u32x4 *out;
    long nsites;
    int Ls, spb, dagger, inverse;
    double d, e, db, eb, mf;
    M5InvCoef m5i;
};

template <typename A>
__device__ __forceinline__ void m5inv_lds_dyn(const M5Args &a, int Ls, A *lds, int j, int s, A *v) {
    if (a.dagger) m5inv_lds<1>(a.m5i, Ls, lds, j, s, v);
    else m5inv_lds<0>(a.m5i, Ls, lds, j, s, v);
}

template <int P>
__global__ void __launch_bounds__(1024) k_m5(const M5Args a) {
    using A = typename PT<P>::A;
    extern __shared__ unsigned char smem[];
    A *lds = reinterpret_cast<A *>(smem);
    const int Ls = a.Ls;
    const int j = threadIdx.x / Ls;
    const int s = threadIdx.x - j * Ls;
    const long c = (long)blockIdx.x * a.spb + j;
    const bool active = c < a.nsites;
    A v[24], w[24];
    if (active) load_spinor<P>(a.in, c, Ls, s, v);
    else
#pragma unroll
        for (int k = 0; k < 24; ++k) v[k] = 0;
    if (a.inverse) {
#pragma unroll
        for (int k = 0; k < 24; ++k) w[k] = v[k];
    } else {
        // own term d x (+ db z) and the shifted one e x (+ eb z)
        const A d = (A)a.d, e = (A)a.e;
        if (a.in2 && active) {
            A z[24];
            load_spinor<P>(a.in2, c, Ls, s, z);
            const A db = (A)a.db, eb = (A)a.eb;
#pragma unroll
            for (int k = 0; k < 24; ++k) {
                w[k] = e * v[k] + eb * z[k];
                v[k] = d * v[k] + db * z[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < 24; ++k) {
                w[k] = e * v[k];
                v[k] = d * v[k];
            }
        }
    }
    if (a.inverse) {  // every lane of the workgroup takes part (two barriers)
        m5inv_lds_dyn(a, Ls, lds, j, s, w);
        if (!active) return;
        store_spinor<P>(a.out, c, Ls, s, w);
        return;
    }
    A *mine = lds + (j * Ls + s) * 25;
#pragma unroll
    for (int k = 0; k < 24; ++k) mine[k] = w[k];
    __syncthreads();
    if (!active) return;
    const A *site = lds + j * Ls * 25;
    const A mf = (A)a.mf;
    A o[24];
    const int su = s + 1 < Ls ? s + 1 : 0, sd = s >= 1 ? s - 1 : Ls - 1;
    const A fu = s + 1 < Ls ? (A)1 : -mf, fd = s >= 1 ? (A)1 : -mf;
    const A *zu = site + su * 25, *zd = site + sd * 25;
    // upper spins: P_+ takes s-1 (adjoint: s+1); lower spins: P_- takes s+1 (adjoint: s-1)
#pragma unroll
    for (int k = 0; k < 12; ++k) o[k] = v[k] - (a.dagger ? fu * zu[k] : fd * zd[k]);
#pragma unroll
    for (int k = 12; k < 24; ++k) o[k] = v[k] - (a.dagger ? fd * zd[k] : fu * zu[k]);
    store_spinor<P>(a.out, c, Ls, s, o);
}

static int launch_m5_args(const Geom &g, M5Args &a, long nsites, int prec, hipStream_t st) {
    a.nsites = nsites;
    a.Ls = g.Ls;
    a.spb = default_shape(g).spb;
    a.mf = g.mf;
    const int threads = a.spb * g.Ls;
    const unsigned nb = (unsigned)((nsites + a.spb - 1) / a.spb);
    const size_t areal = prec == DWF_F64 ? 8 : 4;
    const size_t shm = (size_t)threads * 25 * areal;
    switch (prec) {
        case DWF_F64: hipLaunchKernelGGL(k_m5<DWF_F64>, nb, threads, shm, st, a); break;
        case DWF_F32: hipLaunchKernelGGL(k_m5<DWF_F32>, nb, threads, shm, st, a); break;
        case DWF_F16: hipLaunchKernelGGL(k_m5<DWF_F16>, nb, threads, shm, st, a); break;
        default: hipLaunchKernelGGL(k_m5<DWF_BF16>, nb, threads, shm, st, a); break;
    }
    DWF_HIP(hipGetLastError());
    return DWF_OK;
}

int launch_m5(const Geom &g, void *out, const void *in, int dagger, int inverse, long nsites, int prec,
              hipStream_t st) {
    M5Args a;
    a.in = (const u32x4 *)in;
    a.in2 = nullptr;
    a.out = (u32x4 *)out;
    a.dagger = dagger;
    a.inverse = inverse;
    a.d = mooee_d(g);
    a.e = mooee_e(g);
    a.db = a.eb = 0.0;
    m5inv_setup(g, a.m5i, false);
    return launch_m5_args(g, a, nsites, prec, st);
}

int launch_m5_op(const Geom &g, void *out, const void *x, double d, double e, const void *z, double db, double eb,
                 int dagger, long nsites, int prec, hipStream_t st) {
    M5Args a;
    a.in = (const u32x4 *)x;
    a.in2 = (const u32x4 *)z;
    a.out = (u32x4 *)out;
    a.dagger = dagger;
    a.inverse = 0;
    a.d = d;
    a.e = e;
    a.db = db;
    a.eb = eb;
    m5inv_setup(g, a.m5i, false);
    return launch_m5_args(g, a, nsites, prec, st);
}

}  // namespace dwf
