// Checkerboarded 4D Wilson hopping term applied on every fifth-dimension
// slice (the domain-wall D_h), with fused fifth-dimension epilogues.
//
// One lane per (output checkerboard site c, s).  A workgroup holds spb whole
// sites (spb * Ls lanes), so the Ls lanes of a site are adjacent: every link is
// loaded once per site and broadcast to its Ls lanes, and every neighbour
// spinor component is read as Ls consecutive 16-byte vectors.  Per direction
// the lane spin-projects the neighbour (12 -> 6 complex), multiplies both
// colour vectors by the gathered link, and reconstructs into 24 accumulators
// (the projection identities are in dwf_spin.h).
//
// Epilogues fuse the fifth-dimension term into the same pass: M5op of a second
// field z at the output parity (z(s+-1) are read by the neighbouring lanes and
// come from L1), or M5op^-1 applied across the site's Ls lanes through LDS.
#include <algorithm>
#include <type_traits>

#include "dwf_dhop_core.h"

namespace dwf {

struct DhopArgs {
    const char *in;
    char *out;
    const char *z;
    const char *links;
    Lat lat;
    long half;
    int Ls, spb, parity, xcd, nt_store;
    double alpha, beta, d5, mf;
    double coef[kMaxLs];
};

// Apply M5op^-1 (DAG: M5op^-dag) to the Ls-vector v held by the site's lanes,
// through LDS.  Lower spins (2,3) couple s to s+n, upper spins (0,1) to s-n
// (swapped for the adjoint); coef[n] = d^-(n+1) / (1 + mf d^-Ls).
template <int DAG, typename A>
__device__ __forceinline__ void m5inv_lds(const DhopArgs &a, int Ls, A *lds, int j, int s, A *v) {
    A *mine = lds + (j * Ls + s) * 25;
#pragma unroll
    for (int k = 0; k < 24; ++k) mine[k] = v[k];
    __syncthreads();
    A o[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) o[k] = 0;
    const A *site = lds + j * Ls * 25;
    for (int n = 0; n < Ls; ++n) {
        const A cf = (A)a.coef[n];
        int sp = s + n;
        const A fp = sp < Ls ? cf : (A)(-a.mf) * cf;
        sp = sp < Ls ? sp : sp - Ls;
        int sm = s - n;
        const A fm = sm >= 0 ? cf : (A)(-a.mf) * cf;
        sm = sm >= 0 ? sm : sm + Ls;
        const A *vu = site + (DAG ? sp : sm) * 25;  // upper spins
        const A *vl = site + (DAG ? sm : sp) * 25;  // lower spins
        const A fu = DAG ? fp : fm, fl = DAG ? fm : fp;
#pragma unroll
        for (int k = 0; k < 12; ++k) o[k] += fu * vu[k];
#pragma unroll
        for (int k = 12; k < 24; ++k) o[k] += fl * vl[k];
    }
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = o[k];
}

// LS > 0: Ls fixed at compile time and 32-bit field offsets; LS == 0: generic.
template <int PI, int PO, int DAG, int EPI, int LS>
__global__ void __launch_bounds__(kMaxDhopThreads) k_dhop(const DhopArgs a) {
    using A = typename PT<PI>::A;
    using Off = typename std::conditional<(LS > 0), unsigned, long>::type;
    const int Ls = LS > 0 ? LS : a.Ls;
    const int t = threadIdx.x;
    const int j = t / Ls;
    const int s = t - j * Ls;
    const long blk = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (long)blockIdx.x;
    const long c = blk * a.spb + j;
    const bool active = c < a.half;

    A acc[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] = 0;

    if (active) dhop_site<PI, DAG, Off>(a.links, a.in, a.lat, Ls, a.parity, c, s, acc);

    const A alpha = (A)a.alpha;
    const Off zoff = spinor_off<PI, Off>(c, Ls, s);
    if constexpr (EPI == EPI_SCALE) {
        if (!active) return;
#pragma unroll
        for (int k = 0; k < 24; ++k) acc[k] *= alpha;
    } else if constexpr (EPI == EPI_AXPY) {
        if (!active) return;
        A zv[24];
        load_spinor_off<PI>(a.z, zoff, Ls * 16, zv);
        const A beta = (A)a.beta;
#pragma unroll
        for (int k = 0; k < 24; ++k) acc[k] = beta * zv[k] + alpha * acc[k];
    } else if constexpr (EPI == EPI_M5) {
        if (!active) return;
        // out = (5-M5) z(s) - P_- z~(s+1) - P_+ z~(s-1) + alpha D psi   (adjoint: P_+ <-> P_-)
        A z0[24], zu[24], zd[24];
        const Off row = zoff - (Off)(s * 16);
        load_spinor_off<PI>(a.z, zoff, Ls * 16, z0);
        load_spinor_off<PI>(a.z, row + (Off)((s + 1 < Ls ? s + 1 : 0) * 16), Ls * 16, zu);
        load_spinor_off<PI>(a.z, row + (Off)((s >= 1 ? s - 1 : Ls - 1) * 16), Ls * 16, zd);
        const A fu = s + 1 < Ls ? (A)1 : (A)(-a.mf);
        const A fd = s >= 1 ? (A)1 : (A)(-a.mf);
        const A d5 = (A)a.d5;
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = d5 * z0[k] - (DAG ? fu * zu[k] : fd * zd[k]) + alpha * acc[k];
#pragma unroll
        for (int k = 12; k < 24; ++k) acc[k] = d5 * z0[k] - (DAG ? fd * zd[k] : fu * zu[k]) + alpha * acc[k];
    } else {  // EPI_M5INV
        extern __shared__ unsigned char smem[];
        A *lds = reinterpret_cast<A *>(smem);
#pragma unroll
        for (int k = 0; k < 24; ++k) acc[k] *= alpha;
        if (a.z != nullptr && active) {
            A zv[24];
            load_spinor_off<PI>(a.z, zoff, Ls * 16, zv);
            const A beta = (A)a.beta;
#pragma unroll
            for (int k = 0; k < 24; ++k) acc[k] += beta * zv[k];
        }
        m5inv_lds<DAG>(a, Ls, lds, j, s, acc);
        if (!active) return;
    }
    store_spinor_off<PO>(a.out, spinor_off<PO, Off>(c, Ls, s), Ls * 16, acc, a.nt_store != 0);
}

DhopShape default_shape(const Geom &g) {
    DhopShape sh;
    int spb = 256 / g.Ls;
    if (spb < 1) spb = 1;
    for (int k = spb; k >= 1; --k)
        if ((k * g.Ls) % 64 == 0) {
            spb = k;
            break;
        }
    sh.spb = spb;
    sh.xcd = 1;
    return sh;
}

void m5inv_coefficients(const Geom &g, double *coef) {
    const double d = 5.0 - g.M5;
    double dn = 1.0;
    for (int n = 0; n < g.Ls; ++n) dn /= d;  // d^-Ls
    const double norm = 1.0 / (1.0 + g.mf * dn);
    double p = 1.0 / d;
    for (int n = 0; n < kMaxLs; ++n) {
        coef[n] = n < g.Ls ? p * norm : 0.0;
        p /= d;
    }
}

template <int PI, int PO, int DAG, int EPI>
static int launch_t(const DhopArgs &a, int ls_t, long nblocks, int threads, hipStream_t st) {
    using A = typename PT<PI>::A;
    const size_t shm = EPI == EPI_M5INV ? (size_t)a.spb * a.Ls * 25 * sizeof(A) : 0;
    const dim3 grid((unsigned)nblocks), block(threads);
    switch (ls_t) {
        case 8: hipLaunchKernelGGL((k_dhop<PI, PO, DAG, EPI, 8>), grid, block, shm, st, a); break;
        case 12: hipLaunchKernelGGL((k_dhop<PI, PO, DAG, EPI, 12>), grid, block, shm, st, a); break;
        case 16: hipLaunchKernelGGL((k_dhop<PI, PO, DAG, EPI, 16>), grid, block, shm, st, a); break;
        default: hipLaunchKernelGGL((k_dhop<PI, PO, DAG, EPI, 0>), grid, block, shm, st, a); break;
    }
    DWF_HIP(hipGetLastError());
    return DWF_OK;
}

template <int PI, int PO>
static int launch_pp(const DhopArgs &a, int ls_t, int dagger, int epi, long nb, int th, hipStream_t st) {
    if (dagger) {
        switch (epi) {
            case EPI_SCALE: return launch_t<PI, PO, 1, EPI_SCALE>(a, ls_t, nb, th, st);
            case EPI_AXPY: return launch_t<PI, PO, 1, EPI_AXPY>(a, ls_t, nb, th, st);
            case EPI_M5: return launch_t<PI, PO, 1, EPI_M5>(a, ls_t, nb, th, st);
            default: return launch_t<PI, PO, 1, EPI_M5INV>(a, ls_t, nb, th, st);
        }
    }
    switch (epi) {
        case EPI_SCALE: return launch_t<PI, PO, 0, EPI_SCALE>(a, ls_t, nb, th, st);
        case EPI_AXPY: return launch_t<PI, PO, 0, EPI_AXPY>(a, ls_t, nb, th, st);
        case EPI_M5: return launch_t<PI, PO, 0, EPI_M5>(a, ls_t, nb, th, st);
        default: return launch_t<PI, PO, 0, EPI_M5INV>(a, ls_t, nb, th, st);
    }
}

int launch_dhop(dwf_ctx ctx, const DhopCall &c, const DhopShape &shape_in, hipStream_t st) {
    const Geom &g = ctx->g;
    DhopShape shape = shape_in.spb > 0 ? shape_in : default_shape(g);
    DhopArgs a;
    a.in = (const char *)c.in;
    a.out = (char *)c.out;
    a.z = (const char *)c.z;
    a.links = (const char *)ctx->links[c.prec_in][c.out_parity];
    a.lat = make_lat(g.L);
    a.half = g.half;
    a.Ls = g.Ls;
    a.spb = shape.spb;
    a.parity = c.out_parity;
    a.xcd = shape.xcd;
    a.nt_store = shape.nt_store;
    a.alpha = c.alpha;
    a.beta = c.beta;
    a.d5 = 5.0 - g.M5;
    a.mf = g.mf;
    m5inv_coefficients(g, a.coef);
    const int threads = shape.spb * g.Ls;
    if (threads > kMaxDhopThreads || threads < 1) return fail(DWF_EINVAL, "hopping kernel: workgroup size out of range");
    const long nblocks = (g.half + shape.spb - 1) / shape.spb;
    // the specialised kernels use 32-bit byte offsets: every field they touch must be below 4 GiB
    const size_t big = std::max(cb_bytes(g, c.prec_in), cb_bytes(g, c.prec_out));
    const int ls_t = big < (size_t(1) << 32) ? g.Ls : 0;
    const int pi = c.prec_in, po = c.prec_out;
    if (pi == DWF_F64 && po == DWF_F64) return launch_pp<DWF_F64, DWF_F64>(a, ls_t, c.dagger, c.epi, nblocks, threads, st);
    if (pi == DWF_F32 && po == DWF_F32) return launch_pp<DWF_F32, DWF_F32>(a, ls_t, c.dagger, c.epi, nblocks, threads, st);
    if (pi == DWF_F16 && po == DWF_F16) return launch_pp<DWF_F16, DWF_F16>(a, ls_t, c.dagger, c.epi, nblocks, threads, st);
    if (pi == DWF_BF16 && po == DWF_BF16)
        return launch_pp<DWF_BF16, DWF_BF16>(a, ls_t, c.dagger, c.epi, nblocks, threads, st);
    if (pi == DWF_F16 && po == DWF_F32) return launch_pp<DWF_F16, DWF_F32>(a, ls_t, c.dagger, c.epi, nblocks, threads, st);
    if (pi == DWF_BF16 && po == DWF_F32)
        return launch_pp<DWF_BF16, DWF_F32>(a, ls_t, c.dagger, c.epi, nblocks, threads, st);
    return fail(DWF_EUNSUP, "hopping kernel: unsupported precision pair");
}

}  // namespace dwf
