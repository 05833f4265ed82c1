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
    // row kernel: rows per workgroup, number of rows, traversal tile and its reciprocals
    int rows;
    unsigned nrows, ty, tz, tt, nty, ntt;
    unsigned lds_pad;  // host side: minimum LDS request of the row kernel (residency cap)
    float inv_per, inv_ty, inv_tz, inv_ntt, inv_ntyt;
    double alpha, beta, d5, mf;
    double *norm_out;
    const double *cg_alpha, *cg_live;
    double coef[kMaxLs];
};

// partials[blockIdx.x] = sum over the workgroup's active lanes of |v|^2, by a
// fixed LDS tree (bitwise reproducible).  Every lane of the workgroup calls it.
template <typename A>
__device__ __forceinline__ void block_norm_partial(double *partials, const A *v, bool active) {
    __shared__ double red[kMaxDhopThreads];
    double x = 0;
    if (active)
#pragma unroll
        for (int k = 0; k < 24; ++k) x += (double)v[k] * (double)v[k];
    const int t = threadIdx.x, n = blockDim.x;
    red[t] = x;
    __syncthreads();
    for (int stride = kMaxDhopThreads / 2; stride > 0; stride >>= 1) {
        if (t < stride && t + stride < n) red[t] += red[t + stride];
        __syncthreads();
    }
    if (t == 0) partials[blockIdx.x] = red[0];
}

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
        for (int k = 0; k < 12; ++k) o[k] = fma_(fu, vu[k], o[k]);
#pragma unroll
        for (int k = 12; k < 24; ++k) o[k] = fma_(fl, vl[k], o[k]);
    }
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = o[k];
}

// acc = M5op z + alpha acc at lane (c, s) (adjoint: P_+ <-> P_-), zoff = offset of z(c, s):
// M5op z(s) = (5-M5) z(s) - P_- z~(s+1) - P_+ z~(s-1), z~ carrying -mf across the wall.
template <int PI, int DAG, typename Off>
__device__ __forceinline__ void m5_combine(const DhopArgs &a, Off zoff, int Ls, int s, typename PT<PI>::A *acc) {
    using A = typename PT<PI>::A;
    A z0[24], zu[24], zd[24];
    const Off row = zoff - (Off)(s * 16);
    load_spinor_off<PI>(a.z, zoff, Ls * 16, z0);
    load_spinor_off<PI>(a.z, row + (Off)((s + 1 < Ls ? s + 1 : 0) * 16), Ls * 16, zu);
    load_spinor_off<PI>(a.z, row + (Off)((s >= 1 ? s - 1 : Ls - 1) * 16), Ls * 16, zd);
    const A fu = s + 1 < Ls ? (A)1 : (A)(-a.mf);
    const A fd = s >= 1 ? (A)1 : (A)(-a.mf);
    const A d5 = (A)a.d5, alpha = (A)a.alpha;
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = d5 * z0[k] - (DAG ? fu * zu[k] : fd * zd[k]) + alpha * acc[k];
#pragma unroll
    for (int k = 12; k < 24; ++k) acc[k] = d5 * z0[k] - (DAG ? fd * zd[k] : fu * zu[k]) + alpha * acc[k];
}

// CG residual update with the lane's y = A p in registers: r(c, s) -= cg_alpha * y in
// r's own precision PO (FP32 or FP64), then the workgroup's partial of the new |r|^2.
// Every lane of the workgroup calls it.
template <int PI, int PO, typename Off>
__device__ __forceinline__ void cg_update(const DhopArgs &a, long c, int Ls, int s, bool active,
                                          const typename PT<PI>::A *y) {
    using RA = typename PT<PO>::A;
    RA rv[24];
    const Off roff = spinor_off<PO, Off>(c, Ls, s);
    if (active) {
        const RA ca = (RA)*a.cg_alpha;
        load_spinor_off<PO>(a.out, roff, Ls * 16, rv);
#pragma unroll
        for (int k = 0; k < 24; ++k) rv[k] = rv[k] - ca * (RA)y[k];
    }
    block_norm_partial(a.norm_out, rv, active);
    if (active) store_spinor_off<PO>(a.out, roff, Ls * 16, rv, false);
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
    if constexpr (EPI == EPI_CG)
        if (*a.cg_live == 0) return;  // the solver has stopped: r stays as it is

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
        if (active) m5_combine<PI, DAG>(a, zoff, Ls, s, acc);
        if (a.norm_out != nullptr) block_norm_partial(a.norm_out, acc, active);
        if (!active) return;
    } else if constexpr (EPI == EPI_CG) {
        if (active) m5_combine<PI, DAG>(a, zoff, Ls, s, acc);
        cg_update<PI, PO, Off>(a, c, Ls, s, active, acc);
        return;
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


// Physical row (x1 + L1 (x2 + L2 x3)) of logical row q: rows are visited tile by
// tile, (ty, tz, tt) rows per tile with y fastest inside a tile, tiles with t
// fastest, so a run of consecutive logical rows is a compact (y, z, t) block.
__device__ __forceinline__ void rowmap(const DhopArgs &a, unsigned q, unsigned &x1, unsigned &x2, unsigned &x3) {
    const unsigned per = a.ty * a.tz * a.tt;
    const unsigned T = fdiv(q, per, a.inv_per);
    const unsigned w = q - T * per;
    const unsigned w1 = fdiv(w, a.ty, a.inv_ty);
    const unsigned ly = w - w1 * a.ty;
    const unsigned lt = fdiv(w1, a.tz, a.inv_tz);
    const unsigned lz = w1 - lt * a.tz;
    const unsigned T1 = fdiv(T, a.ntt, a.inv_ntt);  // T = Tt + ntt (Ty + nty Tz)
    const unsigned Tt = T - T1 * a.ntt;
    const unsigned Tz = fdiv(T1, a.nty, a.inv_ntyt);
    const unsigned Ty = T1 - Tz * a.nty;
    x1 = Ty * a.ty + ly;
    x2 = Tz * a.tz + lz;
    x3 = Tt * a.tt + lt;
}

// Row kernel: a workgroup owns `rows` whole x-rows (L0h sites x Ls slices each).
// The rows' 8 L0h links and the input rows at the same (y, z, t) (which hold
// both x-neighbours of every output site) are first copied to LDS with
// contiguous 16-byte loads; the x-hops and every link then come from LDS and
// only the y, z and t neighbours are read from global memory.
template <int PI, int PO, int DAG, int EPI, int LS>
__global__ void __launch_bounds__(kMaxDhopThreads) k_dhop_rows(const DhopArgs a) {
    using A = typename PT<PI>::A;
    using Off = typename std::conditional<(LS > 0), unsigned, long>::type;
    constexpr int G = PT<PI>::G, NG = 12 / G, R2 = 2 * G;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int Ls = LS > 0 ? LS : a.Ls;
    const int L0h = (int)a.lat.L0h;
    const int per_row = L0h * Ls;
    const int nthr = a.rows * per_row;
    const int t = threadIdx.x;
    const int r = t / per_row;
    const int wi = t - r * per_row;
    const int xh = wi / Ls;
    const int s = wi - xh * Ls;
    const long lb = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (long)blockIdx.x;
    const unsigned q0 = (unsigned)lb * (unsigned)a.rows;
    if constexpr (EPI == EPI_CG)
        if (*a.cg_live == 0) return;  // the solver has stopped: r stays as it is

    // lane coordinates and neighbour rows
    const bool active = q0 + r < a.nrows;
    unsigned x1 = 0, x2 = 0, x3 = 0;
    if (active) rowmap(a, q0 + r, x1, x2, x3);
    const long rest = x1 + (long)a.lat.L1 * (x2 + (long)a.lat.L2 * x3);
    const long c = rest * L0h + xh;
    const unsigned L0 = 2 * a.lat.L0h, L1 = a.lat.L1, L2 = a.lat.L2, L3 = a.lat.L3;
    const unsigned x0 = 2 * xh + ((a.parity + x1 + x2 + x3) & 1);
    const int lx0 = (int)((x0 + 1 == L0 ? 0 : x0 + 1) >> 1);
    const int lx4 = (int)((x0 == 0 ? L0 - 1 : x0 - 1) >> 1);
    const long s2 = L1, s3 = (long)L1 * L2;
    const long nb1 = (rest + (x1 + 1 == L1 ? -(long)(L1 - 1) : 1)) * L0h + xh;
    const long nb5 = (rest + (x1 == 0 ? (long)(L1 - 1) : -1)) * L0h + xh;
    const long nb2 = (rest + (x2 + 1 == L2 ? -(long)(L2 - 1) * s2 : s2)) * L0h + xh;
    const long nb6 = (rest + (x2 == 0 ? (long)(L2 - 1) * s2 : -s2)) * L0h + xh;
    const long nb3 = (rest + (x3 + 1 == L3 ? -(long)(L3 - 1) * s3 : s3)) * L0h + xh;
    const long nb7 = (rest + (x3 == 0 ? (long)(L3 - 1) * s3 : -s3)) * L0h + xh;

    // LDS: the rows' link blocks (as stored in global memory), then the input rows
    const int VX = L0h * NG * Ls;                   // 16-byte vectors per field row
    const int VL = L0h * 8 * 18 * PT<PI>::RB / 16;  // 16-byte vectors of links per row
    u32x4 *lds_l = reinterpret_cast<u32x4 *>(smem);
    u32x4 *lds_x = lds_l + a.rows * VL;
    // Each lane issues up to kStage loads of a row before its first LDS write, so
    // the copy of a row costs about one memory latency instead of one per vector.
    constexpr int kStage = 12;
    const int nrow_here = (int)min((unsigned)a.rows, a.nrows - q0);
    for (int rr = 0; rr < nrow_here; ++rr) {
        unsigned y1, y2, y3;  // uniform across the workgroup
        rowmap(a, q0 + rr, y1, y2, y3);
        const size_t prow = y1 + a.lat.L1 * (y2 + a.lat.L2 * y3);
        const u32x4 *gl = (const u32x4 *)a.links + prow * VL;
        const u32x4 *gx = (const u32x4 *)a.in + prow * VX;
        u32x4 *dl = lds_l + rr * VL;
        u32x4 *dx = lds_x + rr * VX;
        const int n = VL + VX;
        for (int v0 = t; v0 < n; v0 += kStage * nthr) {
            u32x4 buf[kStage];
#pragma unroll
            for (int u = 0; u < kStage; ++u) {
                const int v = v0 + u * nthr;
                if (v < n) buf[u] = *(v < VL ? gl + v : gx + (v - VL));
            }
#pragma unroll
            for (int u = 0; u < kStage; ++u) {
                const int v = v0 + u * nthr;
                if (v < n) *(v < VL ? dl + v : dx + (v - VL)) = buf[u];
            }
        }
    }
    __syncthreads();

    A acc[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] = 0;
    if (active) {
        const char *lk = reinterpret_cast<const char *>(lds_l) + (size_t)(r * L0h + xh) * 8 * 18 * PT<PI>::RB;
        const u32x4 *xr = lds_x + r * VX;
        constexpr int SG = DAG ? 1 : -1;
#define DWF_HOP_LDS(DIR, MU, TAU, LX)                                                        \
    {                                                                                        \
        A w[18], p[24], h[12];                                                               \
        load_link<PI>(lk, 0, DIR, w);                                                        \
        _Pragma("unroll") for (int g = 0; g < NG; ++g) unpack16<PI>(xr[((LX)*NG + g) * Ls + s], p + R2 * g); \
        project<MU, TAU>(p, h);                                                              \
        mul_reconstruct<MU, TAU>(w, h, acc);                                                 \
    }
#define DWF_HOP_GLB(DIR, MU, TAU, NB)                                                        \
    {                                                                                        \
        A w[18], p[24], h[12];                                                               \
        load_link<PI>(lk, 0, DIR, w);                                                        \
        load_spinor_off<PI>(a.in, spinor_off<PI, Off>(NB, Ls, s), Ls * 16, p);               \
        project<MU, TAU>(p, h);                                                              \
        mul_reconstruct<MU, TAU>(w, h, acc);                                                 \
    }
        DWF_HOP_LDS(0, 0, SG, lx0)
        DWF_HOP_GLB(1, 1, SG, nb1)
        DWF_HOP_GLB(2, 2, SG, nb2)
        DWF_HOP_GLB(3, 3, SG, nb3)
        DWF_HOP_LDS(4, 0, -SG, lx4)
        DWF_HOP_GLB(5, 1, -SG, nb5)
        DWF_HOP_GLB(6, 2, -SG, nb6)
        DWF_HOP_GLB(7, 3, -SG, nb7)
#undef DWF_HOP_LDS
#undef DWF_HOP_GLB
    }

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
        if (active) m5_combine<PI, DAG>(a, zoff, Ls, s, acc);
        if (a.norm_out != nullptr) block_norm_partial(a.norm_out, acc, active);
        if (!active) return;
    } else if constexpr (EPI == EPI_CG) {
        if (active) m5_combine<PI, DAG>(a, zoff, Ls, s, acc);
        cg_update<PI, PO, Off>(a, c, Ls, s, active, acc);
        return;
    } else {  // EPI_M5INV: the LDS staging area is reused once every lane is done with it
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
        __syncthreads();
        m5inv_lds<DAG>(a, Ls, lds, r * L0h + xh, s, acc);
        if (!active) return;
    }
    store_spinor_off<PO>(a.out, spinor_off<PO, Off>(c, Ls, s), Ls * 16, acc, a.nt_store != 0);
}

size_t row_lds_bytes(int rows, int L0h, int Ls, int prec) {
    return (size_t)rows * (size_t)L0h * (8 * 18 + (size_t)Ls * 24) * real_bytes(prec);
}

bool row_shape_ok(const Geom &g, const DhopShape &sh, int prec, size_t lds_limit) {
    if (sh.rows < 1) return false;
    const int threads = sh.rows * (g.L[0] / 2) * g.Ls;
    if (threads > kMaxDhopThreads) return false;
    if (g.L[1] % sh.ty || g.L[2] % sh.tz || g.L[3] % sh.tt) return false;
    size_t need = row_lds_bytes(sh.rows, g.L[0] / 2, g.Ls, prec);
    need = std::max(need, (size_t)threads * 25 * (prec == DWF_F64 ? 8 : 4));
    return need <= lds_limit;
}

DhopShape default_row_shape(const Geom &g, int prec, size_t lds_limit) {
    DhopShape sh = default_shape(g);
    const int per_row = (g.L[0] / 2) * g.Ls;
    if (per_row > kMaxDhopThreads) return sh;
    DhopShape r = sh;
    r.rows = std::max(1, 256 / per_row);
    r.ty = g.L[1] % 8 == 0 ? 8 : (g.L[1] % 4 == 0 ? 4 : 1);
    r.tz = g.L[2] % 4 == 0 ? 4 : 1;
    r.tt = g.L[3];
    return row_shape_ok(g, r, prec, lds_limit) ? r : sh;
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
    const dim3 grid((unsigned)nblocks), block(threads);
    if (a.rows > 0) {
        const size_t shm = std::max({row_lds_bytes(a.rows, (int)a.lat.L0h, a.Ls, PI),
                                     EPI == EPI_M5INV ? (size_t)threads * 25 * sizeof(A) : (size_t)0,
                                     (size_t)a.lds_pad});
        switch (ls_t) {
            case 8: hipLaunchKernelGGL((k_dhop_rows<PI, PO, DAG, EPI, 8>), grid, block, shm, st, a); break;
            case 12: hipLaunchKernelGGL((k_dhop_rows<PI, PO, DAG, EPI, 12>), grid, block, shm, st, a); break;
            case 16: hipLaunchKernelGGL((k_dhop_rows<PI, PO, DAG, EPI, 16>), grid, block, shm, st, a); break;
            default: hipLaunchKernelGGL((k_dhop_rows<PI, PO, DAG, EPI, 0>), grid, block, shm, st, a); break;
        }
        DWF_HIP(hipGetLastError());
        return DWF_OK;
    }
    const size_t shm = EPI == EPI_M5INV ? (size_t)a.spb * a.Ls * 25 * sizeof(A) : 0;
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
    if (epi == EPI_CG) {
        // the solver's residual update: adjoint kernel, r in FP32 or FP64
        if constexpr (PO == DWF_F32 || PO == DWF_F64)
            if (dagger) return launch_t<PI, PO, 1, EPI_CG>(a, ls_t, nb, th, st);
        return fail(DWF_EUNSUP, "hopping kernel: CG epilogue needs the adjoint and an FP32/FP64 residual");
    }
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
    DhopShape shape = (shape_in.spb > 0 || shape_in.rows > 0) ? shape_in : default_shape(g);
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
    a.norm_out = (c.epi == EPI_M5 || c.epi == EPI_CG) ? c.norm_out : nullptr;
    a.cg_alpha = c.cg_alpha;
    a.cg_live = c.cg_live;
    if (c.epi == EPI_CG && (!c.norm_out || !c.cg_alpha || !c.cg_live || !c.z))
        return fail(DWF_EINVAL, "hopping kernel: CG epilogue needs z, partials and the solver scalars");
    a.d5 = 5.0 - g.M5;
    a.mf = g.mf;
    m5inv_coefficients(g, a.coef);
    const bool rows_mode = shape.rows > 0 && row_shape_ok(g, shape, c.prec_in, ctx->lds_limit);
    a.rows = rows_mode ? shape.rows : 0;
    a.nrows = (unsigned)(g.vol / g.L[0]);
    a.ty = rows_mode ? shape.ty : 1;
    a.tz = rows_mode ? shape.tz : 1;
    a.tt = rows_mode ? shape.tt : 1;
    a.nty = g.L[1] / a.ty;
    a.ntt = g.L[3] / a.tt;
    a.inv_per = 1.0f / (float)(a.ty * a.tz * a.tt);
    a.inv_ty = 1.0f / (float)a.ty;
    a.inv_tz = 1.0f / (float)a.tz;
    a.inv_ntt = 1.0f / (float)a.ntt;
    a.inv_ntyt = 1.0f / (float)a.nty;
    // residency cap: request enough LDS that at most occ workgroups fit on one CU
    a.lds_pad = 0;
    if (rows_mode && shape.occ > 0) {
        const size_t pad = (ctx->lds_per_cu / (size_t)(shape.occ + 1) + 1024) & ~(size_t)255;
        if (pad <= ctx->lds_limit) a.lds_pad = (unsigned)pad;
    }
    int threads;
    long nblocks;
    if (rows_mode) {
        threads = shape.rows * (g.L[0] / 2) * g.Ls;
        nblocks = ((long)a.nrows + shape.rows - 1) / shape.rows;
    } else {
        if (shape.spb < 1) shape = default_shape(g);
        a.spb = shape.spb;
        threads = shape.spb * g.Ls;
        nblocks = (g.half + shape.spb - 1) / shape.spb;
    }
    if (threads > kMaxDhopThreads || threads < 1) return fail(DWF_EINVAL, "hopping kernel: workgroup size out of range");
    if (c.nparts_out) *c.nparts_out = nblocks;
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
