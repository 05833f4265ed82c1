// Body of the row-block hopping kernel, shared by the single-field launch and
// the batched multi-field launch.  A block of `rows` whole x-rows (L0h sites x
// Ls slices each, one lane per (site, slice)) is computed by the first
// rows * L0h * Ls lanes of a workgroup; further lanes only take part in the
// barriers.  The rows' links and the input rows at the same (y, z, t) (which
// hold both x-neighbours of every output site) are first copied to LDS with
// contiguous 16-byte loads; the x-hops and every link then come from LDS and
// only the y, z and t neighbours are read from global memory.
//
// Epilogues fuse the fifth-dimension term into the same pass: M5op of a second
// field z at the output parity (z(s+-1) are read by the neighbouring lanes and
// come from L1), M5op^-1 applied across the site's Ls lanes through LDS, or the
// CG residual update.
#pragma once

#include <type_traits>

#include "dwf_dhop_core.h"
#include "dwf_m5inv.h"

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
    double alpha, beta, d5, e5, mf;  // Mooee = d5 - e5 K
    double *norm_out;
    const double *cg_alpha, *cg_live;
    M5InvCoef m5i;  // EPI_M5INV: Mooee^-1 (or the Moebius Schur factor)
    unsigned dd_cut;  // EPI_INTERIOR, EPI_EXTERIOR: cut directions (bit mu)
    const double *stop;  // when non-null and *stop != 0 the launch does nothing (a solver that has stopped)
    const unsigned *row_list;  // EPI_EXTERIOR: physical rows y + L1 (z + L2 t), nrows of them
    const char *recv;          // EPI_EXTERIOR, 16-bit storage: received faces (half spinors, 12 reals of the
                               //   arithmetic type, one (face site, s) after the other)
    const char *ghost;         // EPI_EXTERIOR, FP32 / FP64: received faces as spinor sites of the field layout
                               //   (upper spin pair = the half spinor, lower pair = 0), site seg_off[seg] + face index
    long seg_off[9];           // EPI_EXTERIOR: first face site of segment 2 mu + side, prefix sums
};

// Face site index, within its segment, of the input site reached from output site (xh; x1, x2,
// x3) across cut mu: faces are ordered like the lattice with mu removed; the x faces hold one
// site per row pair, indexed by (y / 2, z, t).
__device__ __forceinline__ long dd_face_index(int mu, unsigned xh, unsigned x1, unsigned x2, unsigned x3,
                                              unsigned L0h, unsigned L1, unsigned L2) {
    if (mu == 0) return (long)(x1 >> 1) + (long)(L1 / 2) * ((long)x2 + (long)L2 * x3);
    if (mu == 1) return (long)xh + (long)L0h * ((long)x2 + (long)L2 * x3);
    if (mu == 2) return (long)xh + (long)L0h * ((long)x1 + (long)L1 * x3);
    return (long)xh + (long)L0h * ((long)x1 + (long)L1 * x2);
}

// Whether an output site has a hop across a cut of a domain decomposition: its coordinate
// along a cut direction mu is 0 (backward hop) or L_mu - 1 (forward hop).
__device__ __forceinline__ bool dd_boundary(unsigned cut, unsigned x0, unsigned x1, unsigned x2, unsigned x3,
                                            unsigned L0, unsigned L1, unsigned L2, unsigned L3) {
    return ((cut & 1u) && (x0 == 0 || x0 + 1 == L0)) || ((cut & 2u) && (x1 == 0 || x1 + 1 == L1)) ||
           ((cut & 4u) && (x2 == 0 || x2 + 1 == L2)) || ((cut & 8u) && (x3 == 0 || x3 + 1 == L3));
}

// Host side: fills the geometry, launch-shape and link fields of a for one output
// parity (alpha = 1, no fields attached); returns whether the row-block kernel
// applies to this shape (otherwise the site kernel does).
bool fill_dhop_args(dwf_ctx ctx, const DhopShape &shape, int prec_in, int out_parity, DhopArgs &a);

// partials[blockIdx.x] = sum over the workgroup's active lanes of |v|^2 in a
// fixed order (bitwise reproducible): a wavefront shuffle tree, then the wave
// sums in wave order.  A workgroup whose size is not a multiple of 64 has a
// partial last wave whose missing lanes a shuffle must not read; it sums
// through an LDS tree instead.  Every lane of the workgroup calls it.
template <typename A>
__device__ __forceinline__ void block_norm_partial(double *partials, const A *v, bool active) {
    __shared__ double red[kMaxDhopThreads];
    double x = 0;
    if (active)
#pragma unroll
        for (int k = 0; k < 24; ++k) x += (double)v[k] * (double)v[k];
    const int t = threadIdx.x, n = blockDim.x;
    if ((n & 63) == 0) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
        if ((t & 63) == 0) red[t >> 6] = x;
        __syncthreads();
        if (t == 0) {
            double sum = 0;
            for (int w = 0; w < (n >> 6); ++w) sum += red[w];
            partials[blockIdx.x] = sum;
        }
        return;
    }
    red[t] = x;
    __syncthreads();
    for (int stride = kMaxDhopThreads / 2; stride > 0; stride >>= 1) {
        if (t < stride && t + stride < n) red[t] += red[t + stride];
        __syncthreads();
    }
    if (t == 0) partials[blockIdx.x] = red[0];
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
    // e5 (1 for Shamir) folded into the shift factors
    const A fu = (A)(s + 1 < Ls ? a.e5 : -a.mf * a.e5);
    const A fd = (A)(s >= 1 ? a.e5 : -a.mf * a.e5);
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

// Coordinates of logical row q: the traversal order, or the listed row (EPI_EXTERIOR).
template <int EPI>
__device__ __forceinline__ void row_coords(const DhopArgs &a, unsigned q, unsigned &x1, unsigned &x2, unsigned &x3) {
    if constexpr (EPI == EPI_EXTERIOR) {
        const unsigned r = a.row_list[q];
        const unsigned r2 = fdiv(r, a.lat.L1, a.lat.inv1);
        x1 = r - r2 * a.lat.L1;
        x3 = fdiv(r2, a.lat.L2, a.lat.inv2);
        x2 = r2 - x3 * a.lat.L2;
    } else {
        rowmap(a, q, x1, x2, x3);
    }
}

// Row block starting at logical row q0 (see the file comment); every lane of
// the workgroup calls it.  smem holds row_lds_bytes(rows, L0h, Ls, PI) bytes
// (and threads * 25 reals for EPI_M5INV).
template <int PI, int PO, int DAG, int EPI, int LS>
__device__ __forceinline__ void row_block(const DhopArgs &a, unsigned q0, const char *__restrict__ in_f,
                                          char *__restrict__ out_f, const char *__restrict__ links_g,
                                          unsigned char *smem) {
    using A = typename PT<PI>::A;
    using Off = typename std::conditional<(LS > 0), unsigned, long>::type;
    constexpr int G = PT<PI>::G, NG = 12 / G, R2 = 2 * G;
    const int Ls = LS > 0 ? LS : a.Ls;
    const int L0h = (int)a.lat.L0h;
    const int per_row = L0h * Ls;
    const int nthr = a.rows * per_row;
    const int t = threadIdx.x;
    // FP32 / FP64 exterior: one row per workgroup (the host launches it so), so the row coordinates,
    // and with them every y, z and t cut test, are uniform across the workgroup
    constexpr bool kGhost = EPI == EPI_EXTERIOR && (PI == DWF_F32 || PI == DWF_F64);
    const int r = kGhost ? 0 : t / per_row;
    const int wi = t - r * per_row;
    const int xh = wi / Ls;
    const int s = wi - xh * Ls;

    // lane coordinates and neighbour rows
    const bool active = t < nthr && q0 + r < a.nrows;
    unsigned x1 = 0, x2 = 0, x3 = 0;
    if (kGhost) row_coords<EPI>(a, q0, x1, x2, x3);
    else if (active) row_coords<EPI>(a, q0 + r, x1, x2, x3);
    if constexpr (EPI == EPI_INTERIOR || EPI == EPI_INTERIOR_ROWS) {
        // a block whose rows all lie on a y, z or t cut has no interior site: the whole workgroup leaves
        bool any = false;
        const unsigned nr = min((unsigned)a.rows, a.nrows - q0);
        for (unsigned rr = 0; rr < nr && !any; ++rr) {
            unsigned y1, y2, y3;
            row_coords<EPI>(a, q0 + rr, y1, y2, y3);
            any = !dd_boundary(a.dd_cut & 14u, 1, y1, y2, y3, 4, a.lat.L1, a.lat.L2, a.lat.L3);
        }
        if (!any) return;
    }
    // row indices in the offset type (32-bit when every field is below 4 GiB; the
    // wrap-around steps are exact in modular arithmetic)
    const unsigned L0 = 2 * a.lat.L0h, L1 = a.lat.L1, L2 = a.lat.L2, L3 = a.lat.L3;
    const Off rest = (Off)x1 + (Off)L1 * ((Off)x2 + (Off)L2 * (Off)x3);
    const Off c = rest * (Off)L0h + (Off)xh;
    const unsigned x0 = 2 * xh + ((a.parity + x1 + x2 + x3) & 1);
    const int lx0 = (int)((x0 + 1 == L0 ? 0 : x0 + 1) >> 1);
    const int lx4 = (int)((x0 == 0 ? L0 - 1 : x0 - 1) >> 1);
    const Off s2 = L1, s3 = (Off)L1 * L2, o0 = 0;
    const Off nb1 = (rest + (x1 + 1 == L1 ? o0 - (Off)(L1 - 1) : (Off)1)) * (Off)L0h + (Off)xh;
    const Off nb5 = (rest + (x1 == 0 ? (Off)(L1 - 1) : o0 - 1)) * (Off)L0h + (Off)xh;
    const Off nb2 = (rest + (x2 + 1 == L2 ? o0 - (Off)(L2 - 1) * s2 : s2)) * (Off)L0h + (Off)xh;
    const Off nb6 = (rest + (x2 == 0 ? (Off)(L2 - 1) * s2 : o0 - s2)) * (Off)L0h + (Off)xh;
    const Off nb3 = (rest + (x3 + 1 == L3 ? o0 - (Off)(L3 - 1) * s3 : s3)) * (Off)L0h + (Off)xh;
    const Off nb7 = (rest + (x3 == 0 ? (Off)(L3 - 1) * s3 : o0 - s3)) * (Off)L0h + (Off)xh;

    // LDS: the rows' link blocks (as stored in global memory), then the input rows
    const int VX = L0h * NG * Ls;                   // 16-byte vectors per field row
    const int VL = L0h * 8 * 18 * PT<PI>::RB / 16;  // 16-byte vectors of links per row
    u32x4 *lds_l = reinterpret_cast<u32x4 *>(smem);
    u32x4 *lds_x = lds_l + a.rows * VL;
    // The links are read by this workgroup only: their loads are non-temporal, so they do not
    // push the input rows that neighbouring workgroups still read out of L2 (measured: 2-6%).
    // Each lane issues its first kL link and kX row loads (branch-free, clamped
    // index) before its first LDS write, so the copy of a row costs about one
    // memory latency instead of one per vector; kL, kX cover the common shapes and
    // larger rows finish in a plain loop.
    constexpr int kL = PI == DWF_F64 ? 5 : (PI == DWF_F32 ? 3 : 2);
    constexpr int kX = PI == DWF_F64 ? 12 : (PI == DWF_F32 ? 6 : 3);
    const int nrow_here = (int)min((unsigned)a.rows, a.nrows - q0);
    // FP16 storage: the six global neighbours of the lane (18 vectors) are requested together with
    // the staging loads, so a workgroup's reads of each neighbour row fall close together in time
    // and the rows neighbouring workgroups share are still in L2 (measured: ~10% less fetch and
    // 5-7% less time; at FP32 and BF16 the extra registers cost more occupancy than that gains).
    constexpr bool kPrefetch = PI == DWF_F16;
    u32x4 nbv[kPrefetch ? 6 : 1][NG];
    if constexpr (kPrefetch) {
        const bool stager = t < nthr;
        {  // first row of the block: its staging loads, the neighbour loads, then the LDS writes
            unsigned y1, y2, y3;  // uniform across the workgroup
            row_coords<EPI>(a, q0, y1, y2, y3);
            const size_t prow = y1 + a.lat.L1 * (y2 + a.lat.L2 * y3);
            const u32x4 *gl = (const u32x4 *)links_g + prow * VL;
            const u32x4 *gx = (const u32x4 *)in_f + prow * VX;
            u32x4 bl[kL], bx[kX];
#pragma unroll
            for (int u = 0; u < kL; ++u) bl[u] = __builtin_nontemporal_load(gl + min(t + u * nthr, VL - 1));
#pragma unroll
            for (int u = 0; u < kX; ++u) bx[u] = gx[min(t + u * nthr, VX - 1)];
            const Off nbs[6] = {nb1, nb2, nb3, nb5, nb6, nb7};  // in bounds for idle lanes too (row 0)
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const Off off = spinor_off<PI, Off>(nbs[k], Ls, s);
#pragma unroll
                for (int g = 0; g < NG; ++g) nbv[k][g] = *(const u32x4 *)(in_f + off + (Off)(g * Ls * 16));
            }
#pragma unroll
            for (int u = 0; u < kL; ++u)
                if (stager && t + u * nthr < VL) lds_l[t + u * nthr] = bl[u];
#pragma unroll
            for (int u = 0; u < kX; ++u)
                if (stager && t + u * nthr < VX) lds_x[t + u * nthr] = bx[u];
            if (stager) {
                for (int v = t + kL * nthr; v < VL; v += nthr) lds_l[v] = __builtin_nontemporal_load(gl + v);
                for (int v = t + kX * nthr; v < VX; v += nthr) lds_x[v] = gx[v];
            }
        }
        for (int rr = 1; rr < nrow_here && stager; ++rr) {
            unsigned y1, y2, y3;
            row_coords<EPI>(a, q0 + rr, y1, y2, y3);
            const size_t prow = y1 + a.lat.L1 * (y2 + a.lat.L2 * y3);
            const u32x4 *gl = (const u32x4 *)links_g + prow * VL;
            const u32x4 *gx = (const u32x4 *)in_f + prow * VX;
            for (int v = t; v < VL; v += nthr) lds_l[rr * VL + v] = __builtin_nontemporal_load(gl + v);
            for (int v = t; v < VX; v += nthr) lds_x[rr * VX + v] = gx[v];
        }
    } else {
        for (int rr = 0; rr < nrow_here && t < nthr; ++rr) {
            unsigned y1, y2, y3;  // uniform across the workgroup
            row_coords<EPI>(a, q0 + rr, y1, y2, y3);
            const size_t prow = y1 + a.lat.L1 * (y2 + a.lat.L2 * y3);
            const u32x4 *gl = (const u32x4 *)links_g + prow * VL;
            const u32x4 *gx = (const u32x4 *)in_f + prow * VX;
            u32x4 *dl = lds_l + rr * VL;
            u32x4 *dx = lds_x + rr * VX;
            u32x4 bl[kL], bx[kX];
#pragma unroll
            for (int u = 0; u < kL; ++u) bl[u] = __builtin_nontemporal_load(gl + min(t + u * nthr, VL - 1));
#pragma unroll
            for (int u = 0; u < kX; ++u) bx[u] = gx[min(t + u * nthr, VX - 1)];
#pragma unroll
            for (int u = 0; u < kL; ++u)
                if (t + u * nthr < VL) dl[t + u * nthr] = bl[u];
#pragma unroll
            for (int u = 0; u < kX; ++u)
                if (t + u * nthr < VX) dx[t + u * nthr] = bx[u];
            for (int v = t + kL * nthr; v < VL; v += nthr) dl[v] = __builtin_nontemporal_load(gl + v);
            for (int v = t + kX * nthr; v < VX; v += nthr) dx[v] = gx[v];
        }
    }
    if constexpr (kGhost) {
        // x cut: the row's one site whose x-hop crosses (the last site hopping forward when the row
        // starts at odd x, else the first hopping backward) reads its neighbour from an extra LDS
        // slot after the x-row, filled here from the received face
        if (a.dd_cut & 1u) {
            const unsigned o = ((unsigned)a.parity + x1 + x2 + x3) & 1u;
            const unsigned fi = (unsigned)a.seg_off[o ? 0 : 1] +
                                (unsigned)dd_face_index(0, o ? (unsigned)L0h - 1u : 0u, x1, x2, x3, (unsigned)L0h,
                                                        a.lat.L1, a.lat.L2);
            const u32x4 *gs = reinterpret_cast<const u32x4 *>(a.ghost) + (size_t)fi * (size_t)(NG * Ls);
            for (int v = t; v < NG * Ls; v += nthr) lds_x[VX + v] = gs[v];
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
        // EPI_EXTERIOR: a hop that crosses a cut (FWD: from coordinate L - 1, else from 0) takes the
        // received half spinor of face segment 2 mu + (FWD ? 0 : 1): FP32 / FP64 read it as a field
        // site (upper pair = half spinor, lower pair = 0, so the projection returns it unchanged) by
        // a select of address, 16-bit storage (face in the wider arithmetic type) by a branch; the
        // other instantiations drop this test at compile time.
#define DWF_CROSS(MU, FWD, XC, LM) (EPI == EPI_EXTERIOR && ((a.dd_cut >> (MU)) & 1u) && ((FWD) ? (XC) + 1 == (LM) : (XC) == 0))
#define DWF_FACE(MU, FWD)                                                                    \
    {                                                                                        \
        const unsigned fi_ = ((unsigned)a.seg_off[2 * (MU) + ((FWD) ? 0 : 1)] +              \
                              (unsigned)dd_face_index(MU, (unsigned)xh, x1, x2, x3, (unsigned)L0h, L1, L2)) * \
                                 (unsigned)Ls + (unsigned)s;                                 \
        const u32x4 *src_ = reinterpret_cast<const u32x4 *>(a.recv) + fi_ * (unsigned)(12 * sizeof(A) / 16); \
        u32x4 hv_[12 * sizeof(A) / 16];                                                      \
        _Pragma("unroll") for (int k = 0; k < (int)(12 * sizeof(A) / 16); ++k) hv_[k] = src_[k]; \
        __builtin_memcpy(h, hv_, sizeof(hv_));                                               \
    }
#define DWF_HOP_LDS(DIR, MU, TAU, LX, FWD)                                                   \
    {                                                                                        \
        A w[18], h[12];                                                                      \
        load_link<PI>(lk, 0, DIR, w);                                                        \
        if constexpr (kGhost) {                                                              \
            const int lx_ = DWF_CROSS(MU, FWD, x0, L0) ? L0h : (LX);                         \
            u32x4 v[NG];                                                                     \
            _Pragma("unroll") for (int g = 0; g < NG; ++g) v[g] = xr[(lx_ * NG + g) * Ls + s];\
            project_vecs<PI, MU, TAU>(v, h);                                                 \
        } else if (DWF_CROSS(MU, FWD, x0, L0)) DWF_FACE(MU, FWD)                             \
        else {                                                                               \
            u32x4 v[NG];                                                                     \
            _Pragma("unroll") for (int g = 0; g < NG; ++g) v[g] = xr[((LX)*NG + g) * Ls + s];\
            project_vecs<PI, MU, TAU>(v, h);                                                 \
        }                                                                                    \
        mul_reconstruct<MU, TAU>(w, h, acc);                                                 \
    }
#define DWF_HOP_GLB(DIR, MU, TAU, NB, FWD, XC, LM)                                           \
    {                                                                                        \
        A w[18], h[12];                                                                      \
        load_link<PI>(lk, 0, DIR, w);                                                        \
        if constexpr (kGhost) {                                                              \
            /* a crossing hop reads the received face site like a field site: no branch */   \
            const bool cr_ = DWF_CROSS(MU, FWD, XC, LM);                                     \
            const char *b_ = cr_ ? a.ghost : in_f;                                           \
            const unsigned fr_ = (MU) == 1 ? x2 + L2 * x3 : ((MU) == 2 ? x1 + L1 * x3 : x1 + L1 * x2); \
            const unsigned fb_ = (unsigned)a.seg_off[2 * (MU) + ((FWD) ? 0 : 1)] + (unsigned)L0h * fr_; \
            const Off st_ = cr_ ? (Off)(fb_ + (unsigned)xh) : (Off)(NB);                      \
            const Off off_ = spinor_off<PI, Off>(st_, Ls, s);                                \
            u32x4 v[NG];                                                                     \
            _Pragma("unroll") for (int g = 0; g < NG; ++g) v[g] =                            \
                *(const u32x4 *)(b_ + off_ + (Off)(g * Ls * 16));                            \
            project_vecs<PI, MU, TAU>(v, h);                                                 \
        } else if (DWF_CROSS(MU, FWD, XC, LM)) DWF_FACE(MU, FWD)                             \
        else {                                                                               \
            u32x4 v[NG];                                                                     \
            const Off off_ = spinor_off<PI, Off>(NB, Ls, s);                                 \
            _Pragma("unroll") for (int g = 0; g < NG; ++g) v[g] =                            \
                *(const u32x4 *)(in_f + off_ + (Off)(g * Ls * 16));                          \
            project_vecs<PI, MU, TAU>(v, h);                                                 \
        }                                                                                    \
        mul_reconstruct<MU, TAU>(w, h, acc);                                                 \
    }
#define DWF_HOP_REG(DIR, MU, TAU, K, FWD, XC, LM)                                            \
    {                                                                                        \
        A w[18], h[12];                                                                      \
        load_link<PI>(lk, 0, DIR, w);                                                        \
        if (DWF_CROSS(MU, FWD, XC, LM)) DWF_FACE(MU, FWD)                                    \
        else project_vecs<PI, MU, TAU>(nbv[K], h);                                           \
        mul_reconstruct<MU, TAU>(w, h, acc);                                                 \
    }
        if constexpr (kPrefetch) {
            DWF_HOP_LDS(0, 0, SG, lx0, true)
            DWF_HOP_REG(1, 1, SG, 0, true, x1, L1)
            DWF_HOP_REG(2, 2, SG, 1, true, x2, L2)
            DWF_HOP_REG(3, 3, SG, 2, true, x3, L3)
            DWF_HOP_LDS(4, 0, -SG, lx4, false)
            DWF_HOP_REG(5, 1, -SG, 3, false, x1, L1)
            DWF_HOP_REG(6, 2, -SG, 4, false, x2, L2)
            DWF_HOP_REG(7, 3, -SG, 5, false, x3, L3)
        } else {
            DWF_HOP_LDS(0, 0, SG, lx0, true)
            DWF_HOP_GLB(1, 1, SG, nb1, true, x1, L1)
            DWF_HOP_GLB(2, 2, SG, nb2, true, x2, L2)
            DWF_HOP_GLB(3, 3, SG, nb3, true, x3, L3)
            DWF_HOP_LDS(4, 0, -SG, lx4, false)
            DWF_HOP_GLB(5, 1, -SG, nb5, false, x1, L1)
            DWF_HOP_GLB(6, 2, -SG, nb6, false, x2, L2)
            DWF_HOP_GLB(7, 3, -SG, nb7, false, x3, L3)
        }
#undef DWF_CROSS
#undef DWF_FACE
#undef DWF_HOP_REG
#undef DWF_HOP_LDS
#undef DWF_HOP_GLB
    }

    const A alpha = (A)a.alpha;
    const Off zoff = spinor_off<PI, Off>(c, Ls, s);
    if constexpr (EPI == EPI_SCALE || EPI == EPI_INTERIOR || EPI == EPI_EXTERIOR || EPI == EPI_INTERIOR_ROWS) {
        if (!active) return;
        if (EPI == EPI_INTERIOR && dd_boundary(a.dd_cut, x0, x1, x2, x3, L0, L1, L2, L3)) return;
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
        m5inv_lds<DAG>(a.m5i, Ls, lds, r * L0h + xh, s, acc);
        if (!active) return;
    }
    store_spinor_off<PO>(out_f, spinor_off<PO, Off>(c, Ls, s), Ls * 16, acc, a.nt_store != 0);
}

}  // namespace dwf
