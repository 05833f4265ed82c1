// Domain-decomposed hopping term, the communication pattern the paper's library runs between
// GPUs (face assembly, halo exchange, interior compute overlapping the exchange), on one GPU
// whose neighbour domain across every cut direction is itself.
//
// A plan cuts any set of the four directions (the decomposition 2x2x2x1 of eight GPUs cuts x, y
// and z; each GPU then holds this lattice as its domain).  An output site is on the boundary
// when one of its hops crosses a cut (coordinate 0 or L_mu - 1 along a cut mu).
//
//   faces     one kernel spin-projects every face the neighbour domains need into one send
//             buffer: per cut mu, the input slice x_mu = 0 with the forward-hop projector and
//             the slice x_mu = L_mu - 1 with the backward-hop one, half spinors of 6 complex per
//             site and s in the arithmetic type.  The x faces live in the halved-x checkerboard
//             layout: the slice x = 0 of one parity holds site xh = 0 of every other row.
//   exchange  one device copy of the send buffer into the receive buffer (the stand-in for the
//             peer transfers: every face comes back to this domain).  FP32 / FP64 receive into
//             ghost sites of the field layout: the half spinor lands in a site's upper spin pair,
//             the lower pair stays zero, so the projection of the crossing hop returns it as it
//             was sent and the hopping kernel reads a crossing neighbour like any other site.
//   interior  the hopping kernel writing only the output sites with no hop across a cut, on the
//             caller's stream, overlapping the faces and the exchange on the plan's stream: a
//             workgroup whose rows all lie on a y, z or t cut leaves at once, and the other boundary
//             sites skip their store (EPI_INTERIOR), a test the launch drops when the boundary is
//             whole rows, one per workgroup (no x cut: EPI_INTERIOR_ROWS).
//   exterior  after the exchange, the boundary output sites are computed whole, hops across a
//             cut from the received half spinors and the rest from the local input, and written
//             (no read-modify-write of the output): the rows on a y, z or t cut by the row-block
//             kernel (EPI_EXTERIOR: its links and x-rows staged in LDS like every row launch),
//             the remaining x-cut sites by a kernel with one lane per (site, s).  With the x
//             direction cut, FP32 / FP64 compute every row in the exterior kernel instead (each
//             row holds one x-boundary site; its crossing neighbour comes from an LDS slot), and
//             there is no interior launch.
//
// Every hop runs through the same projection and link multiply as dwf_dhop, in the same order,
// so the decomposed apply equals dwf_dhop bit for bit.
#include <algorithm>
#include <vector>

#include "dwf_rows.h"

namespace dwf {

constexpr int kDdSegs = 8;  // face segments: 2 * mu + side (side 0: slice x_mu = 0, 1: x_mu = L_mu - 1)

struct FaceGeom {
    unsigned L0h, L1, L2, L3;
    int Ls, parity;  // output parity p; faces hold input sites (parity 1 - p)
    unsigned cut;
    long seg_off[kDdSegs + 1];  // first face site of each segment, prefix sums (empty for uncut mu)
};

// Input checkerboard row of face site i of segment seg (see the file comment).
__device__ __forceinline__ long face_src_row(const FaceGeom &f, int seg, long i) {
    const int mu = seg >> 1, side = seg & 1;
    const unsigned q = 1u - (unsigned)f.parity;
    unsigned xh, y, z, t;
    if (mu == 0) {
        const unsigned yh2 = f.L1 / 2;
        const unsigned yh = (unsigned)(i % yh2), zt = (unsigned)(i / yh2);
        z = zt % f.L2;
        t = zt / f.L2;
        const unsigned xs = side ? 2 * f.L0h - 1 : 0;
        y = 2 * yh + ((q + xs + z + t) & 1u);
        xh = xs >> 1;
    } else {
        xh = (unsigned)(i % f.L0h);
        const unsigned r = (unsigned)(i / f.L0h);
        if (mu == 1) {
            z = r % f.L2;
            t = r / f.L2;
            y = side ? f.L1 - 1 : 0;
        } else if (mu == 2) {
            y = r % f.L1;
            t = r / f.L1;
            z = side ? f.L2 - 1 : 0;
        } else {
            y = r % f.L1;
            z = r / f.L1;
            t = side ? f.L3 - 1 : 0;
        }
    }
    return ((long)y + (long)f.L1 * ((long)z + (long)f.L2 * t)) * f.L0h + xh;
}

// Face site index of the input site reached from output site (x0..x3, xh) across cut mu.
__device__ __forceinline__ long face_index(const FaceGeom &f, int mu, unsigned xh, unsigned x1, unsigned x2,
                                           unsigned x3) {
    return dd_face_index(mu, xh, x1, x2, x3, f.L0h, f.L1, f.L2);
}

// All faces in one launch: lane (face site, s) of the concatenated segments.
template <int PI, int DAG>
__global__ void __launch_bounds__(256) k_dd_faces(typename PT<PI>::A *send, const char *in, const FaceGeom f) {
    using A = typename PT<PI>::A;
    constexpr int NG = 12 / PT<PI>::G;
    constexpr int SG = DAG ? 1 : -1;  // projector sign of the forward hops
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    const long site = t / f.Ls;
    if (site >= f.seg_off[kDdSegs]) return;
    const int s = (int)(t - site * f.Ls);
    int seg = 0;
    while (site >= f.seg_off[seg + 1]) ++seg;
    const long row = face_src_row(f, seg, site - f.seg_off[seg]);
    u32x4 v[NG];
    const long off = spinor_off<PI, long>(row, f.Ls, s);
#pragma unroll
    for (int g = 0; g < NG; ++g) v[g] = *(const u32x4 *)(in + off + (long)g * f.Ls * 16);
    A h[12];
    switch (seg) {
        case 0: project_vecs<PI, 0, SG>(v, h); break;
        case 1: project_vecs<PI, 0, -SG>(v, h); break;
        case 2: project_vecs<PI, 1, SG>(v, h); break;
        case 3: project_vecs<PI, 1, -SG>(v, h); break;
        case 4: project_vecs<PI, 2, SG>(v, h); break;
        case 5: project_vecs<PI, 2, -SG>(v, h); break;
        case 6: project_vecs<PI, 3, SG>(v, h); break;
        default: project_vecs<PI, 3, -SG>(v, h); break;
    }
    if constexpr (PI == DWF_F32 || PI == DWF_F64) {
        // the upper spin pair of a field-layout site: the exchange drops it into the ghost sites
        constexpr int NH = NG / 2;
        u32x4 hv[NH];
        __builtin_memcpy(hv, h, sizeof(hv));
        u32x4 *dst = reinterpret_cast<u32x4 *>(send) + (site * NH) * f.Ls + s;
#pragma unroll
        for (int g = 0; g < NH; ++g) dst[(long)g * f.Ls] = hv[g];
    } else {
        A *dst = send + t * 12;
#pragma unroll
        for (int k = 0; k < 12; ++k) dst[k] = h[k];
    }
}

// Listed boundary sites: the whole stencil, hops across a cut from the received faces (FP32 /
// FP64: recv is the ghost buffer, the half spinor in the upper spin pair of each site).
template <int PI, int DAG>
__global__ void __launch_bounds__(256) k_dd_exterior(char *out, const char *in, const char *links,
                                                     const typename PT<PI>::A *recv, const unsigned *blist, long nb,
                                                     const FaceGeom f) {
    using A = typename PT<PI>::A;
    constexpr int NG = 12 / PT<PI>::G;
    constexpr int SG = DAG ? 1 : -1;
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    const long b = t / f.Ls;
    if (b >= nb) return;
    const int s = (int)(t - b * f.Ls);
    const long c = blist[b];
    const unsigned L0h = f.L0h, L0 = 2 * L0h, L1 = f.L1, L2 = f.L2, L3 = f.L3;
    const long rest = c / L0h;
    const unsigned xh = (unsigned)(c - rest * L0h);
    const unsigned x1 = (unsigned)(rest % L1), x2 = (unsigned)((rest / L1) % L2), x3 = (unsigned)(rest / ((long)L1 * L2));
    const unsigned x0 = 2 * xh + (((unsigned)f.parity + x1 + x2 + x3) & 1u);
    const unsigned xs[4] = {x0, x1, x2, x3}, Ln[4] = {L0, L1, L2, L3};
    const long st[4] = {1, (long)L1, (long)L1 * L2, (long)L1 * L2 * L3};  // row strides of y, z, t
    A acc[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] = 0;
#define DWF_DD_HOP(DIR, MU, TAU, FWD)                                                                   \
    {                                                                                                  \
        const bool cross = ((f.cut >> MU) & 1u) && (FWD ? xs[MU] + 1 == Ln[MU] : xs[MU] == 0);         \
        A w[18], h[12];                                                                                \
        load_link<PI>(links, c, DIR, w);                                                               \
        if (cross) {                                                                                   \
            const int seg = 2 * MU + (FWD ? 0 : 1);                                                    \
            const long fi = f.seg_off[seg] + face_index(f, MU, xh, x1, x2, x3);                        \
            if constexpr (PI == DWF_F32 || PI == DWF_F64) { /* upper pair of the ghost site */       \
                u32x4 hv[NG / 2];                                                                      \
                const u32x4 *src = reinterpret_cast<const u32x4 *>(recv) + (fi * NG) * f.Ls + s;       \
                _Pragma("unroll") for (int g = 0; g < NG / 2; ++g) hv[g] = src[(long)g * f.Ls];        \
                __builtin_memcpy(h, hv, sizeof(hv));                                                   \
            } else {                                                                                   \
                const A *src = recv + (fi * f.Ls + s) * 12;                                            \
                _Pragma("unroll") for (int k = 0; k < 12; ++k) h[k] = src[k];                         \
            }                                                                                          \
        } else {                                                                                       \
            long nbr;                                                                                  \
            if (MU == 0) {                                                                             \
                const unsigned xn = FWD ? (x0 + 1 == L0 ? 0 : x0 + 1) : (x0 == 0 ? L0 - 1 : x0 - 1);   \
                nbr = rest * L0h + (xn >> 1);                                                          \
            } else {                                                                                   \
                const long d = FWD ? (xs[MU] + 1 == Ln[MU] ? -(long)(Ln[MU] - 1) : 1)                  \
                                   : (xs[MU] == 0 ? (long)(Ln[MU] - 1) : -1);                          \
                nbr = (rest + d * st[MU - 1]) * L0h + xh;                                              \
            }                                                                                          \
            u32x4 v[NG];                                                                               \
            const long off = spinor_off<PI, long>(nbr, f.Ls, s);                                       \
            _Pragma("unroll") for (int g = 0; g < NG; ++g) v[g] = *(const u32x4 *)(in + off + (long)g * f.Ls * 16); \
            project_vecs<PI, MU, TAU>(v, h);                                                           \
        }                                                                                              \
        mul_reconstruct<MU, TAU>(w, h, acc);                                                           \
    }
    DWF_DD_HOP(0, 0, SG, true)
    DWF_DD_HOP(1, 1, SG, true)
    DWF_DD_HOP(2, 2, SG, true)
    DWF_DD_HOP(3, 3, SG, true)
    DWF_DD_HOP(4, 0, -SG, false)
    DWF_DD_HOP(5, 1, -SG, false)
    DWF_DD_HOP(6, 2, -SG, false)
    DWF_DD_HOP(7, 3, -SG, false)
#undef DWF_DD_HOP
    store_spinor_off<PI>(out, spinor_off<PI, long>(c, f.Ls, s), f.Ls * 16, acc, false);
}

}  // namespace dwf

struct dwf_dd_s {
    dwf_ctx ctx = nullptr;
    int prec = 0;
    unsigned cut = 0;
    long seg_off[dwf::kDdSegs + 1] = {};
    void *send = nullptr, *recv = nullptr;  // all faces, concatenated by segment (16-bit storage: recv)
    void *ghost = nullptr;  // FP32 / FP64: the received faces as field-layout sites (upper spin pair =
                            // half spinor, lower pair zero from creation on); the exchange fills the upper pairs
    size_t face_bytes = 0;
    unsigned *blist[2] = {};  // boundary output sites left to the site kernel, per output parity
    long nb[2] = {};
    unsigned *brows = nullptr;  // rows on a y, z or t cut (computed by the row kernel)
    long nbrows = 0;
    dwf::DhopShape row_shape;   // launch shape of the exterior rows
    bool all_rows = false;      // every row is an exterior row (FP32 / FP64 with the x direction cut)
    hipStream_t comm = nullptr;
    hipEvent_t ready = nullptr, halo = nullptr;
};

namespace dwf {

int dd_destroy(dwf_dd d) {
    if (!d) return DWF_OK;
    (void)hipDeviceSynchronize();
    (void)hipFree(d->send);
    (void)hipFree(d->recv);
    (void)hipFree(d->ghost);
    for (unsigned *p : d->blist) (void)hipFree(p);
    (void)hipFree(d->brows);
    if (d->comm) (void)hipStreamDestroy(d->comm);
    if (d->ready) (void)hipEventDestroy(d->ready);
    if (d->halo) (void)hipEventDestroy(d->halo);
    delete d;
    return DWF_OK;
}

int dd_create(dwf_ctx ctx, int prec, unsigned cut, dwf_dd *out) {
    const Geom &g = ctx->g;
    dwf_dd d = new (std::nothrow) dwf_dd_s();
    if (!d) return fail(DWF_ENOMEM, "dwf_dd_create: out of host memory");
    d->ctx = ctx;
    d->prec = prec;
    d->cut = cut;
    auto bail = [&](int code, const char *msg) {
        dd_destroy(d);
        return fail(code, msg);
    };
    // face segments: V / (2 L_mu) input sites per face of a cut direction
    d->seg_off[0] = 0;
    for (int seg = 0; seg < kDdSegs; ++seg) {
        const int mu = seg >> 1;
        d->seg_off[seg + 1] = d->seg_off[seg] + (((cut >> mu) & 1u) ? g.half / g.L[mu] : 0);
    }
    const size_t areal = prec == DWF_F64 ? 8 : 4;
    const bool wide = prec == DWF_F32 || prec == DWF_F64;
    d->face_bytes = (size_t)d->seg_off[kDdSegs] * g.Ls * 12 * areal;
    if (hipMalloc(&d->send, d->face_bytes) != hipSuccess)
        return bail(DWF_ENOMEM, "dwf_dd_create: hipMalloc of the face buffers failed");
    if (wide) {
        if (hipMalloc(&d->ghost, 2 * d->face_bytes) != hipSuccess)
            return bail(DWF_ENOMEM, "dwf_dd_create: hipMalloc of the ghost sites failed");
        if (hipMemset(d->ghost, 0, 2 * d->face_bytes) != hipSuccess)
            return bail(DWF_EHIP, "dwf_dd_create: clearing the ghost sites failed");
    } else if (hipMalloc(&d->recv, d->face_bytes) != hipSuccess) {
        return bail(DWF_ENOMEM, "dwf_dd_create: hipMalloc of the face buffers failed");
    }
    // the exterior: rows on a y, z or t cut go to the row kernel when it applies to this lattice,
    // the other boundary sites (x cut) to the site kernel
    const unsigned L0 = g.L[0], L1 = g.L[1], L2 = g.L[2], L3 = g.L[3], L0h = L0 / 2;
    d->row_shape = ctx->shape[prec][0].rows > 0 ? ctx->shape[prec][0] : default_row_shape(g, prec, ctx->lds_limit);
    if (wide) d->row_shape.rows = 1;  // the FP32 / FP64 exterior kernel takes one row per workgroup
    const bool by_rows = d->row_shape.rows > 0 && row_shape_ok(g, d->row_shape, prec, ctx->lds_limit) &&
                         (!wide || row_lds_bytes(1, (int)L0h, g.Ls, prec) + (size_t)g.Ls * 24 * areal <= ctx->lds_limit);
    auto row_cut = [&](unsigned x1, unsigned x2, unsigned x3) {
        return ((cut & 2u) && (x1 == 0 || x1 + 1 == L1)) || ((cut & 4u) && (x2 == 0 || x2 + 1 == L2)) ||
               ((cut & 8u) && (x3 == 0 || x3 + 1 == L3));
    };
    // With the x direction cut every x-row holds a boundary site (the row's first or last site,
    // by parity); FP32 / FP64 then compute every row after the exchange in the exterior kernel (the
    // crossing x-hop from an LDS slot) instead of splitting each row between the interior launch and
    // a site kernel, which re-reads eight scattered neighbours per boundary site.
    d->all_rows = wide && by_rows && (cut & 1u);
    if (by_rows) {
        // the rows in the traversal order of the plain apply (tiles of the launch shape), so the
        // workgroups in flight on one XCD share their neighbour rows as they do there
        const unsigned ty = (unsigned)d->row_shape.ty, tz = (unsigned)d->row_shape.tz, tt = (unsigned)d->row_shape.tt;
        const unsigned per = ty * tz * tt, nty = L1 / ty, ntt = L3 / tt;
        std::vector<unsigned> rows;
        for (unsigned q = 0; q < L1 * L2 * L3; ++q) {
            const unsigned T = q / per, w = q % per, ly = w % ty, lz = (w / ty) % tz, lt = w / ty / tz;
            const unsigned Tt = T % ntt, Ty = (T / ntt) % nty, Tz = T / ntt / nty;
            const unsigned x1 = Ty * ty + ly, x2 = Tz * tz + lz, x3 = Tt * tt + lt;
            if (d->all_rows || row_cut(x1, x2, x3)) rows.push_back(x1 + L1 * (x2 + L2 * x3));
        }
        d->nbrows = (long)rows.size();
        if (hipMalloc(&d->brows, std::max<size_t>(1, rows.size()) * sizeof(unsigned)) != hipSuccess)
            return bail(DWF_ENOMEM, "dwf_dd_create: hipMalloc of the boundary rows failed");
        if (!rows.empty() &&
            hipMemcpy(d->brows, rows.data(), rows.size() * sizeof(unsigned), hipMemcpyHostToDevice) != hipSuccess)
            return bail(DWF_EHIP, "dwf_dd_create: copy of the boundary rows failed");
    }
    for (int p = 0; p < 2; ++p) {
        std::vector<unsigned> list;
        for (long c = 0; c < g.half; ++c) {
            const long rest = c / L0h;
            const unsigned xh = (unsigned)(c - rest * L0h);
            const unsigned x1 = (unsigned)(rest % L1), x2 = (unsigned)((rest / L1) % L2),
                           x3 = (unsigned)(rest / ((long)L1 * L2));
            const unsigned x0 = 2 * xh + ((p + x1 + x2 + x3) & 1u);
            const bool on_row = row_cut(x1, x2, x3);
            if (d->all_rows || (by_rows && on_row)) continue;
            if (on_row || ((cut & 1u) && (x0 == 0 || x0 + 1 == L0))) list.push_back((unsigned)c);
        }
        d->nb[p] = (long)list.size();
        if (hipMalloc(&d->blist[p], std::max<size_t>(1, list.size()) * sizeof(unsigned)) != hipSuccess)
            return bail(DWF_ENOMEM, "dwf_dd_create: hipMalloc of the boundary list failed");
        if (!list.empty() && hipMemcpy(d->blist[p], list.data(), list.size() * sizeof(unsigned),
                                       hipMemcpyHostToDevice) != hipSuccess)
            return bail(DWF_EHIP, "dwf_dd_create: copy of the boundary list failed");
    }
    if (hipStreamCreateWithFlags(&d->comm, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&d->ready, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&d->halo, hipEventDisableTiming) != hipSuccess)
        return bail(DWF_EHIP, "dwf_dd_create: stream or event creation failed");
    // the clears and copies above ran on the null stream, which the plan's non-blocking stream and
    // a caller's non-blocking stream do not wait for
    if (hipDeviceSynchronize() != hipSuccess) return bail(DWF_EHIP, "dwf_dd_create: device synchronisation failed");
    *out = d;
    return DWF_OK;
}

static FaceGeom face_geom(const dwf_dd d, int out_parity) {
    const Geom &g = d->ctx->g;
    FaceGeom f;
    f.L0h = (unsigned)(g.L[0] / 2);
    f.L1 = (unsigned)g.L[1];
    f.L2 = (unsigned)g.L[2];
    f.L3 = (unsigned)g.L[3];
    f.Ls = g.Ls;
    f.parity = out_parity;
    f.cut = d->cut;
    for (int k = 0; k <= kDdSegs; ++k) f.seg_off[k] = d->seg_off[k];
    return f;
}

template <int PI>
static int dd_launch(dwf_dd d, char *out, const char *in, int out_parity, int dagger, hipStream_t st, int stage) {
    using A = typename PT<PI>::A;
    const FaceGeom f = face_geom(d, out_parity);
    if (stage == 2) {  // boundary rows by the row kernel
        if (d->nbrows == 0) return DWF_OK;
        DhopCall c{in, out, nullptr, out_parity, dagger, EPI_EXTERIOR, 1.0, 0.0, PI, PI};
        c.dd_cut = d->cut;
        c.row_list = d->brows;
        c.nrows_list = d->nbrows;
        c.recv = d->recv;
        c.ghost = d->ghost;
        c.seg_off = d->seg_off;
        return launch_dhop(d->ctx, c, d->row_shape, st);
    }
    if (stage == 0) {  // every face the neighbour domains need
        const long lanes = f.seg_off[kDdSegs] * f.Ls;
        const unsigned nb = (unsigned)((lanes + 255) / 256);
        if (dagger) hipLaunchKernelGGL((k_dd_faces<PI, 1>), nb, 256, 0, st, (A *)d->send, in, f);
        else hipLaunchKernelGGL((k_dd_faces<PI, 0>), nb, 256, 0, st, (A *)d->send, in, f);
    } else {  // boundary sites from the received faces
        const long n = d->nb[out_parity];
        if (n == 0) return DWF_OK;
        const unsigned nb = (unsigned)((n * f.Ls + 255) / 256);
        const char *lk = (const char *)d->ctx->links[PI][out_parity];
        const A *faces = (const A *)(d->ghost ? d->ghost : d->recv);
        if (dagger)
            hipLaunchKernelGGL((k_dd_exterior<PI, 1>), nb, 256, 0, st, out, in, lk, faces,
                               d->blist[out_parity], n, f);
        else
            hipLaunchKernelGGL((k_dd_exterior<PI, 0>), nb, 256, 0, st, out, in, lk, faces,
                               d->blist[out_parity], n, f);
    }
    DWF_HIP(hipGetLastError());
    return DWF_OK;
}

static int dd_launch_any(dwf_dd d, char *out, const char *in, int out_parity, int dagger, hipStream_t st, int stage) {
    switch (d->prec) {
        case DWF_F64: return dd_launch<DWF_F64>(d, out, in, out_parity, dagger, st, stage);
        case DWF_F32: return dd_launch<DWF_F32>(d, out, in, out_parity, dagger, st, stage);
        case DWF_F16: return dd_launch<DWF_F16>(d, out, in, out_parity, dagger, st, stage);
        default: return dd_launch<DWF_BF16>(d, out, in, out_parity, dagger, st, stage);
    }
}

// The stand-in for the peer transfers: every face comes back to this domain.  FP32 / FP64: into the
// upper spin pair of the ghost sites (one strided copy: rows of a site's half-spinor vectors).
static hipError_t dd_exchange(dwf_dd d, hipStream_t st) {
    if (!d->ghost) return hipMemcpyAsync(d->recv, d->send, d->face_bytes, hipMemcpyDeviceToDevice, st);
    const size_t nsites = (size_t)d->seg_off[kDdSegs];
    if (nsites == 0) return hipSuccess;
    const size_t half = d->face_bytes / nsites;  // one site's half spinors, all s
    return hipMemcpy2DAsync(d->ghost, 2 * half, d->send, half, half, nsites, hipMemcpyDeviceToDevice, st);
}

int dd_dhop(dwf_dd d, void *out, const void *in, int out_parity, int dagger, hipStream_t st) {
    dwf_ctx ctx = d->ctx;
    if (!ctx->gauge_set) return fail(DWF_EUNSUP, "dwf_dd_dhop: gauge not set");
    int rc;
    // the plan's stream starts once `in` is ready on the caller's stream: faces, exchange, exterior
    DWF_HIP(hipEventRecord(d->ready, st));
    DWF_HIP(hipStreamWaitEvent(d->comm, d->ready, 0));
    if ((rc = dd_launch_any(d, nullptr, (const char *)in, out_parity, dagger, d->comm, 0))) return rc;
    DWF_HIP(dd_exchange(d, d->comm));
    if ((rc = dd_launch_any(d, (char *)out, (const char *)in, out_parity, dagger, d->comm, 2))) return rc;
    if ((rc = dd_launch_any(d, (char *)out, (const char *)in, out_parity, dagger, d->comm, 1))) return rc;
    DWF_HIP(hipEventRecord(d->halo, d->comm));
    // interior on the caller's stream, overlapping the faces and the exchange
    if (!d->all_rows) {
        // without an x cut the interior is whole rows: with one row per workgroup the launch needs no
        // per-site test before its stores (that branch costs the kernel ~9% at 32^4 x 16)
        const DhopShape &sh = ctx->shape[d->prec][dagger];
        const bool whole = !(d->cut & 1u) && sh.rows == 1 && row_shape_ok(ctx->g, sh, d->prec, ctx->lds_limit);
        DhopCall c{in, out, nullptr, out_parity, dagger, whole ? EPI_INTERIOR_ROWS : EPI_INTERIOR, 1.0, 0.0, d->prec,
                   d->prec};
        c.dd_cut = d->cut;
        if ((rc = launch_dhop(ctx, c, sh, st))) return rc;
    }
    DWF_HIP(hipStreamWaitEvent(st, d->halo, 0));
    return DWF_OK;
}

int dd_face_only(dwf_dd d, const void *in, int out_parity, int dagger, hipStream_t st) {
    return dd_launch_any(d, nullptr, (const char *)in, out_parity, dagger, st, 0);
}

}  // namespace dwf
