// Domain-decomposed hopping term along t, the communication pattern the
// paper's library uses between GPUs (its face assembly and halo exchange),
// on one GPU: the lattice is one domain whose t-neighbour domain is itself.
//
//   interior  D_h with the t-links that cross the domain boundary set to zero
//             (the unchanged hopping kernel on a cut copy of the link table); it
//             needs no halo and runs on the caller's stream;
//   faces     meanwhile, on a second stream: the boundary slices of the input
//             (t = 0 for the forward hops of t = Lt-1, t = Lt-1 for the
//             backward hops of t = 0) are spin-projected to half spinors
//             (6 complex per site and s) and exchanged (a device copy stands in
//             for the peer transfer: the neighbour domain is this one);
//   exterior  after both, the boundary output sites add link x received half
//             spinor, reconstructed, with the links of the doubled (gathered)
//             table the receiving domain owns.
// Interior + exterior equals D_h up to the order of the last addition.
#include "dwf_dhop_core.h"

namespace dwf {

// Zero the 9 complex entries of direction dir for link-table rows [r0, r0 + n).
__global__ void __launch_bounds__(256) k_zero_links(unsigned *links, long r0, long n, int dir, int words) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= n * words) return;
    const long r = r0 + t / words;
    const int k = (int)(t % words);
    links[(r * 8 + dir) * words + k] = 0u;
}

// Half spinors P^TAU_3 psi of the slice rows [r0, r0 + S) of an input field, as
// face[i][s][12 reals] in the arithmetic type.
template <int PI, int TAU>
__global__ void __launch_bounds__(256) k_face_gather(typename PT<PI>::A *face, const char *in, long r0, long S,
                                                     int Ls) {
    using A = typename PT<PI>::A;
    constexpr int NG = 12 / PT<PI>::G;
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= S * Ls) return;
    const long i = t / Ls;
    const int s = (int)(t - i * Ls);
    u32x4 v[NG];
    const long off = spinor_off<PI, long>(r0 + i, Ls, s);
#pragma unroll
    for (int g = 0; g < NG; ++g) v[g] = *(const u32x4 *)(in + off + (long)g * Ls * 16);
    A h[12];
    project_vecs<PI, 3, TAU>(v, h);
    A *f = face + t * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) f[k] = h[k];
}

// out(r0 + i, s) += reconstruct(W(r0 + i, dir) face[i][s]) for the boundary rows of one face.
template <int PI, int DIR, int TAU>
__global__ void __launch_bounds__(256) k_face_apply(char *out, const char *links, const typename PT<PI>::A *face,
                                                    long r0, long S, int Ls) {
    using A = typename PT<PI>::A;
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= S * Ls) return;
    const long i = t / Ls;
    const int s = (int)(t - i * Ls);
    const long c = r0 + i;
    A w[18], h[12], acc[24];
    load_link<PI>(links, c, DIR, w);
    const A *f = face + t * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) h[k] = f[k];
    const long off = spinor_off<PI, long>(c, Ls, s);
    load_spinor_off<PI>(out, off, Ls * 16, acc);
    mul_reconstruct<3, TAU>(w, h, acc);
    store_spinor_off<PI>(out, off, Ls * 16, acc, false);
}

}  // namespace dwf

struct dwf_dd_s {
    dwf_ctx ctx = nullptr;
    int prec = 0;
    void *cut[2] = {};      // link tables per output parity, boundary t-links zeroed
    void *send[2] = {};     // [0]: forward face (slice t = 0), [1]: backward face (slice t = Lt-1)
    void *recv[2] = {};
    size_t face_bytes = 0;
    hipStream_t comm = nullptr;
    hipEvent_t ready = nullptr, halo = nullptr;
};

namespace dwf {

int dd_destroy(dwf_dd d) {
    if (!d) return DWF_OK;
    (void)hipDeviceSynchronize();
    for (void *p : d->cut) (void)hipFree(p);
    for (void *p : d->send) (void)hipFree(p);
    for (void *p : d->recv) (void)hipFree(p);
    if (d->comm) (void)hipStreamDestroy(d->comm);
    if (d->ready) (void)hipEventDestroy(d->ready);
    if (d->halo) (void)hipEventDestroy(d->halo);
    delete d;
    return DWF_OK;
}

int dd_create(dwf_ctx ctx, int prec, dwf_dd *out) {
    const Geom &g = ctx->g;
    dwf_dd d = new (std::nothrow) dwf_dd_s();
    if (!d) return fail(DWF_ENOMEM, "dwf_dd_create: out of host memory");
    d->ctx = ctx;
    d->prec = prec;
    const long S = g.half / g.L[3];  // checkerboard rows per t-slice
    const size_t areal = prec == DWF_F64 ? 8 : 4;
    d->face_bytes = (size_t)S * g.Ls * 12 * areal;
    auto bail = [&](int code, const char *msg) {
        dd_destroy(d);
        return fail(code, msg);
    };
    const size_t lb = link_bytes(g, prec);
    for (int p = 0; p < 2; ++p)
        if (hipMalloc(&d->cut[p], lb) != hipSuccess) return bail(DWF_ENOMEM, "dwf_dd_create: hipMalloc failed");
    for (int k = 0; k < 2; ++k)
        if (hipMalloc(&d->send[k], d->face_bytes) != hipSuccess || hipMalloc(&d->recv[k], d->face_bytes) != hipSuccess)
            return bail(DWF_ENOMEM, "dwf_dd_create: hipMalloc failed");
    if (hipStreamCreateWithFlags(&d->comm, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&d->ready, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&d->halo, hipEventDisableTiming) != hipSuccess)
        return bail(DWF_EHIP, "dwf_dd_create: stream or event creation failed");
    // cut tables: forward t-link (dir 3) of the last slice and backward t-link (dir 7) of the first
    const int words = 9 * 2 * real_bytes(prec) / 4;
    const unsigned nb = (unsigned)((S * words + 255) / 256);
    for (int p = 0; p < 2; ++p) {
        if (hipMemcpy(d->cut[p], ctx->links[prec][p], lb, hipMemcpyDeviceToDevice) != hipSuccess)
            return bail(DWF_EHIP, "dwf_dd_create: link copy failed");
        hipLaunchKernelGGL(k_zero_links, nb, 256, 0, 0, (unsigned *)d->cut[p], (long)(g.L[3] - 1) * S, S, 3, words);
        hipLaunchKernelGGL(k_zero_links, nb, 256, 0, 0, (unsigned *)d->cut[p], 0L, S, 7, words);
    }
    if (hipDeviceSynchronize() != hipSuccess) return bail(DWF_EHIP, "dwf_dd_create: cutting the link tables failed");
    *out = d;
    return DWF_OK;
}

template <int PI>
static int dd_faces(dwf_dd d, char *out, const char *in, int dagger, long S, int Ls, int L3, hipStream_t st,
                    int stage) {
    using A = typename PT<PI>::A;
    const unsigned nb = (unsigned)((S * Ls + 255) / 256);
    const long last = (long)(L3 - 1) * S;
    if (stage == 0) {  // gather the faces the t-neighbours need
        if (dagger) {
            hipLaunchKernelGGL((k_face_gather<PI, 1>), nb, 256, 0, st, (A *)d->send[0], in, 0L, S, Ls);
            hipLaunchKernelGGL((k_face_gather<PI, -1>), nb, 256, 0, st, (A *)d->send[1], in, last, S, Ls);
        } else {
            hipLaunchKernelGGL((k_face_gather<PI, -1>), nb, 256, 0, st, (A *)d->send[0], in, 0L, S, Ls);
            hipLaunchKernelGGL((k_face_gather<PI, 1>), nb, 256, 0, st, (A *)d->send[1], in, last, S, Ls);
        }
    } else {  // boundary sites add the received halo
        const char *lk = (const char *)d->ctx->links[PI][stage - 1];
        if (dagger) {
            hipLaunchKernelGGL((k_face_apply<PI, 3, 1>), nb, 256, 0, st, out, lk, (const A *)d->recv[0], last, S, Ls);
            hipLaunchKernelGGL((k_face_apply<PI, 7, -1>), nb, 256, 0, st, out, lk, (const A *)d->recv[1], 0L, S, Ls);
        } else {
            hipLaunchKernelGGL((k_face_apply<PI, 3, -1>), nb, 256, 0, st, out, lk, (const A *)d->recv[0], last, S, Ls);
            hipLaunchKernelGGL((k_face_apply<PI, 7, 1>), nb, 256, 0, st, out, lk, (const A *)d->recv[1], 0L, S, Ls);
        }
    }
    DWF_HIP(hipGetLastError());
    return DWF_OK;
}

static int dd_faces_any(dwf_dd d, char *out, const char *in, int dagger, int stage, hipStream_t st) {
    const Geom &g = d->ctx->g;
    const long S = g.half / g.L[3];
    switch (d->prec) {
        case DWF_F64: return dd_faces<DWF_F64>(d, out, in, dagger, S, g.Ls, g.L[3], st, stage);
        case DWF_F32: return dd_faces<DWF_F32>(d, out, in, dagger, S, g.Ls, g.L[3], st, stage);
        case DWF_F16: return dd_faces<DWF_F16>(d, out, in, dagger, S, g.Ls, g.L[3], st, stage);
        default: return dd_faces<DWF_BF16>(d, out, in, dagger, S, g.Ls, g.L[3], st, stage);
    }
}

int dd_dhop(dwf_dd d, void *out, const void *in, int out_parity, int dagger, hipStream_t st) {
    dwf_ctx ctx = d->ctx;
    int rc;
    // the comm stream starts once `in` is ready on the caller's stream
    DWF_HIP(hipEventRecord(d->ready, st));
    DWF_HIP(hipStreamWaitEvent(d->comm, d->ready, 0));
    if ((rc = dd_faces_any(d, nullptr, (const char *)in, dagger, 0, d->comm))) return rc;
    // exchange with the t-neighbour domains (here: this one); forward face to the domain below,
    // backward face to the domain above
    DWF_HIP(hipMemcpyAsync(d->recv[0], d->send[0], d->face_bytes, hipMemcpyDeviceToDevice, d->comm));
    DWF_HIP(hipMemcpyAsync(d->recv[1], d->send[1], d->face_bytes, hipMemcpyDeviceToDevice, d->comm));
    DWF_HIP(hipEventRecord(d->halo, d->comm));
    // interior on the caller's stream with the cut links, overlapping the faces
    DhopCall c{in, out, nullptr, out_parity, dagger, EPI_SCALE, 1.0, 0.0, d->prec, d->prec};
    c.links = d->cut[out_parity];
    if ((rc = launch_dhop(ctx, c, ctx->shape[d->prec][dagger], st))) return rc;
    DWF_HIP(hipStreamWaitEvent(st, d->halo, 0));
    return dd_faces_any(d, (char *)out, nullptr, dagger, 1 + out_parity, st);
}

int dd_face_only(dwf_dd d, const void *in, int dagger, hipStream_t st) {
    return dd_faces_any(d, nullptr, (const char *)in, dagger, 0, st);
}

}  // namespace dwf
