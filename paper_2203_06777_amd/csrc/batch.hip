// Batched hopping term: many right-hand sides of several lattices (of
// different volumes and Ls) in one launch, recorded as a HIP graph.
//
// Work items are (lattice, rhs, row block) with the row blocks innermost, and
// every item runs the row-block body of the single-field kernel (links and
// x-neighbour rows in LDS, each lattice with its own tuned shape).  Each XCD
// owns one contiguous eighth of the item list and its workgroups step through
// it together, so the items in flight on one XCD are neighbouring row blocks of
// one field and share that XCD's L2.  The grid has one workgroup per item: a
// resident grid that walks the list (fewer workgroups, several items each) and
// an order with the RHS innermost (a row block's links shared by all RHS) were
// both measured slower, since they spread the rows in flight over more fields
// than L2 holds.  Lattices whose rows do not fit a workgroup fall back to a
// site-per-lane variant with a resident grid.  The item loops end after a fixed
// count, with no queue or atomics.
#include <algorithm>
#include <vector>

#include "dwf_rows.h"

struct dwf_batch_s;

namespace dwf {

constexpr int kMaxBatchLat = 16;

struct BatchLat {
    const void *links;
    long half;
    long item_begin;  // first item of this lattice
    long tiles;
    Lat lat;
    int Ls, spb, nrhs, rhs_off;
};

struct BatchDesc {
    int nlat;
    int parity;
    long total_items;
    long per_block;
    const u32x4 *const *ins;
    u32x4 *const *outs;
    BatchLat lat[kMaxBatchLat];
};

// Row-block items.
// Pointers the kernel dereferences are typed as global memory: read from this
// descriptor as plain pointers they would be accessed with flat instructions.
typedef const __attribute__((address_space(1))) char *gconst_ptr;
typedef __attribute__((address_space(1))) char *gptr;

struct BatchRowLat {
    DhopArgs a;  // geometry and shape of the lattice (fields and links come per item)
    gconst_ptr links;
    long item_begin;
    long nblk;  // row blocks of the lattice
    int nrhs, rhs_off;
};

struct BatchRowDesc {
    int nlat;
    long total_items;
    const gconst_ptr *ins;
    const gptr *outs;
    BatchRowLat lat[kMaxBatchLat];
};

constexpr unsigned kXcds = 8;  // workgroup b runs on XCD b % 8

template <int P, int DAG, int LS>
__global__ void __launch_bounds__(kMaxDhopThreads) k_dhop_batch_rows(const BatchRowDesc *__restrict__ d) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const unsigned x = blockIdx.x % kXcds, w = blockIdx.x / kXcds, nw = gridDim.x / kXcds;
    const long chunk = (d->total_items + kXcds - 1) / kXcds;
    const long begin = (long)x * chunk;
    const long end = begin + chunk < d->total_items ? begin + chunk : d->total_items;
    for (long item = begin + w; item < end; item += nw) {
        int l = 0;
        while (l + 1 < d->nlat && item >= d->lat[l + 1].item_begin) ++l;
        const BatchRowLat &L = d->lat[l];
        const long local = item - L.item_begin;
        const int rhs = (int)(local / L.nblk);
        const long blk = local - (long)rhs * L.nblk;
        row_block<P, P, DAG, EPI_SCALE, LS>(L.a, (unsigned)blk * (unsigned)L.a.rows, (const char *)d->ins[L.rhs_off + rhs],
                                            (char *)d->outs[L.rhs_off + rhs], (const char *)L.links, smem);
        __syncthreads();  // the next item stages its rows into the same LDS
    }
}

// Site items (fallback).
template <int P, int DAG>
__global__ void __launch_bounds__(kMaxDhopThreads) k_dhop_batch(const BatchDesc *__restrict__ d) {
    using A = typename PT<P>::A;
    const long lb = xcd_remap(blockIdx.x, gridDim.x);
    const long begin = lb * d->per_block;
    long end = begin + d->per_block;
    if (end > d->total_items) end = d->total_items;
    for (long item = begin; item < end; ++item) {
        int l = 0;
        while (l + 1 < d->nlat && item >= d->lat[l + 1].item_begin) ++l;
        const BatchLat &L = d->lat[l];
        const long local = item - L.item_begin;
        const long tile = local / L.nrhs;
        const int rhs = (int)(local - tile * L.nrhs);
        const int Ls = L.Ls;
        const int j = threadIdx.x / Ls;
        const int s = threadIdx.x - j * Ls;
        const long c = tile * L.spb + j;
        if (j >= L.spb || c >= L.half) continue;
        A acc[24];
#pragma unroll
        for (int k = 0; k < 24; ++k) acc[k] = 0;
        dhop_site<P, DAG, long>((const char *)L.links, (const char *)d->ins[L.rhs_off + rhs], L.lat, Ls, d->parity,
                                c, s, acc);
        store_spinor_off<P>((char *)d->outs[L.rhs_off + rhs], spinor_off<P, long>(c, Ls, s), Ls * 16, acc, true);
    }
}

}  // namespace dwf

using namespace dwf;

struct dwf_batch_s {
    std::vector<dwf_ctx> ctxs;
    std::vector<int> nrhs;
    std::vector<DhopShape> shapes;
    int prec = 0, dagger = 0, nlat = 0, total_rhs = 0, threads = 0, ls_t = 0;
    bool rows = false;
    size_t lds = 0;
    long nblocks = 0;
    BatchDesc host{};
    BatchDesc *dev = nullptr;
    BatchRowDesc rhost{};
    BatchRowDesc *rdev = nullptr;
    void **ptrs = nullptr;  // device: ins[total_rhs], outs[total_rhs]
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace dwf {

static const void *batch_kernel(int prec, int dagger) {
    switch (prec) {
        case DWF_F64: return dagger ? (const void *)k_dhop_batch<DWF_F64, 1> : (const void *)k_dhop_batch<DWF_F64, 0>;
        case DWF_F32: return dagger ? (const void *)k_dhop_batch<DWF_F32, 1> : (const void *)k_dhop_batch<DWF_F32, 0>;
        case DWF_F16: return dagger ? (const void *)k_dhop_batch<DWF_F16, 1> : (const void *)k_dhop_batch<DWF_F16, 0>;
        default: return dagger ? (const void *)k_dhop_batch<DWF_BF16, 1> : (const void *)k_dhop_batch<DWF_BF16, 0>;
    }
}

template <int P>
static const void *batch_rows_kernel_p(int dagger, int ls_t) {
    switch (ls_t) {
        case 8: return dagger ? (const void *)k_dhop_batch_rows<P, 1, 8> : (const void *)k_dhop_batch_rows<P, 0, 8>;
        case 12: return dagger ? (const void *)k_dhop_batch_rows<P, 1, 12> : (const void *)k_dhop_batch_rows<P, 0, 12>;
        case 16: return dagger ? (const void *)k_dhop_batch_rows<P, 1, 16> : (const void *)k_dhop_batch_rows<P, 0, 16>;
        default: return dagger ? (const void *)k_dhop_batch_rows<P, 1, 0> : (const void *)k_dhop_batch_rows<P, 0, 0>;
    }
}

static const void *batch_rows_kernel(int prec, int dagger, int ls_t) {
    switch (prec) {
        case DWF_F64: return batch_rows_kernel_p<DWF_F64>(dagger, ls_t);
        case DWF_F32: return batch_rows_kernel_p<DWF_F32>(dagger, ls_t);
        case DWF_F16: return batch_rows_kernel_p<DWF_F16>(dagger, ls_t);
        default: return batch_rows_kernel_p<DWF_BF16>(dagger, ls_t);
    }
}

// Row-block plan: every lattice must have a row shape that fits one workgroup.
static bool plan_rows(dwf_batch p, const dwf_ctx *ctxs, int nlat, const int *nrhs) {
    int threads = 0, ls_common = ctxs[0]->g.Ls;
    size_t lds = 0, big = 0;
    long items = 0;
    int rhs_off = 0;
    for (int l = 0; l < nlat; ++l) {
        dwf_ctx c = ctxs[l];
        const Geom &g = c->g;
        DhopShape sh = c->shape[p->prec][p->dagger];
        if (sh.rows <= 0 || !row_shape_ok(g, sh, p->prec, c->lds_limit)) sh = default_row_shape(g, p->prec, c->lds_limit);
        if (sh.rows <= 0 || !row_shape_ok(g, sh, p->prec, c->lds_limit)) return false;
        BatchRowLat &L = p->rhost.lat[l];
        if (!fill_dhop_args(c, sh, p->prec, 0, L.a)) return false;
        threads = std::max(threads, sh.rows * (g.L[0] / 2) * g.Ls);
        lds = std::max(lds, row_lds_bytes(sh.rows, g.L[0] / 2, g.Ls, p->prec));
        big = std::max(big, cb_bytes(g, p->prec));
        if (g.Ls != ls_common) ls_common = 0;
        L.item_begin = items;
        L.nrhs = nrhs[l];
        L.rhs_off = rhs_off;
        L.nblk = (long)((L.a.nrows + sh.rows - 1) / sh.rows);
        items += L.nblk * nrhs[l];
        rhs_off += nrhs[l];
        p->shapes.push_back(sh);
    }
    if (lds > ctxs[0]->lds_limit) return false;
    p->rows = true;
    p->threads = threads;
    p->lds = lds;
    p->ls_t = (big < (size_t(1) << 32) && (ls_common == 8 || ls_common == 12 || ls_common == 16)) ? ls_common : 0;
    p->rhost.nlat = nlat;
    p->rhost.total_items = items;
    p->total_rhs = rhs_off;
    return true;
}

int batch_plan(const dwf_ctx *ctxs, int nlat, const int *nrhs, int prec, int dagger, dwf_batch *out) {
    dwf_batch p = new dwf_batch_s();
    p->prec = prec;
    p->dagger = dagger;
    p->nlat = nlat;
    for (int l = 0; l < nlat; ++l) {
        p->ctxs.push_back(ctxs[l]);
        p->nrhs.push_back(nrhs[l]);
    }
    if (plan_rows(p, ctxs, nlat, nrhs)) {
        // one workgroup per item, rounded up to a multiple of the XCD count
        p->nblocks = (p->rhost.total_items + kXcds - 1) / kXcds * kXcds;
        if (hipMalloc(&p->rdev, sizeof(BatchRowDesc)) != hipSuccess ||
            hipMalloc(&p->ptrs, sizeof(void *) * 2 * (size_t)p->total_rhs) != hipSuccess) {
            (void)hipFree(p->rdev);
            delete p;
            return fail(DWF_ENOMEM, "dwf_batch_plan: hipMalloc failed");
        }
        p->rhost.ins = (const gconst_ptr *)p->ptrs;
        p->rhost.outs = (const gptr *)(p->ptrs + p->total_rhs);
        *out = p;
        return DWF_OK;
    }
    p->ctxs.clear();
    p->nrhs.clear();
    p->shapes.clear();
    p->rows = false;
    int threads = 0;
    for (int l = 0; l < nlat; ++l) {
        const Geom &g = ctxs[l]->g;
        const DhopShape &sh = ctxs[l]->shape[prec][dagger];
        int spb = sh.spb > 0 ? sh.spb : default_shape(g).spb;
        while (spb > 1 && spb * g.Ls > kMaxDhopThreads) --spb;
        if (spb * g.Ls > threads) threads = spb * g.Ls;
    }
    long items = 0;
    int rhs_off = 0;
    for (int l = 0; l < nlat; ++l) {
        const Geom &g = ctxs[l]->g;
        BatchLat &L = p->host.lat[l];
        L.links = ctxs[l]->links[prec][0];
        L.half = g.half;
        L.lat = make_lat(g.L);
        L.Ls = g.Ls;
        L.spb = threads / g.Ls;
        L.tiles = (g.half + L.spb - 1) / L.spb;
        L.nrhs = nrhs[l];
        L.rhs_off = rhs_off;
        L.item_begin = items;
        items += L.tiles * nrhs[l];
        rhs_off += nrhs[l];
        p->ctxs.push_back(ctxs[l]);
        p->nrhs.push_back(nrhs[l]);
    }
    p->total_rhs = rhs_off;
    p->threads = threads;
    p->host.nlat = nlat;
    p->host.total_items = items;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel(prec, dagger), threads, 0);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    int dev = 0, cus = 0;
    DWF_HIP(hipGetDevice(&dev));
    DWF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    long nb = (long)cus * per_cu;
    if (nb > items) nb = items;
    if (nb < 1) nb = 1;
    p->nblocks = nb;
    p->host.per_block = (items + nb - 1) / nb;
    if (hipMalloc(&p->dev, sizeof(BatchDesc)) != hipSuccess ||
        hipMalloc(&p->ptrs, sizeof(void *) * 2 * (size_t)p->total_rhs) != hipSuccess) {
        (void)hipFree(p->dev);
        delete p;
        return fail(DWF_ENOMEM, "dwf_batch_plan: hipMalloc failed");
    }
    p->host.ins = (const u32x4 *const *)p->ptrs;
    p->host.outs = (u32x4 *const *)(p->ptrs + p->total_rhs);
    *out = p;
    return DWF_OK;
}

int batch_capture(dwf_batch p, void *const *outs, const void *const *ins, int out_parity, hipStream_t st) {
    std::vector<void *> host(2 * (size_t)p->total_rhs);
    for (int r = 0; r < p->total_rhs; ++r) {
        host[r] = const_cast<void *>(ins[r]);
        host[p->total_rhs + r] = outs[r];
    }
    DWF_HIP(hipMemcpyAsync(p->ptrs, host.data(), host.size() * sizeof(void *), hipMemcpyHostToDevice, st));
    if (p->rows) {
        for (int l = 0; l < p->nlat; ++l) {
            BatchRowLat &L = p->rhost.lat[l];
            fill_dhop_args(p->ctxs[l], p->shapes[l], p->prec, out_parity, L.a);
            L.links = (gconst_ptr)L.a.links;
        }
        DWF_HIP(hipMemcpyAsync(p->rdev, &p->rhost, sizeof(BatchRowDesc), hipMemcpyHostToDevice, st));
    } else {
        for (int l = 0; l < p->nlat; ++l) p->host.lat[l].links = p->ctxs[l]->links[p->prec][out_parity];
        p->host.parity = out_parity;
        DWF_HIP(hipMemcpyAsync(p->dev, &p->host, sizeof(BatchDesc), hipMemcpyHostToDevice, st));
    }
    DWF_HIP(hipStreamSynchronize(st));
    if (p->exec) {
        (void)hipGraphExecDestroy(p->exec);
        p->exec = nullptr;
    }
    if (p->graph) {
        (void)hipGraphDestroy(p->graph);
        p->graph = nullptr;
    }
    DWF_HIP(hipGraphCreate(&p->graph, 0));
    hipKernelNodeParams kp{};
    const BatchDesc *arg = p->dev;
    const BatchRowDesc *rarg = p->rdev;
    void *args[] = {(void *)&arg};
    void *rargs[] = {(void *)&rarg};
    kp.func = const_cast<void *>(p->rows ? batch_rows_kernel(p->prec, p->dagger, p->ls_t)
                                         : batch_kernel(p->prec, p->dagger));
    kp.gridDim = dim3((unsigned)p->nblocks);
    kp.blockDim = dim3((unsigned)p->threads);
    kp.sharedMemBytes = (unsigned)p->lds;
    kp.kernelParams = p->rows ? rargs : args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    DWF_HIP(hipGraphAddKernelNode(&node, p->graph, nullptr, 0, &kp));
    DWF_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    return DWF_OK;
}

int batch_launch(dwf_batch p, hipStream_t st) {
    if (!p->exec) return fail(DWF_EUNSUP, "dwf_batch_launch: plan has not been captured");
    DWF_HIP(hipGraphLaunch(p->exec, st));
    return DWF_OK;
}

int batch_free(dwf_batch p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    (void)hipFree(p->dev);
    (void)hipFree(p->rdev);
    (void)hipFree(p->ptrs);
    delete p;
    return DWF_OK;
}

}  // namespace dwf
