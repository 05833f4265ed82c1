// Batched hopping term: many right-hand sides of several lattices (of
// different volumes and Ls) in one persistent launch, recorded as a HIP graph.
//
// Work items are (lattice, tile, rhs) with the RHS index innermost, so the
// items that share a tile's links run at the same time and the links are
// read from HBM once for all right-hand sides.  A fixed grid of resident
// workgroups walks the item list: workgroup b takes one contiguous run of
// items, and the XCD remap gives each XCD one contiguous part of the list, so
// neighbouring tiles share that XCD's L2.  The item loop ends for every
// workgroup after a fixed count, with no queue or atomics.
#include <vector>

#include "dwf_dhop_core.h"

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
    int prec = 0, dagger = 0, nlat = 0, total_rhs = 0, threads = 0;
    long nblocks = 0;
    BatchDesc host{};
    BatchDesc *dev = nullptr;
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

int batch_plan(const dwf_ctx *ctxs, int nlat, const int *nrhs, int prec, int dagger, dwf_batch *out) {
    dwf_batch p = new dwf_batch_s();
    p->prec = prec;
    p->dagger = dagger;
    p->nlat = nlat;
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
        hipFree(p->dev);
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
    for (int l = 0; l < p->nlat; ++l) p->host.lat[l].links = p->ctxs[l]->links[p->prec][out_parity];
    p->host.parity = out_parity;
    DWF_HIP(hipMemcpyAsync(p->ptrs, host.data(), host.size() * sizeof(void *), hipMemcpyHostToDevice, st));
    DWF_HIP(hipMemcpyAsync(p->dev, &p->host, sizeof(BatchDesc), hipMemcpyHostToDevice, st));
    DWF_HIP(hipStreamSynchronize(st));
    if (p->exec) {
        hipGraphExecDestroy(p->exec);
        p->exec = nullptr;
    }
    if (p->graph) {
        hipGraphDestroy(p->graph);
        p->graph = nullptr;
    }
    DWF_HIP(hipGraphCreate(&p->graph, 0));
    hipKernelNodeParams kp{};
    const BatchDesc *arg = p->dev;
    void *args[] = {(void *)&arg};
    kp.func = const_cast<void *>(batch_kernel(p->prec, p->dagger));
    kp.gridDim = dim3((unsigned)p->nblocks);
    kp.blockDim = dim3((unsigned)p->threads);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
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
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    hipFree(p->dev);
    hipFree(p->ptrs);
    delete p;
    return DWF_OK;
}

}  // namespace dwf
