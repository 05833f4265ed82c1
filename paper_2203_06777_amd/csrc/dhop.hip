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
//
// This file holds that site kernel, the launcher of the row-block kernel whose
// body (links and x-neighbour rows staged in LDS) is in dwf_rows.h, and the
// launch-shape helpers.
#include <algorithm>
#include <type_traits>

#include "dwf_rows.h"

namespace dwf {

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
    if (a.stop != nullptr && *a.stop != 0) return;

    A acc[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] = 0;

    if (active) dhop_site<PI, DAG, Off>(a.links, a.in, a.lat, Ls, a.parity, c, s, acc);

    const A alpha = (A)a.alpha;
    const Off zoff = spinor_off<PI, Off>(c, Ls, s);
    if constexpr (EPI == EPI_SCALE || EPI == EPI_INTERIOR) {
        if (!active) return;
        if constexpr (EPI == EPI_INTERIOR) {
            const Lat &g = a.lat;
            const unsigned uc = (unsigned)c, rest = fdiv(uc, g.L0h, g.inv0h), xh = uc - rest * g.L0h;
            const unsigned r2 = fdiv(rest, g.L1, g.inv1), x1 = rest - r2 * g.L1;
            const unsigned x3 = fdiv(r2, g.L2, g.inv2), x2 = r2 - x3 * g.L2;
            const unsigned x0 = 2 * xh + ((a.parity + x1 + x2 + x3) & 1);
            if (dd_boundary(a.dd_cut, x0, x1, x2, x3, 2 * g.L0h, g.L1, g.L2, g.L3)) return;
        }
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
        m5inv_lds<DAG>(a.m5i, Ls, lds, j, s, acc);
        if (!active) return;
    }
    store_spinor_off<PO>(a.out, spinor_off<PO, Off>(c, Ls, s), Ls * 16, acc, a.nt_store != 0);
}

template <int PI, int PO, int DAG, int EPI, int LS>
__global__ void __launch_bounds__(kMaxDhopThreads) k_dhop_rows(const DhopArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    if constexpr (EPI == EPI_CG)
        if (*a.cg_live == 0) return;  // the solver has stopped: r stays as it is
    if (a.stop != nullptr && *a.stop != 0) return;
    const long lb = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (long)blockIdx.x;
    row_block<PI, PO, DAG, EPI, LS>(a, (unsigned)lb * (unsigned)a.rows, a.in, a.out, a.links, smem);
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
    // FP64 rows are twice as long in bytes and two workgroups fit a CU (LDS): a 4 x 4 tile keeps
    // the rows a tile shares closer together (measured at 32^4 x 16: 1079-1090 us against
    // 1162-1164 us for 8 x 4; the other precisions within 1-3% of each other on either tile)
    const int ty = prec == DWF_F64 ? 4 : 8;
    r.ty = g.L[1] % ty == 0 ? ty : (g.L[1] % 4 == 0 ? 4 : 1);
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

// Mooee = d - e K:  Mooee^-1 = sum_n coef[n] K^n with coef[n] = q^-(n+1) / (e (1 + mf q^-Ls)),
// q = d / e, and the recurrence factors 1/d, e/d.  The Moebius Schur factor
// Mooee^-1 (b + c K) = -(c/e) + (b + c q) Mooee^-1 (b + c K differs from Mooee by a multiple of
// the identity) is applied as y -> f y + g v after the inverse.
void m5inv_setup(const Geom &g, M5InvCoef &m, bool schur) {
    const double d = mooee_d(g), e = mooee_e(g), q = d / e;
    double dn = 1.0;
    for (int n = 0; n < g.Ls; ++n) dn /= q;  // q^-Ls
    const double norm = 1.0 / (1.0 + g.mf * dn) / e;
    double p = 1.0 / q;
    for (int n = 0; n < kMaxLs; ++n) {
        m.coef[n] = n < g.Ls ? p * norm : 0.0;
        p /= q;
    }
    m.mf = g.mf;
    m.id = 1.0 / d;
    m.ed = e / d;
    m.schur = schur && g.mobius ? 1 : 0;
    m.f = m.schur ? g.b5 + g.c5 * q : 1.0;
    m.g = m.schur ? -g.c5 / e : 0.0;
}

template <int PI, int PO, int DAG, int EPI>
static int launch_t(const DhopArgs &a, int ls_t, long nblocks, int threads, hipStream_t st) {
    using A = typename PT<PI>::A;
    const dim3 grid((unsigned)nblocks), block(threads);
    if (a.rows > 0) {
        // FP32 / FP64 exterior: one more site slot after the x-row (the x-cut neighbour)
        constexpr bool ghost = EPI == EPI_EXTERIOR && (PI == DWF_F32 || PI == DWF_F64);
        const size_t shm = std::max({row_lds_bytes(a.rows, (int)a.lat.L0h, a.Ls, PI) +
                                         (ghost ? (size_t)a.Ls * 24 * sizeof(A) : (size_t)0),
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
    if constexpr (EPI == EPI_EXTERIOR || EPI == EPI_INTERIOR_ROWS) {
        return fail(DWF_EUNSUP, "hopping kernel: this decomposed launch needs the row kernel");
    } else {
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
}

template <int PI, int PO>
static int launch_pp(const DhopArgs &a, int ls_t, int dagger, int epi, long nb, int th, hipStream_t st) {
    if (epi == EPI_INTERIOR || epi == EPI_EXTERIOR || epi == EPI_INTERIOR_ROWS) {
        // the interior or the boundary rows of a decomposed apply: same storage in and out
        if constexpr (PI == PO) {
            if (epi == EPI_EXTERIOR) {
                if (dagger) return launch_t<PI, PO, 1, EPI_EXTERIOR>(a, ls_t, nb, th, st);
                return launch_t<PI, PO, 0, EPI_EXTERIOR>(a, ls_t, nb, th, st);
            }
            if (epi == EPI_INTERIOR_ROWS) {
                if (dagger) return launch_t<PI, PO, 1, EPI_INTERIOR_ROWS>(a, ls_t, nb, th, st);
                return launch_t<PI, PO, 0, EPI_INTERIOR_ROWS>(a, ls_t, nb, th, st);
            }
            if (dagger) return launch_t<PI, PO, 1, EPI_INTERIOR>(a, ls_t, nb, th, st);
            return launch_t<PI, PO, 0, EPI_INTERIOR>(a, ls_t, nb, th, st);
        }
        return fail(DWF_EUNSUP, "hopping kernel: a decomposed launch needs equal input and output precision");
    }
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

bool fill_dhop_args(dwf_ctx ctx, const DhopShape &shape, int prec_in, int out_parity, DhopArgs &a) {
    const Geom &g = ctx->g;
    a = DhopArgs{};
    a.links = (const char *)ctx->links[prec_in][out_parity];
    a.lat = make_lat(g.L);
    a.half = g.half;
    a.Ls = g.Ls;
    a.spb = shape.spb;
    a.parity = out_parity;
    a.xcd = shape.xcd;
    a.nt_store = shape.nt_store;
    a.alpha = 1.0;
    a.d5 = mooee_d(g);
    a.e5 = mooee_e(g);
    a.mf = g.mf;
    m5inv_setup(g, a.m5i, false);
    const bool rows_mode = shape.rows > 0 && row_shape_ok(g, shape, prec_in, ctx->lds_limit);
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
    return rows_mode;
}

int launch_dhop(dwf_ctx ctx, const DhopCall &c, const DhopShape &shape_in, hipStream_t st) {
    const Geom &g = ctx->g;
    DhopShape shape = (shape_in.spb > 0 || shape_in.rows > 0) ? shape_in : default_shape(g);
    DhopArgs a;
    const bool rows_mode = fill_dhop_args(ctx, shape, c.prec_in, c.out_parity, a);
    a.in = (const char *)c.in;
    a.out = (char *)c.out;
    a.z = (const char *)c.z;
    a.alpha = c.alpha;
    a.beta = c.beta;
    a.norm_out = (c.epi == EPI_M5 || c.epi == EPI_CG) ? c.norm_out : nullptr;
    a.cg_alpha = c.cg_alpha;
    a.cg_live = c.cg_live;
    if (c.schur_coef) m5inv_setup(g, a.m5i, true);
    if (c.links) a.links = (const char *)c.links;
    a.dd_cut = (c.epi == EPI_INTERIOR || c.epi == EPI_EXTERIOR || c.epi == EPI_INTERIOR_ROWS) ? c.dd_cut : 0u;
    a.stop = c.stop;
    if (c.epi == EPI_EXTERIOR) {
        const bool wide = c.prec_in == DWF_F32 || c.prec_in == DWF_F64;
        if (!rows_mode || !c.row_list || !c.seg_off || !(wide ? c.ghost : c.recv))
            return fail(DWF_EINVAL, "hopping kernel: the exterior launch needs the row kernel, a row list and faces");
        if (wide && shape.rows != 1)
            return fail(DWF_EINVAL, "hopping kernel: the FP32 / FP64 exterior launch takes one row per workgroup");
        a.row_list = c.row_list;
        a.nrows = (unsigned)c.nrows_list;
        a.recv = (const char *)c.recv;
        a.ghost = (const char *)c.ghost;
        for (int k = 0; k < 9; ++k) a.seg_off[k] = c.seg_off[k];
        if (c.nrows_list == 0) return DWF_OK;
    }
    if (c.epi == EPI_INTERIOR_ROWS && (!rows_mode || shape.rows != 1 || (c.dd_cut & 1u)))
        return fail(DWF_EINVAL, "hopping kernel: the whole-row interior launch needs one row per workgroup and no x cut");
    if (c.epi == EPI_CG && (!c.norm_out || !c.cg_alpha || !c.cg_live || !c.z))
        return fail(DWF_EINVAL, "hopping kernel: CG epilogue needs z, partials and the solver scalars");
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
