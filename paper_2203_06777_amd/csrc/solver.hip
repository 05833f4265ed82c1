// Conjugate gradient on the Schur normal operator M_pc^dag M_pc, in FP64 and
// as FP64 defect correction around a low-precision inner CG.
//
// An iteration is six launches with no host round trip:
//   y = M_pc p                     two hopping kernels; the second also writes
//                                  partials of |y|^2 = <p, A p>
//   alpha = |r|^2 / |y|^2          one single-block kernel
//   r -= alpha M_pc^dag y          two hopping kernels; A p lives only in registers of
//                                  the second, which updates r and writes |r|^2 partials
//   beta, |r|^2, stop flag         one single-block kernel
//   x += alpha p ; p = r + beta p  one streaming kernel
// The scalars live in device memory.  The host reads the stop flag one
// iteration behind (the beta kernel also writes it into mapped host memory; the host
// waits on an event), so the GPU queue never drains; in an iteration queued after the stop every hopping kernel
// finds the stop flag set and returns at once, the alpha kernel clears the live
// flag, and x, r and p stay untouched.  With a 16-bit
// operator the search direction is kept only in that format: it is the
// hopping kernels' input, and x moves along exactly the p that A was applied to.
#include <chrono>
#include <cmath>

#include "dwf_device.h"

namespace dwf {

enum { S_RR = 0, S_PAP = 1, S_ALPHA = 2, S_BETA = 3, S_STOP = 4, S_DONE = 5, S_ITERS = 6, S_LIVE = 7, S_RED = 8 };
constexpr int kSumThreads = 1024;

// Sum of n per-workgroup partials by one workgroup of kSumThreads lanes, in a
// fixed order: four independent strided loads per round keep the requests in
// flight (the sums are latency bound), then a wave shuffle tree and an LDS pass.
// The result is valid in thread 0.
__device__ inline double sum_partials(const double *partials, long n) {
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    long k = threadIdx.x;
    for (; k + 3 * kSumThreads < n; k += 4 * kSumThreads) {
        a0 += partials[k];
        a1 += partials[k + kSumThreads];
        a2 += partials[k + 2 * kSumThreads];
        a3 += partials[k + 3 * kSumThreads];
    }
    for (; k < n; k += kSumThreads) a0 += partials[k];
    double v = (a0 + a1) + (a2 + a3);
    __shared__ double sa[kSumThreads / 64];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (threadIdx.x % 64 == 0) sa[threadIdx.x / 64] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        v = 0;
        for (int w = 0; w < kSumThreads / 64; ++w) v += sa[w];
    }
    return v;
}

// alpha = |r|^2 / <p, A p>, with <p, A p> = |M_pc p|^2 summed from the hopping kernel's
// partials; S_LIVE says whether this iteration updates x, r and p.
__global__ void __launch_bounds__(kSumThreads) k_cg_alpha(double *scal, const double *partials, long nparts) {
    const double pap = sum_partials(partials, nparts);
    if (threadIdx.x != 0) return;
    scal[S_LIVE] = 0;
    if (scal[S_DONE] != 0) return;
    scal[S_PAP] = pap;
    if (!isfinite(pap) || pap <= 0.0) {
        scal[S_DONE] = 2;
        return;
    }
    scal[S_ALPHA] = scal[S_RR] / pap;
    scal[S_LIVE] = 1;
}

// |r|^2 of the updated residual -> beta and the stop flag; the flag is also written to
// host memory (host_done), which the host polls instead of copying the scalars back.
__global__ void __launch_bounds__(kSumThreads) k_cg_beta(double *scal, const double *partials, long nparts,
                                                         double *host_done) {
    const double rr = sum_partials(partials, nparts);
    if (threadIdx.x != 0 || scal[S_LIVE] == 0) return;
    scal[S_ITERS] += 1;
    if (!isfinite(rr)) {
        scal[S_DONE] = 2;
        *host_done = 2;
        return;
    }
    scal[S_BETA] = rr / scal[S_RR];
    scal[S_RR] = rr;
    if (rr <= scal[S_STOP]) {
        scal[S_DONE] = 1;
        *host_done = 1;
    }
}

// x += alpha p ; p = r + beta p.  x and r in PV (FP64 or FP32), p in PP (PV, or the
// 16-bit operator format), arithmetic in PV's type.
template <int PV, int PP>
__global__ void __launch_bounds__(256) k_cg_px(u32x4 *x, const u32x4 *r, u32x4 *p, const double *scal, long nrows,
                                               int Ls) {
    if (scal[S_LIVE] == 0) return;
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= nrows * Ls) return;
    const long c = t / Ls;
    const int s = (int)(t - c * Ls);
    using A = typename PT<PV>::A;
    const A alpha = (A)scal[S_ALPHA], beta = (A)scal[S_BETA];
    A xv[24], rv[24], pv[24];
    load_spinor<PP>(p, c, Ls, s, pv);
    load_spinor<PV>(x, c, Ls, s, xv);
    load_spinor<PV>(r, c, Ls, s, rv);
#pragma unroll
    for (int k = 0; k < 24; ++k) {
        xv[k] = xv[k] + alpha * pv[k];
        pv[k] = rv[k] + beta * pv[k];
    }
    store_spinor<PV>(x, c, Ls, s, xv);
    store_spinor<PP>(p, c, Ls, s, pv);
}

// out = factor * in with a precision change.
template <int PI, int PO>
__global__ void __launch_bounds__(256) k_convert_scale(u32x4 *out, const u32x4 *in, double factor, long nrows,
                                                       int Ls) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= nrows * Ls) return;
    const long c = t / Ls;
    const int s = (int)(t - c * Ls);
    double v[24];
    load_spinor<PI>(in, c, Ls, s, v);
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] *= factor;
    store_spinor<PO>(out, c, Ls, s, v);
}

// The FP64 residual refresh of the FP32 inner iteration (a reliable update): with r the
// recursive FP32 residual and p the direction the last iteration built from it (old scaling),
// r' = scale * r64 is the true residual in the new scaling and the direction is rebuilt from it,
//   p' = r' + c (p - r),   c = (|r_true|^2 / |r|^2) (scale / old scale),
// i.e. p - r = beta p_prev (the previous direction) carried over with the beta of the true residual.
__global__ void __launch_bounds__(256) k_refresh_f32(u32x4 *r, u32x4 *p, const u32x4 *r64, double scale, double c,
                                                     long nrows, int Ls) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= nrows * Ls) return;
    const long row = t / Ls;
    const int s = (int)(t - row * Ls);
    double rt[24];
    float rv[24], pv[24];
    load_spinor<DWF_F64>(r64, row, Ls, s, rt);
    load_spinor<DWF_F32>(r, row, Ls, s, rv);
    load_spinor<DWF_F32>(p, row, Ls, s, pv);
    const float cf = (float)c;
#pragma unroll
    for (int k = 0; k < 24; ++k) {
        const float rn = (float)(scale * rt[k]);
        pv[k] = rn + cf * (pv[k] - rv[k]);
        rv[k] = rn;
    }
    store_spinor<DWF_F32>(r, row, Ls, s, rv);
    store_spinor<DWF_F32>(p, row, Ls, s, pv);
}

// y (FP64) += a * x (FP32).
__global__ void __launch_bounds__(256) k_axpy_f32_to_f64(u32x4 *y, const u32x4 *x, double a, long nrows, int Ls) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= nrows * Ls) return;
    const long c = t / Ls;
    const int s = (int)(t - c * Ls);
    double yv[24], xv[24];
    load_spinor<DWF_F64>(y, c, Ls, s, yv);
    load_spinor<DWF_F32>(x, c, Ls, s, xv);
#pragma unroll
    for (int k = 0; k < 24; ++k) yv[k] += a * xv[k];
    store_spinor<DWF_F64>(y, c, Ls, s, yv);
}

// r (PR) -= alpha * w (PW) when the iteration is live, with one FP64 partial of
// the new |r|^2 per workgroup (fixed-order shuffle tree); the streaming form of the
// CG epilogue for operators whose last factor is not a hopping kernel.
template <int PR, int PW>
__global__ void __launch_bounds__(256) k_cg_residual(u32x4 *r, const u32x4 *w, const double *cg_alpha,
                                                     const double *cg_live, double *partials, long nrows, int Ls) {
    if (*cg_live == 0) return;  // the sums are ignored when the iteration is not live
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    const bool active = t < nrows * Ls;
    using RA = typename PT<PR>::A;
    double part = 0;
    if (active) {
        const long c = t / Ls;
        const int s = (int)(t - c * Ls);
        RA rv[24];
        typename PT<PW>::A wv[24];
        load_spinor<PR>(r, c, Ls, s, rv);
        load_spinor<PW>(w, c, Ls, s, wv);
        const RA ca = (RA)*cg_alpha;
#pragma unroll
        for (int k = 0; k < 24; ++k) {
            rv[k] = rv[k] - ca * (RA)wv[k];
            part += (double)rv[k] * (double)rv[k];
        }
        store_spinor<PR>(r, c, Ls, s, rv);
    }
    // wavefront shuffle tree, then the four wave sums in order
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) part += __shfl_xor(part, off, 64);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_set_scalars(double *scal, double stop) {
    if (threadIdx.x != 0) return;
    scal[S_RR] = scal[S_RED];
    scal[S_STOP] = stop;
    scal[S_DONE] = 0;
    scal[S_ITERS] = 0;
    scal[S_LIVE] = 0;
}

static inline unsigned nb256(long n) { return (unsigned)((n + 255) / 256); }

int launch_cg_residual(dwf_ctx ctx, void *r, int prec_r, const void *w, int prec_w, const double *cg_alpha,
                       const double *cg_live, double *partials, long *nparts, hipStream_t st) {
    const Geom &g = ctx->g;
    const unsigned nb = nb256(g.half * g.Ls);
    if (nparts) *nparts = nb;
    u32x4 *r4 = (u32x4 *)r;
    const u32x4 *w4 = (const u32x4 *)w;
#define DWF_RES(PR, PW) hipLaunchKernelGGL((k_cg_residual<PR, PW>), nb, 256, 0, st, r4, w4, cg_alpha, cg_live, \
                                           partials, g.half, g.Ls)
    if (prec_r == DWF_F64 && prec_w == DWF_F64) DWF_RES(DWF_F64, DWF_F64);
    else if (prec_r == DWF_F32 && prec_w == DWF_F32) DWF_RES(DWF_F32, DWF_F32);
    else if (prec_r == DWF_F32 && prec_w == DWF_F16) DWF_RES(DWF_F32, DWF_F16);
    else if (prec_r == DWF_F32 && prec_w == DWF_BF16) DWF_RES(DWF_F32, DWF_BF16);
    else return fail(DWF_EUNSUP, "CG residual update: unsupported precision pair");
#undef DWF_RES
    DWF_HIP(hipGetLastError());
    return DWF_OK;
}

static int ensure_work(dwf_ctx ctx) {
    CgWork &w = ctx->work;
    if (w.x64) return DWF_OK;
    const Geom &g = ctx->g;
    const size_t b64 = cb_bytes(g, DWF_F64), b32 = cb_bytes(g, DWF_F32), b16 = cb_bytes(g, DWF_F16);
    void **f64[] = {&w.x64, &w.r64, &w.p64, &w.ap64};
    void **f32[] = {&w.e32, &w.r32, &w.p32};
    for (void **p : f64)
        if (hipMalloc(p, b64) != hipSuccess) return fail(DWF_ENOMEM, "solver workspace: hipMalloc failed");
    for (void **p : f32)
        if (hipMalloc(p, b32) != hipSuccess) return fail(DWF_ENOMEM, "solver workspace: hipMalloc failed");
    if (hipMalloc(&w.p16, b16) != hipSuccess) return fail(DWF_ENOMEM, "solver workspace: hipMalloc failed");
    if (hipMalloc(&w.full_tmp, 2 * b64) != hipSuccess) return fail(DWF_ENOMEM, "solver workspace: hipMalloc failed");
    w.bytes = 4 * b64 + 3 * b32 + b16 + 2 * b64;
    return DWF_OK;
}

// Synchronous FP64 norm of an internal field.
static int norm2_sync(dwf_ctx ctx, const void *x, int prec, double *out, hipStream_t st) {
    const long n = ctx->g.half * ctx->g.Ls * 12;
    int rc = launch_reduce(ctx->partials, ctx->scal + S_RED, x, nullptr, n, prec, 0, st);
    if (rc) return rc;
    DWF_HIP(hipMemcpyAsync(ctx->host_scal, ctx->scal + S_RED, sizeof(double), hipMemcpyDeviceToHost, st));
    DWF_HIP(hipStreamSynchronize(st));
    *out = ctx->host_scal[0];
    return DWF_OK;
}

// CG iterations on A e = r from the current (x, r) until |r|^2 <= stop_rr or the
// iteration budget is used: from p = r, or (keep_p) from the search direction p
// the caller left in place.  vprec is the precision of x and r (F64 or F32);
// oprec the operator's, which p is stored in.
static int cg_core(dwf_ctx ctx, int vprec, int oprec, void *x, void *r, void *p, double stop_rr, int budget,
                   bool keep_p, int *iters_out, int *status_out, hipStream_t st, double *rr_out = nullptr) {
    const Geom &g = ctx->g;
    const long n = g.half * g.Ls * 12;
    const unsigned nb = nb256(g.half * g.Ls);
    u32x4 *x4 = (u32x4 *)x, *p4 = (u32x4 *)p;
    const u32x4 *r4 = (const u32x4 *)r;
    double *scal = ctx->scal, *parts = ctx->dhop_partials;
    void *y = ctx->tmp[1];
    int rc;
    // |r|^2 -> scal[S_RED] -> scal[S_RR]; p = r
    if ((rc = launch_reduce(ctx->partials, scal + S_RED, r, nullptr, n, vprec, 0, st))) return rc;
    hipLaunchKernelGGL(k_set_scalars, 1, 64, 0, st, scal, stop_rr);
    if (!keep_p) {
        if (oprec == vprec) DWF_HIP(hipMemcpyAsync(p, r, cb_bytes(g, vprec), hipMemcpyDeviceToDevice, st));
        else if ((rc = launch_convert(g, p, oprec, r, vprec, 1, st))) return rc;
    }
    hipEvent_t ev[2] = {(hipEvent_t)ctx->events[0], (hipEvent_t)ctx->events[1]};
    double *hs = ctx->host_scal;
    *ctx->host_flag = 0;  // the previous solve has drained the stream
    for (int it = 0; it < budget; ++it) {
        long np_y = 0, np_r = 0;
        // every hopping kernel of an iteration queued after the stop returns at once (S_DONE set)
        if ((rc = op_mpc(ctx, y, p, 0, oprec, st, parts, &np_y, scal + S_DONE))) return rc;
        hipLaunchKernelGGL(k_cg_alpha, 1, kSumThreads, 0, st, scal, parts, np_y);
        if ((rc = op_mpcdag_cg(ctx, r, vprec, y, oprec, scal + S_ALPHA, scal + S_LIVE, parts, &np_r, st,
                               scal + S_DONE)))
            return rc;
        hipLaunchKernelGGL(k_cg_beta, 1, kSumThreads, 0, st, scal, parts, np_r, ctx->host_flag_dev);
        if (vprec == DWF_F64)
            hipLaunchKernelGGL((k_cg_px<DWF_F64, DWF_F64>), nb, 256, 0, st, x4, r4, p4, scal, g.half, g.Ls);
        else if (oprec == DWF_F16)
            hipLaunchKernelGGL((k_cg_px<DWF_F32, DWF_F16>), nb, 256, 0, st, x4, r4, p4, scal, g.half, g.Ls);
        else if (oprec == DWF_BF16)
            hipLaunchKernelGGL((k_cg_px<DWF_F32, DWF_BF16>), nb, 256, 0, st, x4, r4, p4, scal, g.half, g.Ls);
        else
            hipLaunchKernelGGL((k_cg_px<DWF_F32, DWF_F32>), nb, 256, 0, st, x4, r4, p4, scal, g.half, g.Ls);
        DWF_HIP(hipGetLastError());
        // stop flag, read one iteration behind: once iteration it - 1 has completed, the flag
        // holds its stop decision (or a later one)
        DWF_HIP(hipEventRecord(ev[it & 1], st));
        if (it >= 1) {
            DWF_HIP(hipEventSynchronize(ev[(it - 1) & 1]));
            if (*ctx->host_flag != 0) break;
        }
    }
    DWF_HIP(hipStreamSynchronize(st));
    DWF_HIP(hipMemcpy(hs, scal, 8 * sizeof(double), hipMemcpyDeviceToHost));
    *iters_out = (int)hs[S_ITERS];
    *status_out = (int)hs[S_DONE];
    if (rr_out) *rr_out = hs[S_RR];
    return DWF_OK;
}

int cg_solve(dwf_ctx ctx, void *x, const void *b, double tol, int maxit, int mode, dwf_cg_stats *stats,
             hipStream_t st) {
    auto t0 = std::chrono::steady_clock::now();
    int rc = ensure_work(ctx);
    if (rc) return rc;
    const Geom &g = ctx->g;
    CgWork &w = ctx->work;
    const long n = g.half * g.Ls * 12;
    const size_t b64 = cb_bytes(g, DWF_F64);
    double bb;
    if ((rc = norm2_sync(ctx, b, DWF_F64, &bb, st))) return rc;
    if (!std::isfinite(bb)) return fail(DWF_ENAN, "dwf_cg: right-hand side is not finite");
    dwf_cg_stats s{0, 0, 0.0, 0.0};
    auto finish = [&](int code) {
        s.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (stats) *stats = s;
        return code;
    };
    if (bb == 0.0) {
        DWF_HIP(hipMemsetAsync(x, 0, b64, st));
        DWF_HIP(hipStreamSynchronize(st));
        return finish(DWF_OK);
    }
    const int oprec = mode == 1 ? DWF_F32 : mode == 2 ? DWF_F16 : DWF_BF16;
    // Each inner solve gains a few digits, then the residual is recomputed in FP64.  With the
    // FP32 operator the iteration goes on from it (a reliable update): the true residual
    // replaces the recursive one and the search direction is rebuilt from it with the
    // previous direction carried over, so the Krylov space is kept; a 16-bit direction
    // carries too much rounding to be kept (172 against 165 iterations on the 24^4 x 12
    // workload), so those restart from p = r.
    // Defaults: FP32 inner solves gain four digits (three FP64 refreshes to 1e-10), 16-bit ones two
    // (their operator's rounding limits what one inner solve can win).
    double inner_tol = ctx->inner_tol > 0 ? ctx->inner_tol : (mode == 1 ? 1e-4 : 1e-2);
    int inner_maxit = ctx->inner_maxit > 0 ? ctx->inner_maxit : 2000;
    int total = 0;
    double rr = 0, prev_scale = 0, xx = 0, rec_rr = 0;  // rec_rr: the last inner solve's recursive |r|^2
    if ((rc = norm2_sync(ctx, x, DWF_F64, &xx, st))) return rc;
    bool x_zero = xx == 0.0;  // a zero start needs no operator application for its residual
    for (;;) {
        // r = b - A x (FP64)
        if (x_zero) {
            DWF_HIP(hipMemcpyAsync(w.r64, b, b64, hipMemcpyDeviceToDevice, st));
            rr = bb;
            x_zero = false;
        } else {
            if ((rc = op_mdagm(ctx, w.ap64, x, DWF_F64, ctx->tmp[1], st))) return rc;
            if ((rc = launch_residual64(ctx->partials, ctx->scal + S_RED, w.r64, b, w.ap64, n, st))) return rc;
            DWF_HIP(hipMemcpyAsync(ctx->host_scal, ctx->scal + S_RED, sizeof(double), hipMemcpyDeviceToHost, st));
            DWF_HIP(hipStreamSynchronize(st));
            rr = ctx->host_scal[0];
        }
        s.true_rel_resid = std::sqrt(rr / bb);
        if (!std::isfinite(rr)) return finish(fail(DWF_ENAN, "dwf_cg: residual is not finite"));
        if (s.true_rel_resid <= tol) return finish(DWF_OK);
        if (total >= maxit) {
            s.inner_iters = total;
            return finish(fail(DWF_ENOCONV, "dwf_cg: iteration limit reached before tolerance"));
        }
        s.outer_iters += 1;
        int it = 0, status = 0;
        if (mode == 0) {
            if ((rc = cg_core(ctx, DWF_F64, DWF_F64, x, w.r64, w.p64, tol * tol * bb, maxit - total, false, &it,
                              &status, st)))
                return rc;
        } else {
            // inner solve A e = r^, r^ = r * sqrt(n)/|r| in FP32 (components of order one)
            const double scale = std::sqrt((double)n) / std::sqrt(rr);
            const unsigned nbv = nb256(g.half * g.Ls);
            void *p = oprec == DWF_F32 ? w.p32 : w.p16;
            const bool keep_p = oprec == DWF_F32 && prev_scale > 0 && rec_rr > 0;
            if (keep_p) {  // reliable update: true residual in the new scaling, direction rebuilt from it
                const double c = (prev_scale / scale) * (double)n / rec_rr;
                hipLaunchKernelGGL(k_refresh_f32, nbv, 256, 0, st, (u32x4 *)w.r32, (u32x4 *)p, (const u32x4 *)w.r64,
                                   scale, c, g.half, g.Ls);
            } else {
                hipLaunchKernelGGL((k_convert_scale<DWF_F64, DWF_F32>), nbv, 256, 0, st, (u32x4 *)w.r32,
                                   (const u32x4 *)w.r64, scale, g.half, g.Ls);
            }
            DWF_HIP(hipGetLastError());
            DWF_HIP(hipMemsetAsync(w.e32, 0, cb_bytes(g, DWF_F32), st));
            const int budget = std::min(inner_maxit, maxit - total);
            prev_scale = scale;
            // relative reduction of this inner solve: inner_tol, but no further than the outer
            // tolerance needs (with a factor 2 of margin for the FP64 residual it is checked on)
            const double want = std::max(inner_tol, 0.5 * tol * std::sqrt(bb / rr));
            if ((rc = cg_core(ctx, DWF_F32, oprec, w.e32, w.r32, p, want * want * (double)n, budget, keep_p, &it,
                              &status, st, &rec_rr)))
                return rc;
            hipLaunchKernelGGL(k_axpy_f32_to_f64, nb256(g.half * g.Ls), 256, 0, st, (u32x4 *)x,
                               (const u32x4 *)w.e32, 1.0 / scale, g.half, g.Ls);
            DWF_HIP(hipGetLastError());
        }
        total += it;
        s.inner_iters = total;
        if (status == 2) return finish(fail(DWF_ENAN, "dwf_cg: non-finite value in the iteration"));
        if (it == 0) return finish(fail(DWF_ENOCONV, "dwf_cg: no progress"));
    }
}

}  // namespace dwf
