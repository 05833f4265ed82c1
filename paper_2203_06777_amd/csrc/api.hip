// The C ABI of libdwf.so: argument validation, context lifetime and the
// composition of kernel launches for each entry point.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "dwf_common.h"

namespace dwf {

static thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    if (std::getenv("DWF_LOG")) std::fprintf(stderr, "[dwf] error %d: %s\n", code, msg.c_str());
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(DWF_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int batch_plan(const dwf_ctx *ctxs, int nlat, const int *nrhs, int prec, int dagger, dwf_batch *out);
int batch_capture(dwf_batch p, void *const *outs, const void *const *ins, int out_parity, hipStream_t st);
int batch_launch(dwf_batch p, hipStream_t st);
int batch_free(dwf_batch p);
int dd_create(dwf_ctx ctx, int prec, unsigned cut, dwf_dd *out);
int dd_dhop(dwf_dd d, void *out, const void *in, int out_parity, int dagger, hipStream_t st);
int dd_face_only(dwf_dd d, const void *in, int out_parity, int dagger, hipStream_t st);
int dd_destroy(dwf_dd d);

static bool valid_prec(int p) { return p >= DWF_F64 && p <= DWF_BF16; }

#define CHECK(cond, msg)                                  \
    do {                                                  \
        if (!(cond)) return ::dwf::fail(DWF_EINVAL, msg); \
    } while (0)

#define CHECK_CTX(ctx) CHECK((ctx) != nullptr, "null context")
#define CHECK_GAUGE(ctx)                                                                        \
    do {                                                                                        \
        if (!(ctx)->gauge_set) return ::dwf::fail(DWF_EUNSUP, "gauge field not set (dwf_set_gauge)"); \
    } while (0)

// Tuned launch shapes survive contexts: keyed by (prec, dagger, dims, Ls).
static std::mutex g_tune_mu;
static std::map<std::string, DhopShape> g_tune;
static bool g_tune_loaded = false;

// Cache key; the second field is dagger + 2 * family (0: plain hopping launch, 1: fused Schur pair).
static std::string tune_key(const Geom &g, int prec, int dagger, int family) {
    std::ostringstream k;
    k << prec << ' ' << dagger + 2 * family << ' ' << g.L[0] << ' ' << g.L[1] << ' ' << g.L[2] << ' ' << g.L[3] << ' ' << g.Ls;
    return k.str();
}

static void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("DWF_TUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        int p, d, l0, l1, l2, l3, ls, spb, xcd, spl, rows, ty, tz, tt, occ = 0;
        if (is >> p >> d >> l0 >> l1 >> l2 >> l3 >> ls >> spb >> xcd >> spl >> rows >> ty >> tz >> tt) {
            if (!(is >> occ)) occ = 0;
            std::ostringstream k;
            k << p << ' ' << d << ' ' << l0 << ' ' << l1 << ' ' << l2 << ' ' << l3 << ' ' << ls;
            DhopShape s;
            s.spb = spb;
            s.xcd = xcd;
            s.nt_store = spl;
            s.rows = rows;
            s.ty = ty;
            s.tz = tz;
            s.tt = tt;
            s.occ = occ;
            g_tune[k.str()] = s;
        }
    }
}

static void apply_tuned(dwf_ctx ctx) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    for (int p = 0; p < 4; ++p)
        for (int d = 0; d < 2; ++d) {
            const DhopShape def = default_row_shape(ctx->g, p, ctx->lds_limit);
            auto it = g_tune.find(tune_key(ctx->g, p, d, 0));
            ctx->shape[p][d] = it != g_tune.end() ? it->second : def;
            auto is = g_tune.find(tune_key(ctx->g, p, d, 1));
            ctx->shape_schur[p][d] = is != g_tune.end() ? is->second : def;
        }
}

static long cb_complex(const Geom &g) { return g.half * g.Ls * 12; }

}  // namespace dwf

using namespace dwf;

extern "C" {

const char *dwf_last_error(void) { return g_err.c_str(); }

int dwf_create(const dwf_geom *geom, dwf_ctx *out) {
    CHECK(geom != nullptr && out != nullptr, "dwf_create: null argument");
    *out = nullptr;
    for (int m = 0; m < 4; ++m)
        CHECK(geom->dims[m] >= 2 && geom->dims[m] % 2 == 0, "dwf_create: every extent must be even and >= 2");
    CHECK(geom->Ls >= 1 && geom->Ls <= kMaxLs, "dwf_create: Ls must be in [1, 64]");
    CHECK(std::isfinite(geom->M5) && std::isfinite(geom->mf), "dwf_create: M5 and mf must be finite");
    CHECK(std::fabs(5.0 - geom->M5) > 1e-12, "dwf_create: M5 = 5 makes M5op singular");
    CHECK(std::fabs(1.0 + geom->mf * std::pow(5.0 - geom->M5, -(double)geom->Ls)) > 1e-12,
          "dwf_create: 1 + mf (5 - M5)^-Ls = 0 makes M5op singular");
    const long vol = (long)geom->dims[0] * geom->dims[1] * geom->dims[2] * geom->dims[3];
    CHECK(vol / 2 < (1L << 24), "dwf_create: lattice too large (V/2 must be below 2^24 sites)");
    dwf_ctx c = new (std::nothrow) dwf_ctx_s();
    if (!c) return fail(DWF_ENOMEM, "dwf_create: out of host memory");
    for (int m = 0; m < 4; ++m) c->g.L[m] = geom->dims[m];
    c->g.Ls = geom->Ls;
    c->g.vol = vol;
    c->g.half = vol / 2;
    c->g.M5 = geom->M5;
    c->g.mf = geom->mf;
    c->g.antiperiodic = geom->antiperiodic_t ? 1 : 0;
    auto cleanup = [&](int code, const char *msg) {
        dwf_destroy(c);
        return fail(code, msg);
    };
    if (hipGetDevice(&c->device) != hipSuccess) return cleanup(DWF_EHIP, "dwf_create: no HIP device");
    if (int rc = noalloc_setup(c->device)) {
        const std::string msg = dwf_last_error();
        dwf_destroy(c);
        return fail(rc, msg);
    }
    {
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) == hipSuccess && lds > 0)
            c->lds_limit = (size_t)lds;
        int per_cu = 0;
        if (hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, c->device) ==
                hipSuccess &&
            per_cu > 0)
            c->lds_per_cu = (size_t)per_cu;
    }
    if (std::getenv("DWF_TEST_FAIL_ALLOC")) return cleanup(DWF_ENOMEM, "dwf_create: allocation failure forced");
    for (int p = 0; p < 4; ++p)
        for (int par = 0; par < 2; ++par)
            if (hipMalloc(&c->links[p][par], link_bytes(c->g, p)) != hipSuccess)
                return cleanup(DWF_ENOMEM, "dwf_create: hipMalloc of link tables failed");
    for (int k = 0; k < 2; ++k)
        if (hipMalloc(&c->tmp[k], cb_bytes(c->g, DWF_F64)) != hipSuccess)
            return cleanup(DWF_ENOMEM, "dwf_create: hipMalloc of temporaries failed");
    if (hipMalloc(&c->partials, sizeof(double) * 2 * kRedBlocks) != hipSuccess ||
        hipMalloc(&c->dhop_partials, sizeof(double) * (size_t)c->g.half) != hipSuccess ||
        hipMalloc(&c->scal, sizeof(double) * 16) != hipSuccess)
        return cleanup(DWF_ENOMEM, "dwf_create: hipMalloc of reduction buffers failed");
    if (hipHostMalloc((void **)&c->host_scal, sizeof(double) * 16, hipHostMallocDefault) != hipSuccess)
        return cleanup(DWF_ENOMEM, "dwf_create: pinned host allocation failed");
    // the solver's stop flag, written by the device straight into host memory
    if (hipHostMalloc((void **)const_cast<double **>(&c->host_flag), sizeof(double) * 2, hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void **)&c->host_flag_dev, (void *)c->host_flag, 0) != hipSuccess)
        return cleanup(DWF_ENOMEM, "dwf_create: mapped host allocation failed");
    for (int k = 0; k < 2; ++k)
        if (hipEventCreateWithFlags((hipEvent_t *)&c->events[k], hipEventDisableTiming) != hipSuccess)
            return cleanup(DWF_EHIP, "dwf_create: hipEventCreate failed");
    // cleared on the null stream, which a caller's non-blocking stream does not wait for
    if (hipMemset(c->scal, 0, sizeof(double) * 16) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        return cleanup(DWF_EHIP, "dwf_create: hipMemset failed");
    apply_tuned(c);
    *out = c;
    return DWF_OK;
}

int dwf_destroy(dwf_ctx c) {
    if (!c) return DWF_OK;
    (void)hipDeviceSynchronize();
    for (auto &pp : c->links)
        for (void *p : pp) (void)hipFree(p);
    for (void *p : c->tmp) (void)hipFree(p);
    (void)hipFree(c->partials);
    (void)hipFree(c->dhop_partials);
    (void)hipFree(c->scal);
    if (c->host_scal) (void)hipHostFree(c->host_scal);
    if (c->host_flag) (void)hipHostFree((void *)c->host_flag);
    for (void *e : c->events)
        if (e) (void)hipEventDestroy((hipEvent_t)e);
    CgWork &w = c->work;
    for (void *p : {w.x64, w.r64, w.p64, w.ap64, w.e32, w.r32, w.p32, w.p16, w.full_tmp}) (void)hipFree(p);
    delete c;
    return DWF_OK;
}

int dwf_field_bytes(dwf_ctx ctx, int prec, int full, size_t *bytes) {
    CHECK_CTX(ctx);
    CHECK(valid_prec(prec), "dwf_field_bytes: bad precision");
    CHECK(bytes != nullptr, "dwf_field_bytes: null output");
    *bytes = cb_bytes(ctx->g, prec) * (full ? 2 : 1);
    return DWF_OK;
}

int dwf_set_mobius(dwf_ctx ctx, double b, double c) {
    CHECK_CTX(ctx);
    CHECK(std::isfinite(b) && std::isfinite(c), "dwf_set_mobius: b and c must be finite");
    Geom g = ctx->g;
    g.b5 = b;
    g.c5 = c;
    g.mobius = !(b == 1.0 && c == 0.0);
    const double e = mooee_e(g), d = mooee_d(g);
    CHECK(std::fabs(e) > 1e-12 && std::fabs(d) > 1e-12, "dwf_set_mobius: Mooee = d - e K with d or e = 0");
    CHECK(std::fabs(1.0 + g.mf * std::pow(d / e, -(double)g.Ls)) > 1e-12,
          "dwf_set_mobius: 1 + mf (d/e)^-Ls = 0 makes Mooee singular");
    if (g.mobius && !ctx->tmp[2]) {
        DWF_HIP(hipDeviceSynchronize());
        if (hipMalloc(&ctx->tmp[2], cb_bytes(g, DWF_F64)) != hipSuccess)
            return fail(DWF_ENOMEM, "dwf_set_mobius: hipMalloc of the Moebius temporary failed");
    }
    DWF_HIP(hipDeviceSynchronize());  // work queued with the old coefficients finishes first
    ctx->g = g;
    return DWF_OK;
}

int dwf_get_mobius(dwf_ctx ctx, double *b, double *c) {
    CHECK_CTX(ctx);
    CHECK(b && c, "dwf_get_mobius: null pointer");
    *b = ctx->g.b5;
    *c = ctx->g.c5;
    return DWF_OK;
}

int dwf_set_gauge(dwf_ctx ctx, const double *U, void *stream) {
    CHECK_CTX(ctx);
    CHECK(U != nullptr, "dwf_set_gauge: null gauge pointer");
    hipStream_t st = (hipStream_t)stream;
    for (int p = 0; p < 4; ++p)
        for (int par = 0; par < 2; ++par) {
            int rc = launch_gather_links(ctx->g, ctx->links[p][par], U, par, p, st);
            if (rc) return rc;
        }
    ctx->gauge_set = true;
    return DWF_OK;
}

int dwf_pack(dwf_ctx ctx, void *internal, const double *canonical, int parity, int prec, void *stream) {
    CHECK_CTX(ctx);
    CHECK(internal && canonical, "dwf_pack: null pointer");
    CHECK(parity >= 0 && parity <= 2, "dwf_pack: parity must be 0, 1 or 2 (full)");
    CHECK(valid_prec(prec), "dwf_pack: bad precision");
    return launch_pack(ctx->g, internal, canonical, parity, prec, (hipStream_t)stream);
}

int dwf_unpack(dwf_ctx ctx, double *canonical, const void *internal, int parity, int prec, void *stream) {
    CHECK_CTX(ctx);
    CHECK(internal && canonical, "dwf_unpack: null pointer");
    CHECK(parity >= 0 && parity <= 2, "dwf_unpack: parity must be 0, 1 or 2 (full)");
    CHECK(valid_prec(prec), "dwf_unpack: bad precision");
    return launch_unpack(ctx->g, canonical, internal, parity, prec, (hipStream_t)stream);
}

int dwf_convert(dwf_ctx ctx, void *out, int out_prec, const void *in, int in_prec, int full, void *stream) {
    CHECK_CTX(ctx);
    CHECK(out && in, "dwf_convert: null pointer");
    CHECK(valid_prec(out_prec) && valid_prec(in_prec), "dwf_convert: bad precision");
    CHECK(out != in || out_prec == in_prec, "dwf_convert: in-place conversion between precisions");
    return launch_convert(ctx->g, out, out_prec, in, in_prec, full ? 2 : 1, (hipStream_t)stream);
}

int dwf_dhop(dwf_ctx ctx, void *out, const void *in, int out_parity, int dagger, int prec, void *stream) {
    CHECK_CTX(ctx);
    CHECK_GAUGE(ctx);
    CHECK(out && in, "dwf_dhop: null pointer");
    CHECK(out != in, "dwf_dhop: in and out must not alias");
    CHECK(out_parity == 0 || out_parity == 1, "dwf_dhop: out_parity must be 0 or 1");
    CHECK(dagger == 0 || dagger == 1, "dwf_dhop: dagger must be 0 or 1");
    CHECK(valid_prec(prec), "dwf_dhop: bad precision");
    DhopCall c{in, out, nullptr, out_parity, dagger, EPI_SCALE, 1.0, 0.0, prec, prec};
    return launch_dhop(ctx, c, ctx->shape[prec][dagger], (hipStream_t)stream);
}

int dwf_m5(dwf_ctx ctx, void *out, const void *in, int dagger, int inverse, int full, int prec, void *stream) {
    CHECK_CTX(ctx);
    CHECK(out && in, "dwf_m5: null pointer");
    CHECK((dagger == 0 || dagger == 1) && (inverse == 0 || inverse == 1), "dwf_m5: dagger/inverse must be 0 or 1");
    CHECK(valid_prec(prec), "dwf_m5: bad precision");
    return launch_m5(ctx->g, out, in, dagger, inverse, ctx->g.half * (full ? 2 : 1), prec, (hipStream_t)stream);
}

int dwf_mpc(dwf_ctx ctx, void *out, const void *in, int dagger, int prec, void *stream) {
    CHECK_CTX(ctx);
    CHECK_GAUGE(ctx);
    CHECK(out && in && out != in, "dwf_mpc: null or aliased pointer");
    CHECK(dagger == 0 || dagger == 1, "dwf_mpc: dagger must be 0 or 1");
    CHECK(valid_prec(prec), "dwf_mpc: bad precision");
    return op_mpc(ctx, out, in, dagger, prec, (hipStream_t)stream);
}

int dwf_mdagm(dwf_ctx ctx, void *out, const void *in, int prec, void *stream) {
    CHECK_CTX(ctx);
    CHECK_GAUGE(ctx);
    CHECK(out && in && out != in, "dwf_mdagm: null or aliased pointer");
    CHECK(valid_prec(prec), "dwf_mdagm: bad precision");
    return op_mdagm(ctx, out, in, prec, ctx->tmp[1], (hipStream_t)stream);
}

int dwf_dw(dwf_ctx ctx, void *out, const void *in, int dagger, int prec, void *stream) {
    CHECK_CTX(ctx);
    CHECK_GAUGE(ctx);
    CHECK(out && in && out != in, "dwf_dw: null or aliased pointer");
    CHECK(dagger == 0 || dagger == 1, "dwf_dw: dagger must be 0 or 1");
    CHECK(valid_prec(prec), "dwf_dw: bad precision");
    const size_t cb = cb_bytes(ctx->g, prec);
    const char *i = (const char *)in;
    char *o = (char *)out;
    hipStream_t st = (hipStream_t)stream;
    const Geom &g = ctx->g;
    // out_p = M5op in_p - 1/2 D_h^{p<-1-p} in_{1-p}
    // Moebius: out_p = Mooee in_p - 1/2 D_h^{p<-1-p} (b + cK) in_{1-p}
    //          out_p^dag = Mooee^dag in_p + (b + cK^dag) (-1/2 D_h^dag{p<-1-p} in_{1-p})
    for (int p = 0; p < 2; ++p) {
        int rc;
        if (!g.mobius) {
            DhopCall c{i + (1 - p) * cb, o + p * cb, i + p * cb, p, dagger, EPI_M5, -0.5, 0.0, prec, prec};
            rc = launch_dhop(ctx, c, ctx->shape[prec][dagger], st);
        } else if (!dagger) {
            if ((rc = launch_m5_op(g, ctx->tmp[2], i + (1 - p) * cb, g.b5, -g.c5, nullptr, 0.0, 0.0, 0, g.half, prec,
                                   st)))
                return rc;
            DhopCall c{ctx->tmp[2], o + p * cb, i + p * cb, p, 0, EPI_M5, -0.5, 0.0, prec, prec};
            rc = launch_dhop(ctx, c, ctx->shape[prec][0], st);
        } else {
            DhopCall c{i + (1 - p) * cb, ctx->tmp[2], nullptr, p, 1, EPI_SCALE, -0.5, 0.0, prec, prec};
            if ((rc = launch_dhop(ctx, c, ctx->shape[prec][1], st))) return rc;
            rc = launch_m5_op(g, o + p * cb, i + p * cb, mooee_d(g), mooee_e(g), ctx->tmp[2], g.b5, -g.c5, 1, g.half,
                              prec, st);
        }
        if (rc) return rc;
    }
    return DWF_OK;
}

int dwf_norm2(dwf_ctx ctx, double *result, const void *x, int full, int prec, void *stream) {
    CHECK_CTX(ctx);
    CHECK(result && x, "dwf_norm2: null pointer");
    CHECK(valid_prec(prec), "dwf_norm2: bad precision");
    hipStream_t st = (hipStream_t)stream;
    int rc = launch_reduce(ctx->partials, ctx->scal + 8, x, nullptr, cb_complex(ctx->g) * (full ? 2 : 1), prec, 0, st);
    if (rc) return rc;
    DWF_HIP(hipMemcpyAsync(ctx->host_scal, ctx->scal + 8, sizeof(double), hipMemcpyDeviceToHost, st));
    DWF_HIP(hipStreamSynchronize(st));
    *result = ctx->host_scal[0];
    return DWF_OK;
}

int dwf_cdot(dwf_ctx ctx, double *result, const void *x, const void *y, int full, int prec, void *stream) {
    CHECK_CTX(ctx);
    CHECK(result && x && y, "dwf_cdot: null pointer");
    CHECK(valid_prec(prec), "dwf_cdot: bad precision");
    hipStream_t st = (hipStream_t)stream;
    int rc = launch_reduce(ctx->partials, ctx->scal + 8, x, y, cb_complex(ctx->g) * (full ? 2 : 1), prec, 1, st);
    if (rc) return rc;
    DWF_HIP(hipMemcpyAsync(ctx->host_scal, ctx->scal + 8, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    DWF_HIP(hipStreamSynchronize(st));
    result[0] = ctx->host_scal[0];
    result[1] = ctx->host_scal[1];
    return DWF_OK;
}

int dwf_axpy(dwf_ctx ctx, void *y, double a_re, double a_im, const void *x, int full, int prec, void *stream) {
    CHECK_CTX(ctx);
    CHECK(y && x, "dwf_axpy: null pointer");
    CHECK(valid_prec(prec), "dwf_axpy: bad precision");
    return launch_axpy(y, a_re, a_im, x, cb_complex(ctx->g) * (full ? 2 : 1), prec, (hipStream_t)stream);
}

int dwf_cg_set_inner(dwf_ctx ctx, double inner_tol, int inner_maxit) {
    CHECK_CTX(ctx);
    ctx->inner_tol = inner_tol > 0 ? inner_tol : 0.0;
    ctx->inner_maxit = inner_maxit > 0 ? inner_maxit : 0;
    return DWF_OK;
}

int dwf_cg(dwf_ctx ctx, void *x, const void *b, double tol, int maxit, int mode, dwf_cg_stats *stats, void *stream) {
    CHECK_CTX(ctx);
    CHECK_GAUGE(ctx);
    CHECK(x && b && x != b, "dwf_cg: null or aliased pointer");
    CHECK(tol > 0 && std::isfinite(tol), "dwf_cg: tol must be positive");
    CHECK(maxit >= 1, "dwf_cg: maxit must be >= 1");
    CHECK(mode >= 0 && mode <= 3, "dwf_cg: mode must be 0..3");
    return cg_solve(ctx, x, b, tol, maxit, mode, stats, (hipStream_t)stream);
}

int dwf_solve(dwf_ctx ctx, void *x, const void *b, int dagger, double tol, int maxit, int mode, dwf_cg_stats *stats,
              void *stream) {
    CHECK_CTX(ctx);
    CHECK_GAUGE(ctx);
    CHECK(x && b && x != b, "dwf_solve: null or aliased pointer");
    CHECK(dagger == 0 || dagger == 1, "dwf_solve: dagger must be 0 or 1");
    CHECK(tol > 0 && std::isfinite(tol), "dwf_solve: tol must be positive");
    CHECK(maxit >= 1, "dwf_solve: maxit must be >= 1");
    CHECK(mode >= 0 && mode <= 3, "dwf_solve: mode must be 0..3");
    hipStream_t st = (hipStream_t)stream;
    const size_t cb = cb_bytes(ctx->g, DWF_F64);
    int rc;
    const char *be = (const char *)b, *bo = be + cb;
    char *xe = (char *)x, *xo = xe + cb;
    const Geom &g = ctx->g;
    void *u = ctx->tmp[2];
    // 1. t = M5op^-1 b_e  (into x_e, overwritten at the end)
    if ((rc = launch_m5(g, xe, be, dagger, 1, g.half, DWF_F64, st))) return rc;
    // 2. bh = b_o + 1/2 D^{o<-e} t   (into x_o)
    //    Moebius: bh = b_o + 1/2 D^{o<-e} (b + cK) t;  adjoint: b_o + (b + cK^dag) 1/2 D^dag{o<-e} t
    if (!g.mobius) {
        DhopCall c1{xe, xo, bo, 1, dagger, EPI_AXPY, 0.5, 1.0, DWF_F64, DWF_F64};
        if ((rc = launch_dhop(ctx, c1, ctx->shape[DWF_F64][dagger], st))) return rc;
    } else if (!dagger) {
        if ((rc = launch_m5_op(g, u, xe, g.b5, -g.c5, nullptr, 0.0, 0.0, 0, g.half, DWF_F64, st))) return rc;
        DhopCall c1{u, xo, bo, 1, 0, EPI_AXPY, 0.5, 1.0, DWF_F64, DWF_F64};
        if ((rc = launch_dhop(ctx, c1, ctx->shape[DWF_F64][0], st))) return rc;
    } else {
        DhopCall c1{xe, u, nullptr, 1, 1, EPI_SCALE, 0.5, 0.0, DWF_F64, DWF_F64};
        if ((rc = launch_dhop(ctx, c1, ctx->shape[DWF_F64][1], st))) return rc;
        if ((rc = launch_m5_op(g, xo, bo, 1.0, 0.0, u, g.b5, -g.c5, 1, g.half, DWF_F64, st))) return rc;
    }
    dwf_cg_stats s{0, 0, 0.0, 0.0};
    if (!dagger) {
        // 3. rhs = M_pc^dag bh (into x_e slot), x_o = CG solution from zero
        if ((rc = op_mpc(ctx, xe, xo, 1, DWF_F64, st))) return rc;
        DWF_HIP(hipMemsetAsync(xo, 0, cb, st));
        rc = cg_solve(ctx, xo, xe, tol, maxit, mode, &s, st);
        if (rc && rc != DWF_ENOCONV) return rc;
    } else {
        // 3'. y = (M_pc^dag M_pc)^-1 bh (into x_e slot), x_o = M_pc y
        DWF_HIP(hipMemsetAsync(xe, 0, cb, st));
        rc = cg_solve(ctx, xe, xo, tol, maxit, mode, &s, st);
        if (rc && rc != DWF_ENOCONV) return rc;
        int rc2 = op_mpc(ctx, xo, xe, 0, DWF_F64, st);
        if (rc2) return rc2;
    }
    // 4. x_e = M5op^-1 (b_e + 1/2 D^{e<-o} x_o)
    //    Moebius: Mooee^-1 (b_e + 1/2 D^{e<-o} (b + cK) x_o);  adjoint: Mooee^-dag (b_e + (b + cK^dag) 1/2 D^dag{e<-o} x_o)
    int rc3;
    if (!g.mobius) {
        DhopCall c2{xo, xe, be, 0, dagger, EPI_M5INV, 0.5, 1.0, DWF_F64, DWF_F64};
        rc3 = launch_dhop(ctx, c2, ctx->shape[DWF_F64][dagger], st);
    } else if (!dagger) {
        if ((rc3 = launch_m5_op(g, u, xo, g.b5, -g.c5, nullptr, 0.0, 0.0, 0, g.half, DWF_F64, st))) return rc3;
        DhopCall c2{u, xe, be, 0, 0, EPI_M5INV, 0.5, 1.0, DWF_F64, DWF_F64};
        rc3 = launch_dhop(ctx, c2, ctx->shape[DWF_F64][0], st);
    } else {
        DhopCall c2{xo, u, nullptr, 0, 1, EPI_SCALE, 0.5, 0.0, DWF_F64, DWF_F64};
        if ((rc3 = launch_dhop(ctx, c2, ctx->shape[DWF_F64][1], st))) return rc3;
        if ((rc3 = launch_m5_op(g, u, be, 1.0, 0.0, u, g.b5, -g.c5, 1, g.half, DWF_F64, st))) return rc3;
        rc3 = launch_m5(g, xe, u, 1, 1, g.half, DWF_F64, st);
    }
    if (rc3) return rc3;
    DWF_HIP(hipStreamSynchronize(st));
    if (stats) *stats = s;
    return rc;
}

int dwf_force(dwf_ctx ctx, double *F, const void *X, const void *Y, int kind, double scale, void *stream) {
    CHECK_CTX(ctx);
    CHECK(F && X && Y, "dwf_force: null pointer");
    CHECK(kind == 0 || kind == 1, "dwf_force: kind must be 0 or 1");
    if (kind == 1) CHECK_GAUGE(ctx);
    return launch_force(ctx, F, X, Y, kind, scale, (hipStream_t)stream);
}

int dwf_expi_links(dwf_ctx ctx, double *U, const double *P, double eps, void *stream) {
    CHECK_CTX(ctx);
    CHECK(U && P, "dwf_expi_links: null pointer");
    CHECK(U != P, "dwf_expi_links: U and P must not alias");
    CHECK(std::isfinite(eps), "dwf_expi_links: eps must be finite");
    return launch_expi_links(ctx->g, U, P, eps, (hipStream_t)stream);
}

int dwf_gauge_axpy(dwf_ctx ctx, double *Y, double a, const double *X, void *stream) {
    CHECK_CTX(ctx);
    CHECK(Y && X, "dwf_gauge_axpy: null pointer");
    return launch_axpy(Y, a, 0.0, X, ctx->g.vol * 36, DWF_F64, (hipStream_t)stream);
}

int dwf_gauge_norm2(dwf_ctx ctx, double *result, const double *X, void *stream) {
    CHECK_CTX(ctx);
    CHECK(result && X, "dwf_gauge_norm2: null pointer");
    hipStream_t st = (hipStream_t)stream;
    int rc = launch_reduce(ctx->partials, ctx->scal + 8, X, nullptr, ctx->g.vol * 36, DWF_F64, 0, st);
    if (rc) return rc;
    DWF_HIP(hipMemcpyAsync(ctx->host_scal, ctx->scal + 8, sizeof(double), hipMemcpyDeviceToHost, st));
    DWF_HIP(hipStreamSynchronize(st));
    *result = ctx->host_scal[0];
    return DWF_OK;
}

int dwf_dd_create(dwf_ctx ctx, int prec, int cuts, dwf_dd *dd) {
    CHECK_CTX(ctx);
    CHECK(dd != nullptr, "dwf_dd_create: null output");
    CHECK(valid_prec(prec), "dwf_dd_create: bad precision");
    CHECK(cuts >= 1 && cuts <= 15, "dwf_dd_create: cuts must be a nonzero mask of DWF_CUT_X|Y|Z|T");
    CHECK(ctx->g.half <= 0xffffffffL, "dwf_dd_create: more than 2^32 checkerboard sites");
    *dd = nullptr;
    return dd_create(ctx, prec, (unsigned)cuts, dd);
}

int dwf_dd_dhop(dwf_dd dd, void *out, const void *in, int out_parity, int dagger, void *stream) {
    CHECK(dd != nullptr, "dwf_dd_dhop: null plan");
    CHECK(out && in && out != in, "dwf_dd_dhop: null or aliased pointer");
    CHECK(out_parity == 0 || out_parity == 1, "dwf_dd_dhop: out_parity must be 0 or 1");
    CHECK(dagger == 0 || dagger == 1, "dwf_dd_dhop: dagger must be 0 or 1");
    return dd_dhop(dd, out, in, out_parity, dagger, (hipStream_t)stream);
}

int dwf_dd_faces(dwf_dd dd, const void *in, int out_parity, int dagger, void *stream) {
    CHECK(dd != nullptr && in != nullptr, "dwf_dd_faces: null pointer");
    CHECK(out_parity == 0 || out_parity == 1, "dwf_dd_faces: out_parity must be 0 or 1");
    CHECK(dagger == 0 || dagger == 1, "dwf_dd_faces: dagger must be 0 or 1");
    return dd_face_only(dd, in, out_parity, dagger, (hipStream_t)stream);
}

int dwf_dd_destroy(dwf_dd dd) { return dd_destroy(dd); }

int dwf_batch_plan(const dwf_ctx *ctxs, int nlat, const int *nrhs, int prec, int dagger, dwf_batch *plan) {
    CHECK(ctxs && nrhs && plan, "dwf_batch_plan: null pointer");
    CHECK(nlat >= 1 && nlat <= 16, "dwf_batch_plan: nlat must be in [1, 16]");
    CHECK(valid_prec(prec), "dwf_batch_plan: bad precision");
    CHECK(dagger == 0 || dagger == 1, "dwf_batch_plan: dagger must be 0 or 1");
    for (int l = 0; l < nlat; ++l) {
        CHECK(ctxs[l] != nullptr && nrhs[l] >= 1, "dwf_batch_plan: null context or nrhs < 1");
        CHECK_GAUGE(ctxs[l]);
    }
    return batch_plan(ctxs, nlat, nrhs, prec, dagger, plan);
}

int dwf_batch_capture(dwf_batch plan, void *const *outs, const void *const *ins, int out_parity, void *stream) {
    CHECK(plan && outs && ins, "dwf_batch_capture: null pointer");
    CHECK(out_parity == 0 || out_parity == 1, "dwf_batch_capture: out_parity must be 0 or 1");
    return batch_capture(plan, outs, ins, out_parity, (hipStream_t)stream);
}

int dwf_batch_launch(dwf_batch plan, void *stream) {
    CHECK(plan, "dwf_batch_launch: null plan");
    return batch_launch(plan, (hipStream_t)stream);
}

int dwf_batch_free(dwf_batch plan) {
    if (!plan) return DWF_OK;
    return batch_free(plan);
}

int dwf_tune(dwf_ctx ctx, int prec, int dagger, double *best_us, void *stream) {
    CHECK_CTX(ctx);
    CHECK_GAUGE(ctx);
    CHECK(valid_prec(prec) && (dagger == 0 || dagger == 1), "dwf_tune: bad precision or dagger");
    hipStream_t st = (hipStream_t)stream;
    const Geom &g = ctx->g;
    const size_t cb = cb_bytes(g, prec);
    void *in = nullptr, *out = nullptr, *ref = nullptr;
    unsigned *ndiff = nullptr;
    auto release = [&]() {
        (void)hipFree(in);
        (void)hipFree(out);
        (void)hipFree(ref);
        (void)hipFree(ndiff);
    };
    if (hipMalloc(&in, cb) != hipSuccess || hipMalloc(&out, cb) != hipSuccess || hipMalloc(&ref, cb) != hipSuccess ||
        hipMalloc((void **)&ndiff, sizeof(unsigned)) != hipSuccess) {
        release();
        return fail(DWF_ENOMEM, "dwf_tune: scratch allocation failed");
    }
    int rc = launch_fill_pattern(in, cb, prec, st);
    if (rc) {
        release();
        return rc;
    }
    // candidates: site kernel (workgroup sizes x XCD remap x store kind), row kernel (rows x tiles x remap x cap)
    std::vector<DhopShape> cand;
    for (int nt : {0, 1})
        for (int threads : {64, 128, 192, 256, 320, 384, 448, 512}) {
            if (threads % g.Ls) continue;
            for (int xcd : {0, 1}) {
                DhopShape s;
                s.spb = threads / g.Ls;
                s.xcd = xcd;
                s.nt_store = nt;
                cand.push_back(s);
            }
        }
    {
        const int per_row = (g.L[0] / 2) * g.Ls;
        const int tiles[][3] = {{1, 1, 1},     {4, 4, g.L[3]}, {8, 8, g.L[3]}, {4, 8, g.L[3]}, {8, 4, g.L[3]},
                                {4, 4, 8},     {g.L[1], 1, 1}, {2, 2, g.L[3]}, {2, 4, g.L[3]}};
        for (int rows = 1; rows * per_row <= kMaxDhopThreads; ++rows)
            for (const auto &tl : tiles)
                for (int xcd : {0, 1})
                    for (int occ : {0, 2, 3}) {
                        DhopShape s;
                        s.rows = rows;
                        s.ty = tl[0];
                        s.tz = tl[1];
                        s.tt = tl[2];
                        s.xcd = xcd;
                        s.nt_store = 1;
                        s.occ = occ;
                        if (row_shape_ok(g, s, prec, ctx->lds_limit)) cand.push_back(s);
                    }
    }
    if (cand.empty()) cand.push_back(default_shape(g));
    hipEvent_t e0, e1;
    DWF_HIP(hipEventCreate(&e0));
    DWF_HIP(hipEventCreate(&e1));
    const size_t rb = prec == DWF_F64 ? 8 : 4;  // bytes of the arithmetic type (M5op^-1 LDS exchange)
    // family 0: the plain hopping launch; family 1: the fused Schur pair (M5op^-1 epilogue into a
    // temporary, then the M5op epilogue), the shape the operators and the solvers use
    DhopShape best_s[2] = {cand[0], cand[0]};
    double best[2] = {1e30, 1e30};
    int status = DWF_OK;
    for (int family = 0; family < 2 && status == DWF_OK; ++family) {
        auto run = [&](const DhopShape &s, int parity) -> int {
            if (family == 0) {
                DhopCall c{in, out, nullptr, parity, dagger, EPI_SCALE, 1.0, 0.0, prec, prec};
                return launch_dhop(ctx, c, s, st);
            }
            DhopCall c1{in, ctx->tmp[0], nullptr, 0, dagger, EPI_M5INV, 1.0, 0.0, prec, prec};
            int r = launch_dhop(ctx, c1, s, st);
            if (r) return r;
            DhopCall c2{ctx->tmp[0], out, in, 1, dagger, EPI_M5, -0.25, 0.0, prec, prec};
            return launch_dhop(ctx, c2, s, st);
        };
        bool have_ref = false;
        for (const DhopShape &s : cand) {
            if (family == 1 && s.rows == 0 && (size_t)s.spb * g.Ls * 25 * rb > ctx->lds_limit) continue;
            // every shape must reproduce the first one's output bit for bit
            if ((rc = run(s, 1))) continue;
            if (!have_ref) {
                DWF_HIP(hipMemcpyAsync(ref, out, cb, hipMemcpyDeviceToDevice, st));
                have_ref = true;
            } else {
                DWF_HIP(hipMemsetAsync(ndiff, 0, sizeof(unsigned), st));
                if ((rc = launch_count_diff(out, ref, cb, ndiff, st))) {
                    status = rc;
                    break;
                }
                unsigned h = 0;
                DWF_HIP(hipMemcpyAsync(&h, ndiff, sizeof(unsigned), hipMemcpyDeviceToHost, st));
                DWF_HIP(hipStreamSynchronize(st));
                if (h != 0) {
                    status = fail(DWF_EHIP, "dwf_tune: a launch shape changed the result (" + std::to_string(h) +
                                                " vectors differ): rows=" + std::to_string(s.rows) +
                                                " spb=" + std::to_string(s.spb));
                    break;
                }
            }
            const int reps = 10;
            DWF_HIP(hipEventRecord(e0, st));
            for (int r = 0; r < reps; ++r) run(s, family == 0 ? (r & 1) : 1);
            DWF_HIP(hipEventRecord(e1, st));
            DWF_HIP(hipEventSynchronize(e1));
            float ms = 0;
            DWF_HIP(hipEventElapsedTime(&ms, e0, e1));
            const double us = 1000.0 * ms / reps;
            if (std::getenv("DWF_LOG"))
                std::fprintf(stderr,
                             "[dwf] tune %s prec=%d dagger=%d nt=%d spb=%d rows=%d tile=%dx%dx%d xcd=%d occ=%d: "
                             "%.2f us\n",
                             family ? "schur" : "dhop", prec, dagger, s.nt_store, s.spb, s.rows, s.ty, s.tz, s.tt,
                             s.xcd, s.occ, us);
            if (us < best[family]) {
                best[family] = us;
                best_s[family] = s;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    release();
    if (status != DWF_OK) return status;
    ctx->shape[prec][dagger] = best_s[0];
    ctx->shape_schur[prec][dagger] = best_s[1];
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        g_tune[tune_key(ctx->g, prec, dagger, 0)] = best_s[0];
        g_tune[tune_key(ctx->g, prec, dagger, 1)] = best_s[1];
        if (const char *path = std::getenv("DWF_TUNE_CACHE")) {
            std::ofstream f(path, std::ios::trunc);
            for (auto &kv : g_tune)
                f << kv.first << ' ' << kv.second.spb << ' ' << kv.second.xcd << ' ' << kv.second.nt_store << ' '
                  << kv.second.rows << ' ' << kv.second.ty << ' ' << kv.second.tz << ' ' << kv.second.tt << ' '
                  << kv.second.occ << '\n';
        }
    }
    if (best_us) *best_us = best[0];
    return DWF_OK;
}

}  // extern "C"
