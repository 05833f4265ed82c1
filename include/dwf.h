/*
 * dwf.h — C ABI of the MI355X domain-wall fermion operator library (libdwf.so).
 *
 * The library applies the 5D Shamir domain-wall Dirac operator, which the
 * paper names as the kernel that dominates its run time and that it profiles
 * against memory bandwidth (Introduction; Performance results, the profiler
 * figures of the main DWF kernel; Conclusion, the node-local Wilson matrix).
 * The paper does not write the operator down; the library implements the
 * standard definitions, with these conventions:
 *
 *   sites x = (x0,x1,x2,x3), extents dims = {Lx,Ly,Lz,Lt}, all even;
 *   lex(x) = x0 + Lx*(x1 + Ly*(x2 + Lz*x3)); parity(x) = (x0+x1+x2+x3) mod 2;
 *   checkerboard row c(x) = lex(x) >> 1 (0 <= c < V/2);
 *   gamma_mu = [[0, e_mu],[e_mu^dag, 0]] (chiral), e_0 = -i s1, e_1 = -i s2, e_2 = -i s3, e_3 = 1;
 *   D_h psi(x,s) = sum_mu (1-gamma_mu) eta_mu(x) U_mu(x) psi(x+mu,s)
 *                       + (1+gamma_mu) eta_mu(x-mu) U_mu(x-mu)^dag psi(x-mu,s),
 *     eta_3(x) = -1 on links leaving t = Lt-1 when antiperiodic_t, else +1;
 *     D_h^dag swaps (1-gamma) and (1+gamma);
 *   M5op psi(s) = (5-M5) psi(s) - P_- psi~(s+1) - P_+ psi~(s-1), psi~ wraps with -mf,
 *     P_+ keeps spins 0,1 and P_- spins 2,3;
 *   D_DW = M5op - D_h/2;  M_pc = M5op - 1/4 D_h^{o<-e} M5op^-1 D_h^{e<-o} on the odd checkerboard.
 *
 * Moebius (Cayley) form, after dwf_set_mobius(b, c) (not treated in the paper;
 * the standard Brower-Neff-Orginos operator, b = 1, c = 0 being Shamir):
 *   K psi(s) = P_- psi~(s+1) + P_+ psi~(s-1);  D_W = (4-M5) - D_h/2;
 *   D_DW = D_W (b + c K) + 1 - K = Mooee - D_h (b + c K) / 2,
 *   Mooee = [b (4-M5) + 1] - [1 - c (4-M5)] K, which replaces M5op in dwf_m5;
 *   M_pc = Mooee - 1/4 D_h^{o<-e} (b + cK) Mooee^-1 D_h^{e<-o} (b + cK).
 *
 * Canonical layouts (complex FP64, interleaved re,im, DEVICE memory owned by the caller):
 *   gauge        [Lt][Lz][Ly][Lx][4][3][3]      (U[..][mu][a][b], link x -> x+mu)
 *   full field   [Lt][Lz][Ly][Lx][Ls][4][3]
 *   cb field     [V/2][Ls][4][3]                 (row c(x) of one parity)
 *   force        [Lt][Lz][Ly][Lx][4][3][3]
 * Internal fields (the `void*` field arguments) are in the library's private
 * layout and precision; convert with dwf_pack / dwf_unpack, size them with
 * dwf_field_bytes.  A full internal field is the even checkerboard followed by
 * the odd one.  All pointers are device pointers unless marked host.
 *
 * Streams: `stream` is a hipStream_t (NULL = legacy default stream).  Every
 * call only enqueues work on it and returns, except dwf_cg, dwf_solve,
 * dwf_norm2, dwf_cdot and dwf_tune, which synchronise that stream.
 *
 * Errors: every call returns a dwf_status; on failure dwf_last_error()
 * returns a message for the calling thread.  No C++ exception crosses the ABI.
 * A failed call leaves its outputs unspecified and the context usable.
 *
 * Allocation: dwf_create allocates the link copies and the operator
 * temporaries; dwf_cg / dwf_solve allocate solver workspace on first use;
 * dwf_batch_plan allocates its descriptor tables; dwf_set_mobius allocates one
 * temporary on the first switch to a Moebius operator.  dwf_dhop, dwf_m5, dwf_mpc,
 * dwf_mdagm, dwf_dw, dwf_axpy and dwf_force never allocate.
 * A context may be used from one host thread at a time.
 */
#ifndef DWF_H
#define DWF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dwf_ctx_s *dwf_ctx;
typedef struct dwf_batch_s *dwf_batch;
typedef struct dwf_dd_s *dwf_dd;

/* Storage precision of an internal field.  F16 and BF16 store spinors and
 * links in 16 bits and compute in FP32. */
typedef enum { DWF_F64 = 0, DWF_F32 = 1, DWF_F16 = 2, DWF_BF16 = 3 } dwf_prec;

typedef enum {
    DWF_OK = 0,
    DWF_EINVAL = -1,  /* bad argument: odd/too small extents, Ls out of range, NULL pointer, bad enum */
    DWF_ENOMEM = -2,  /* device allocation failed */
    DWF_EHIP = -3,    /* a HIP runtime call failed; the message carries hipGetErrorString */
    DWF_ENOCONV = -4, /* solver hit maxit before tol; stats are filled and x holds the last iterate */
    DWF_ENAN = -5,    /* solver met a non-finite residual */
    DWF_EUNSUP = -6,  /* valid but unsupported combination (e.g. gauge not set yet) */
} dwf_status;

typedef struct {
    int dims[4];        /* Lx, Ly, Lz, Lt: even, >= 2 */
    int Ls;             /* fifth-dimension extent, 1 <= Ls <= 64 */
    double M5;          /* domain-wall height */
    double mf;          /* quark mass on the s wraps */
    int antiperiodic_t; /* 1: eta_3 = -1 on the time-boundary links */
} dwf_geom;

typedef struct {
    int outer_iters;       /* defect-correction restarts (1 for plain FP64 CG) */
    int inner_iters;       /* total CG iterations (all precisions) */
    double true_rel_resid; /* ||b - A x|| / ||b|| in FP64 at exit */
    double seconds;        /* host wall time of the call */
} dwf_cg_stats;

/* ---- context ------------------------------------------------------------ */

/* Validates geom, binds the current HIP device, allocates link storage for
 * all precisions and two FP64-sized checkerboard temporaries.
 * Paper: Introduction (the domain-wall operator as the case the data layout serves). */
int dwf_create(const dwf_geom *geom, dwf_ctx *out);
int dwf_destroy(dwf_ctx ctx);
const char *dwf_last_error(void);

/* Bytes of one internal checkerboard field (full = 0) or full 5D field (full = 1). */
int dwf_field_bytes(dwf_ctx ctx, int prec, int full, size_t *bytes);

/* Copies the canonical FP64 gauge field into the library's gathered link
 * tables (8 links per checkerboard site, backward links stored daggered,
 * eta folded in) in every precision.  U itself is not modified and may be
 * freed afterwards.  Any complex 3x3 matrices are accepted (not only SU(3)).
 * Paper: Acceleration abstraction (the layout the stencil kernels read). */
int dwf_set_gauge(dwf_ctx ctx, const double *U, void *stream);

/* Switches the context to the Moebius operator with real coefficients b, c
 * (b = 1, c = 0 switches back to Shamir; the default).  Afterwards dwf_m5
 * applies Mooee (and its adjoint and inverse), and dwf_mpc, dwf_mdagm, dwf_dw,
 * dwf_cg and dwf_solve the Moebius operators defined above; dwf_dhop, dwf_force
 * and the batch calls concern D_h only and do not change.  M_pc takes three
 * launches instead of two (the factor b + cK is a site-local kernel), and each
 * CG iteration a streaming residual update.  Returns DWF_EINVAL for non-finite
 * b, c or a singular Mooee.  The first switch to a Moebius operator allocates
 * one FP64 checkerboard temporary; the call synchronises the device. */
int dwf_set_mobius(dwf_ctx ctx, double b, double c);
/* The current coefficients (host pointers). */
int dwf_get_mobius(dwf_ctx ctx, double *b, double *c);

/* Canonical FP64 <-> internal field of precision prec.
 * parity 0 / 1: one checkerboard, canonical [V/2][Ls][4][3];
 * parity 2:     full field, canonical [Lt][Lz][Ly][Lx][Ls][4][3]. */
int dwf_pack(dwf_ctx ctx, void *internal, const double *canonical, int parity, int prec, void *stream);
int dwf_unpack(dwf_ctx ctx, double *canonical, const void *internal, int parity, int prec, void *stream);

/* Element-wise precision change of an internal field (round to nearest even). */
int dwf_convert(dwf_ctx ctx, void *out, int out_prec, const void *in, int in_prec, int full, void *stream);

/* ---- operators (checkerboard fields unless stated) ------------------------ */

/* out = D_h^{p<-1-p} in (dagger = 0) or (D_h^dag)^{p<-1-p} in (dagger = 1),
 * p = out_parity; the raw hopping term, no -1/2. in and out must not alias.
 * Paper: Performance results, the Nsight Compute figure ("main kernel DWF code",
 * bandwidth-bound), and the Conclusion's node-local Wilson matrix. */
int dwf_dhop(dwf_ctx ctx, void *out, const void *in, int out_parity, int dagger, int prec, void *stream);

/* out = M5op in, M5op^dag in, M5op^-1 in or M5op^-dag in (dagger, inverse in {0,1});
 * Mooee in place of M5op for a Moebius context;
 * full = 0: one checkerboard, full = 1: a full field.  in and out may alias.
 * Paper: Conclusion (all kernels of the DWF Dirac operator bandwidth-saturating). */
int dwf_m5(dwf_ctx ctx, void *out, const void *in, int dagger, int inverse, int full, int prec, void *stream);

/* out = M_pc in (dagger = 0) or M_pc^dag in (dagger = 1) on the odd checkerboard.
 * Paper: Conclusion (the kernels of the DWF Dirac operator). */
int dwf_mpc(dwf_ctx ctx, void *out, const void *in, int dagger, int prec, void *stream);

/* out = M_pc^dag M_pc in on the odd checkerboard: the normal operator CG applies.
 * Paper: Performance results, the Nsight Compute figure (the main DWF kernel sequence). */
int dwf_mdagm(dwf_ctx ctx, void *out, const void *in, int prec, void *stream);

/* out = D_DW in (dagger = 0) or D_DW^dag in (dagger = 1) on full fields.
 * Paper: Introduction (the domain-wall fermion operator). */
int dwf_dw(dwf_ctx ctx, void *out, const void *in, int dagger, int prec, void *stream);

/* ---- BLAS-1 and FP64 reductions (deterministic, fixed-order trees) -------- */

/* *result (host) = sum |x|^2 accumulated in FP64. Synchronises the stream.
 * Paper: Acceleration abstraction, Internal API (the reduction primitive a solver needs). */
int dwf_norm2(dwf_ctx ctx, double *result, const void *x, int full, int prec, void *stream);
/* result[0] + i result[1] (host) = <x, y> = sum conj(x) y in FP64. Synchronises. */
int dwf_cdot(dwf_ctx ctx, double *result, const void *x, const void *y, int full, int prec, void *stream);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): result[0] + i result[1] = <x, y> as
 * dwf_cdot computes it (y != NULL), or result[0] = |x|^2, result[1] = 0 as dwf_norm2 does
 * (y == NULL), bit for bit, written to caller-owned DEVICE memory (2 doubles).  Enqueued on
 * the stream; no synchronisation, no allocation, no memset (the call can be captured in a
 * graph).  The per-workgroup partial sums live in one static 16 KiB device array per GPU
 * (set up by dwf_create, held until the process ends) instead of the context's buffer, so
 * calls that overlap on one GPU (other streams or host threads) race on it and must be
 * ordered by the caller.  The array holds the partials of the fixed reduction grid for any
 * field size; a build whose grid did not fit would reject the call with DWF_EINVAL. */
int dwf_cdot_noalloc(dwf_ctx ctx, double *result, const void *x, const void *y, int full, int prec, void *stream);
/* y = (a_re + i a_im) x + y. */
int dwf_axpy(dwf_ctx ctx, void *y, double a_re, double a_im, const void *x, int full, int prec, void *stream);

/* ---- solvers --------------------------------------------------------------
 * The paper names no solver; CG on the Schur normal operator is what the DWF Dirac
 * operator it profiles is applied by (Performance results: the operator sequence). */

/* Solves M_pc^dag M_pc x = b on the odd checkerboard (FP64 internal fields),
 * starting from the x passed in, until ||b - A x|| / ||b|| <= tol (recomputed in FP64).
 * mode 0: FP64 CG.  mode 1/2/3: FP64 defect correction around inner CG whose
 * operator stores spinors and links in FP32 / FP16 / BF16 (FP32 vectors,
 * FP64 reductions); with FP32 the inner iteration keeps its search direction
 * across each FP64 residual refresh (reliable update), the 16-bit ones restart
 * from the refreshed residual.  maxit bounds the total CG iterations.  stats may
 * be NULL. */
int dwf_cg(dwf_ctx ctx, void *x, const void *b, double tol, int maxit, int mode, dwf_cg_stats *stats,
           void *stream);

/* Inner-solve controls of modes 1-3: relative residual reduction of each inner
 * solve (the last one stops where the outer tolerance needs) and its iteration cap
 * (<= 0 restores the defaults: 1e-4 for mode 1, 1e-2 for modes 2 and 3; 2000). */
int dwf_cg_set_inner(dwf_ctx ctx, double inner_tol, int inner_maxit);

/* Solves D_DW x = b (dagger = 0) or D_DW^dag x = b (dagger = 1) on full FP64
 * internal fields via the odd-checkerboard Schur complement and dwf_cg
 * (x is overwritten; b is not modified). */
int dwf_solve(dwf_ctx ctx, void *x, const void *b, int dagger, double tol, int maxit, int mode,
              dwf_cg_stats *stats, void *stream);

/* ---- fermion force ----------------------------------------------------------
 * Not in the paper: the derivative of the action with respect to the links, the
 * differentiable form beside the operator (its outer products are the DWF stencil's
 * transpose). */

/* From full FP64 internal fields X, Y, writes canonical FP64 F (complex
 * [V][4][3][3]):  M_mu(x) = sum_s tr_spin[(1-gamma_mu) X(x+mu,s) Y(x,s)^dag],
 * N_mu(x) = sum_s tr_spin[(1+gamma_mu) X(x,s) Y(x+mu,s)^dag];
 * kind 0: F = scale * eta (M^dag + N), the gradient of Re(Y^dag D_h X) with
 *         respect to U in the convention delta f = Re sum conj(F) delta U;
 * kind 1: F = scale * traceless part of (i/2)(G - G^dag), G = eta (U M - N U^dag),
 *         the su(3) force: d/d(eps) Re(Y^dag D_h X) under U -> exp(i eps Q) U
 *         equals sum tr(Q F) / scale.  kind 1 needs the gauge set. */
int dwf_force(dwf_ctx ctx, double *F, const void *X, const void *Y, int kind, double scale, void *stream);

/* ---- hybrid Monte Carlo molecular dynamics on gauge-shaped fields ---------------
 * (the step that consumes dwf_force; not treated in the paper).  U, P, X, Y are
 * canonical FP64 [Lt][Lz][Ly][Lx][4][3][3] device arrays owned by the caller. */

/* U <- exp(i eps P) U for every link, in place; P is meant to be traceless
 * Hermitian (an su(3) momentum), which is not checked.  exp by scaling and
 * squaring of a degree-14 Taylor polynomial (FP64 rounding level).
 * U and P must not alias. */
int dwf_expi_links(dwf_ctx ctx, double *U, const double *P, double eps, void *stream);
/* Y = a X + Y over the V*4*9 complex entries. */
int dwf_gauge_axpy(dwf_ctx ctx, double *Y, double a, const double *X, void *stream);
/* *result (host) = sum |X_ij|^2 in FP64, i.e. sum_links tr(P^2) for Hermitian P.
 * Synchronises the stream. */
int dwf_gauge_norm2(dwf_ctx ctx, double *result, const double *X, void *stream);

/* ---- domain-decomposed hopping term ------------------------------------------------
 * The communication pattern the paper's library runs between GPUs (its performance
 * section: face assembly and halo exchange overlapped with the interior computation, all
 * DWF kernels including face assembly near the memory-bandwidth peak), on one GPU whose
 * neighbour domain across every cut direction is itself.  A plan cuts a set of directions
 * (DWF_CUT_X | DWF_CUT_Y | DWF_CUT_Z | DWF_CUT_T; x, y and z is the 2x2x2x1 split over eight
 * GPUs).  An output site is on the boundary when a hop crosses a cut.  dwf_dd_dhop runs, on
 * a stream of the plan, one face kernel (the half spinors, 6 complex per site and s in the
 * arithmetic type, of the input slices x_mu = 0 and x_mu = L_mu - 1 of every cut mu, with the
 * projector of the hop that crosses), one device copy standing in for the peer transfers (FP32 /
 * FP64: into ghost sites of the field layout, the half spinor in the upper spin pair), and the
 * boundary sites computed from the received faces; meanwhile the caller's stream runs the
 * hopping kernel on the interior sites only.  FP32 / FP64 plans that cut x (every x-row then
 * holds a boundary site) compute every row from the received faces after the exchange and have
 * no interior launch.  The result equals dwf_dhop bit for bit. */
#define DWF_CUT_X 1
#define DWF_CUT_Y 2
#define DWF_CUT_Z 4
#define DWF_CUT_T 8

/* Plan for precision prec and the cut mask `cuts` (1..15): allocates the send face buffer
 * (sum over cut mu of V/(2 L_mu) x Ls x 12 reals) and the receive side (the same size; FP32 /
 * FP64: ghost sites of twice that size, cleared here), the boundary row and site lists and a
 * stream.  The plan reads the context's link tables at every apply (a gauge
 * change needs no new plan); the context must outlive the plan. */
int dwf_dd_create(dwf_ctx ctx, int prec, int cuts, dwf_dd *dd);
/* out = D_h^{p<-1-p} in (dagger: D_h^dag) through the decomposition; the caller's stream
 * orders it like dwf_dhop.  in and out must not alias. */
int dwf_dd_dhop(dwf_dd dd, void *out, const void *in, int out_parity, int dagger, void *stream);
/* Face assembly alone (every cut face of in for output parity out_parity, into the plan's
 * send buffer), on the caller's stream: its bandwidth measurement. */
int dwf_dd_faces(dwf_dd dd, const void *in, int out_parity, int dagger, void *stream);
int dwf_dd_destroy(dwf_dd dd);

/* ---- batched hopping term ----------------------------------------------------
 * Paper: Acceleration abstraction (one offloaded kernel over many sites; here over
 * many fields and lattices in one graph launch). */

/* A plan applies dwf_dhop (same out_parity, dagger and precision) to nrhs[i]
 * fields of each of nlat contexts (lattices may differ in volume and Ls) in
 * one kernel launch (one workgroup per (lattice, field, row block) item, each
 * lattice with its tuned launch shape).  The contexts must outlive the plan
 * and have their gauge set; a shape tuned after dwf_batch_plan is not seen.  dwf_batch_capture binds the field pointers (outs / ins list the
 * fields lattice by lattice, sum(nrhs) each) and records the launch into a
 * HIP graph on `stream`; dwf_batch_launch replays it. */
int dwf_batch_plan(const dwf_ctx *ctxs, int nlat, const int *nrhs, int prec, int dagger, dwf_batch *plan);
int dwf_batch_capture(dwf_batch plan, void *const *outs, const void *const *ins, int out_parity, void *stream);
int dwf_batch_launch(dwf_batch plan, void *stream);
int dwf_batch_free(dwf_batch plan);

/* ---- autotuning ---------------------------------------------------------------
 * Paper: Acceleration abstraction, Offload primitives and attributes (launch shape as a
 * per-kernel attribute). */

/* Times the launch shapes of the hopping kernel for (prec, dagger) on this
 * context's lattice and keeps the fastest, separately for plain dwf_dhop
 * launches and for the fused Schur-operator kernels (M5op^-1 and M5op
 * epilogues, as used by dwf_mpc, dwf_mdagm, dwf_cg and dwf_solve).  Every
 * candidate must reproduce the first one's output bit for bit (DWF_EHIP
 * otherwise).  The choices are cached in memory and, if the environment
 * variable DWF_TUNE_CACHE names a file, on disk.  *best_us (host, may be NULL)
 * receives the best plain time per apply.  Scratch fields are allocated and
 * freed inside; the context's temporaries are overwritten.  Synchronises the
 * stream. */
int dwf_tune(dwf_ctx ctx, int prec, int dagger, double *best_us, void *stream);

/* ---- software-managed device cache ------------------------------------------
 * Paper: Memory models and software managed cache (the MemoryManager: a table of
 * host buffers with their device copies, views opened with an access intent that
 * migrate whole buffers, a device-memory high watermark, least-recently-used
 * eviction and an "infrequently used" advice).
 *
 * A cache keeps device copies of HOST buffers (pinned memory from hipHostMalloc
 * gives the fastest copies; pageable memory works).  dwf_cache_open returns a view
 * of the buffer for one intent: the device address for DWF_ACC_READ / DWF_ACC_WRITE
 * (valid until the view is closed), the host address for DWF_CPU_READ /
 * DWF_CPU_WRITE.  It copies the whole buffer when the intent and the state ask for
 * it (DWF_ST_*):
 *   ACC_READ   Empty or CpuDirty: host -> device, then Consistent
 *   ACC_WRITE  Empty or CpuDirty: host -> device (a read-write view), then AccDirty
 *   CPU_READ   AccDirty: device -> host, then Consistent
 *   CPU_WRITE  AccDirty: device -> host; then CpuDirty if a device copy exists
 * A buffer is found by its host address; the first open registers it with its
 * size, later opens must give the same size.  Views nest (a count per buffer);
 * every open needs one dwf_cache_close.  The device bytes held (copies and freed
 * blocks kept for reuse) never exceed watermark_bytes: to make room, buffers with
 * no open view lose their device copy (written back first when AccDirty) in
 * least-recently-opened order, buffers advised DWF_ADVISE_INFREQUENT before all
 * others.  DWF_ENOMEM if every resident buffer has an open view.
 *
 * Copies are enqueued on `stream` (a hipStream_t); CPU intents, release, flush and
 * destroy synchronise it, so the host may use a CPU view at once.  Use one stream
 * per cache (or order the streams yourself); the host must not touch a registered
 * buffer outside a CPU view.  backend DWF_CACHE_DEVICE uses device memory of the
 * device current at dwf_cache_create; DWF_CACHE_HOST_SIM keeps the "device" copies
 * in host memory (memcpy, no GPU): the same policy, for testing.  A cache may be
 * used from one host thread at a time. */
typedef struct dwf_cache_s *dwf_cache;
enum { DWF_CPU_READ = 0, DWF_CPU_WRITE = 1, DWF_ACC_READ = 2, DWF_ACC_WRITE = 3 };
enum { DWF_ST_EMPTY = 0, DWF_ST_CPU_DIRTY = 1, DWF_ST_ACC_DIRTY = 2, DWF_ST_CONSISTENT = 3 };
enum { DWF_ADVISE_NORMAL = 0, DWF_ADVISE_INFREQUENT = 1 };
enum { DWF_CACHE_DEVICE = 0, DWF_CACHE_HOST_SIM = 1 };

typedef struct {
    size_t watermark;          /* bytes */
    size_t resident_bytes;     /* device copies of registered buffers */
    size_t held_bytes;         /* resident_bytes plus freed blocks kept for reuse */
    long long entries;         /* registered buffers */
    long long h2d_count, d2h_count, evictions;
    unsigned long long h2d_bytes, d2h_bytes;
} dwf_cache_stats;

int dwf_cache_create(size_t watermark_bytes, int backend, dwf_cache *out);
int dwf_cache_open(dwf_cache c, void *host, size_t bytes, int intent, void **view, void *stream);
int dwf_cache_close(dwf_cache c, void *host);
/* DWF_ADVISE_INFREQUENT: evicted before every normally advised buffer. */
int dwf_cache_advise(dwf_cache c, void *host, int advice);
/* Writes back (if AccDirty) and forgets a buffer with no open view. */
int dwf_cache_release(dwf_cache c, void *host, void *stream);
/* Writes back every AccDirty buffer (they become Consistent). */
int dwf_cache_flush(dwf_cache c, void *stream);
/* state: DWF_ST_*; refs: open views; resident: whether a device copy exists (each may be NULL). */
int dwf_cache_query(dwf_cache c, const void *host, int *state, int *refs, int *resident);
int dwf_cache_get_stats(dwf_cache c, dwf_cache_stats *out);
/* Writes back every AccDirty buffer and frees the device memory; no view may be open. */
int dwf_cache_destroy(dwf_cache c, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DWF_H */
