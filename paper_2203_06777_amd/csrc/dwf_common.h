// Internal declarations shared by the HIP translation units of libdwf.so.
//
// Internal field layout ("Ls-innermost"): a checkerboard field of precision P
// stores, for checkerboard row c, component group g and fifth coordinate s, one
// 16-byte vector of G(P) complex numbers:
//
//     offset16(c, g, s) = (c * NG + g) * Ls + s,      NG = 12 / G
//
// with complex component k = g*G + j = spin*3 + colour.  G = 1 (FP64), 2 (FP32),
// 4 (FP16/BF16), so every load and store is a 16-byte vector, and the Ls lanes
// that share a 4D site read Ls consecutive vectors: one wave reads whole
// contiguous 16*Ls-byte segments, and the site's links are fetched once and
// broadcast to all its s lanes.  A full field is the even checkerboard followed
// by the odd one.
//
// Gathered links: for output parity p and row c, 8 colour matrices
// [c][dir][3][3] (complex, storage precision): dir = mu (0..3) holds
// eta_mu(x) U_mu(x), dir = 4 + mu holds (eta_mu(x-mu) U_mu(x-mu))^dag, so the
// hopping kernel multiplies every direction by a plain matrix.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/dwf.h"

namespace dwf {

constexpr int kMaxLs = 64;

// --------------------------------------------------------------------------
// Precision traits
// --------------------------------------------------------------------------
template <int P> struct PT;
template <> struct PT<DWF_F64> { using A = double; static constexpr int G = 1; static constexpr int RB = 8; };
template <> struct PT<DWF_F32> { using A = float;  static constexpr int G = 2; static constexpr int RB = 4; };
template <> struct PT<DWF_F16> { using A = float;  static constexpr int G = 4; static constexpr int RB = 2; };
template <> struct PT<DWF_BF16> { using A = float; static constexpr int G = 4; static constexpr int RB = 2; };

inline int real_bytes(int prec) { return prec == DWF_F64 ? 8 : prec == DWF_F32 ? 4 : 2; }

struct Geom {
    int L[4];
    int Ls;
    long vol;   // 4D volume
    long half;  // vol / 2
    double M5, mf;
    int antiperiodic;
    // Moebius (Cayley) coefficients: D = D_W(-M5) (b + c K) + 1 - K with the
    // fifth-dimension hop K; mobius == 0 means b = 1, c = 0 (Shamir).
    double b5 = 1.0, c5 = 0.0;
    int mobius = 0;
};

// Site-local part Mooee = d - e K (Shamir: d = 5 - M5, e = 1).
inline double mooee_d(const Geom &g) { return g.mobius ? g.b5 * (4.0 - g.M5) + 1.0 : 5.0 - g.M5; }
inline double mooee_e(const Geom &g) { return g.mobius ? 1.0 - g.c5 * (4.0 - g.M5) : 1.0; }

// Bytes of one internal checkerboard field.
inline size_t cb_bytes(const Geom &g, int prec) { return (size_t)g.half * g.Ls * 24 * real_bytes(prec); }
inline size_t link_bytes(const Geom &g, int prec) { return (size_t)g.half * 8 * 18 * real_bytes(prec); }

// Launch shape of the hopping kernel.
struct DhopShape {
    int spb = 0;        // site kernel: 4D sites per workgroup (workgroup = spb * Ls lanes)
    int xcd = 1;        // XCD-aware block remap on/off
    int nt_store = 1;   // non-temporal stores of the output (it is not re-read by this launch)
    int rows = 0;       // > 0: row kernel with this many whole x-rows per workgroup (links and the
                        //      x-neighbour rows staged in LDS); 0: site kernel
    int ty = 1, tz = 1, tt = 1;  // row kernel: (y, z, t) tile of the row traversal order
    int occ = 0;        // row kernel: > 0 caps the workgroups resident on one CU at occ (by
                        //      padding the LDS request), which bounds the rows in flight per L2
};

constexpr int kMaxDhopThreads = 512;

// Epilogue modes of the hopping kernel (out is at the output parity):
enum Epi {
    EPI_SCALE = 0,  // out = alpha * D psi
    EPI_AXPY = 1,   // out = beta * z + alpha * D psi
    EPI_M5 = 2,     // out = Mooee(z) + alpha * D psi   (Mooee^dag when dagger; Mooee = M5op for Shamir)
    EPI_M5INV = 3,  // out = Mooee^-1 (beta * z + alpha * D psi)   (Mooee^-dag when dagger; z optional);
                    // with DhopCall::schur_coef the Schur factor Mooee^-1 (b + c K) instead
    EPI_CG = 4,     // CG step: y = M5op(z) + alpha * D psi is A p; out (= r, FP32 or FP64, read and
                    // written) -= (*cg_alpha) * y when *cg_live != 0, with |r|^2 partials in norm_out
    EPI_INTERIOR = 5,  // as EPI_SCALE, for the interior of a decomposed apply: output sites with a hop
                       // across a cut (DhopCall::dd_cut) are not written (same input and output precision)
    EPI_EXTERIOR = 6,  // as EPI_SCALE over the rows listed in DhopCall::row_list (row kernel only): a hop
                       // across a cut takes its half spinor from the received faces (DhopCall::recv)
    EPI_INTERIOR_ROWS = 7,  // as EPI_INTERIOR when the boundary is whole rows (x not cut) and a workgroup
                            // holds one row (row kernel only): a workgroup on a cut leaves, the others
                            // store every site (no per-site test before the stores)
};

struct DhopCall {
    const void *in;
    void *out;
    const void *z;  // field at the output parity for the epilogues (may be null for EPI_M5INV)
    int out_parity;
    int dagger;
    int epi;
    double alpha, beta;
    int prec_in, prec_out;  // links use prec_in
    double *norm_out = nullptr;  // EPI_M5, EPI_CG: per-workgroup partial sums of |out|^2 (FP64, fixed order)
    long *nparts_out = nullptr;  // receives the number of partials written
    const double *cg_alpha = nullptr, *cg_live = nullptr;  // EPI_CG: device scalars of the solver
    bool schur_coef = false;     // EPI_M5INV: apply Mooee^-1 (b + c K) (identical to Mooee^-1 for Shamir)
    const void *links = nullptr; // gathered link table to use instead of the context's (same layout)
    unsigned dd_cut = 0;         // EPI_INTERIOR: cut directions, bit mu (x = 1, y = 2, z = 4, t = 8)
    const double *stop = nullptr;  // device flag: when nonzero at launch the kernel does nothing
    const unsigned *row_list = nullptr;  // EPI_EXTERIOR: rows (y + L1 (z + L2 t)) to compute, nrows_list of them
    long nrows_list = 0;
    const void *recv = nullptr;          // EPI_EXTERIOR, 16-bit storage: received faces, segment 2 mu + side from seg_off[]
    const void *ghost = nullptr;         // EPI_EXTERIOR, FP32 / FP64: received faces as field-layout sites
    const long *seg_off = nullptr;       //   (kDdSegs + 1 prefix sums of face sites)
};

// Solver workspace (allocated on first solve).
struct CgWork {
    size_t bytes = 0;
    void *x64 = nullptr, *r64 = nullptr, *p64 = nullptr, *ap64 = nullptr;
    void *e32 = nullptr, *r32 = nullptr, *p32 = nullptr, *p16 = nullptr;
    void *full_tmp = nullptr;  // one full FP64 field for dwf_solve
};

}  // namespace dwf

struct dwf_ctx_s {
    dwf::Geom g;
    int device = 0;
    void *links[4][2] = {};  // [prec][output parity]
    bool gauge_set = false;
    void *tmp[3] = {};       // FP64-sized checkerboard temporaries for M_pc (tmp[2]: Moebius only)
    double *partials = nullptr;  // reduction partials (2 * kRedBlocks doubles)
    double *dhop_partials = nullptr;  // one FP64 partial per hopping-kernel workgroup (V/2 doubles)
    double *scal = nullptr;      // device scalars of the solvers
    double *host_scal = nullptr; // pinned host mirror (16 doubles)
    volatile double *host_flag = nullptr;  // mapped, coherent host memory: the CG stop flag
    double *host_flag_dev = nullptr;       // its device address
    void *events[2] = {};        // hipEvent_t pair for the solver's lagged stop check
    dwf::DhopShape shape[4][2];        // tuned launch shape per (prec, dagger): plain hopping launches
    dwf::DhopShape shape_schur[4][2];  // the same for the fused Schur kernels (M5op, M5op^-1, CG epilogues)
    size_t lds_limit = 65536;    // LDS bytes one workgroup may allocate on this device
    size_t lds_per_cu = 65536;   // LDS bytes of one compute unit
    double inner_tol = 0.0;
    int inner_maxit = 0;
    dwf::CgWork work;
};

namespace dwf {

constexpr int kRedBlocks = 1024;  // fixed reduction grid: results do not depend on timing
constexpr int kRedThreads = 256;

// Error reporting (thread-local message).
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
#define DWF_HIP(call)                                            \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return ::dwf::hip_fail(e_, #call); \
    } while (0)

// Layout kernels (layout.hip).
int launch_pack(const Geom &g, void *internal, const double *canonical, int parity, int prec, hipStream_t st);
int launch_unpack(const Geom &g, double *canonical, const void *internal, int parity, int prec, hipStream_t st);
int launch_gather_links(const Geom &g, void *links, const double *U, int out_parity, int prec, hipStream_t st);
int launch_convert(const Geom &g, void *out, int out_prec, const void *in, int in_prec, long ncb, hipStream_t st);

// Hopping kernel with epilogues (dhop.hip).
int launch_dhop(dwf_ctx ctx, const DhopCall &c, const DhopShape &shape, hipStream_t st);
DhopShape default_shape(const Geom &g);
DhopShape default_row_shape(const Geom &g, int prec, size_t lds_limit);
size_t row_lds_bytes(int rows, int L0h, int Ls, int prec);
bool row_shape_ok(const Geom &g, const DhopShape &sh, int prec, size_t lds_limit);
// M5op family on ncb checkerboard fields (m5.hip).
int launch_m5(const Geom &g, void *out, const void *in, int dagger, int inverse, long nsites, int prec,
              hipStream_t st);
// out = (d x + db z) - K (e x + eb z)  (K^dag when dagger; z optional, out may alias z).
int launch_m5_op(const Geom &g, void *out, const void *x, double d, double e, const void *z, double db, double eb,
                 int dagger, long nsites, int prec, hipStream_t st);

// BLAS-1 and reductions (blas.hip). n = number of complex elements.
int launch_reduce(double *partials, double *dst, const void *x, const void *y, long n, int prec, int dot,
                  hipStream_t st);
int launch_axpy(void *y, double ar, double ai, const void *x, long n, int prec, hipStream_t st);
// r = b - ap (FP64 fields of n complex numbers) and |r|^2 into dst[0], in launch_reduce's order.
int launch_residual64(double *partials, double *dst, void *r, const void *b, const void *ap, long n, hipStream_t st);
int launch_fill_pattern(void *f, size_t bytes, int prec, hipStream_t st);
int launch_count_diff(const void *a, const void *b, size_t bytes, unsigned *count, hipStream_t st);

// Operators composed from kernels (ops.hip).
int op_mpc(dwf_ctx ctx, void *out, const void *in, int dagger, int prec, hipStream_t st, double *norm_out = nullptr,
           long *nparts = nullptr, const double *stop = nullptr);
int op_mdagm(dwf_ctx ctx, void *out, const void *in, int prec, void *tmp_o, hipStream_t st);
int op_mpcdag_cg(dwf_ctx ctx, void *r, int prec_r, const void *y, int prec, const double *cg_alpha,
                 const double *cg_live, double *partials, long *nparts, hipStream_t st, const double *stop = nullptr);

// Static reduction scratch of the no-allocation entry point (noalloc.hip): resolves its
// device address on `device`, which must be current; once per device, thread-safe.
int noalloc_setup(int device);

// Solvers (solver.hip).
// r (prec_r) -= (*cg_alpha) w (prec_w) when *cg_live != 0, with |r|^2 partials (count in *nparts).
int launch_cg_residual(dwf_ctx ctx, void *r, int prec_r, const void *w, int prec_w, const double *cg_alpha,
                       const double *cg_live, double *partials, long *nparts, hipStream_t st);
int cg_solve(dwf_ctx ctx, void *x, const void *b, double tol, int maxit, int mode, dwf_cg_stats *stats,
             hipStream_t st);

// HMC link update U <- exp(i eps P) U on canonical gauge fields (hmc.hip).
int launch_expi_links(const Geom &g, double *U, const double *P, double eps, hipStream_t st);

// Force (force.hip).
int launch_force(dwf_ctx ctx, double *F, const void *X, const void *Y, int kind, double scale, hipStream_t st);

}  // namespace dwf
