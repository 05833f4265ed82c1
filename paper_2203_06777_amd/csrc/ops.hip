// Operators composed from the fused hopping kernels.
//
// Schur complement on the odd checkerboard, M_pc = M5op - 1/4 D_h^{o<-e} M5op^-1 D_h^{e<-o}:
//   t   = M5op^-1 (D_h^{e<-o} in)            one kernel (M5op^-1 fused as an LDS epilogue)
//   out = M5op in - 1/4 D_h^{o<-e} t          one kernel (M5op of the input fused)
// and the adjoint with every factor daggered.  M_pc^dag M_pc is four kernels.
//
// Moebius (Cayley) operator, D = Mooee - 1/2 D_h (b + c K) with Mooee = d - e K:
//   M_pc     = Mooee     - 1/4 D_h^{o<-e} [Mooee^-1 (b + cK)] D_h^{e<-o} (b + cK)
//   M_pc^dag = Mooee^dag - 1/4 (b + cK^dag) D_h^dag{o<-e} [Mooee^-dag (b + cK^dag)] D_h^dag{e<-o}
// The bracket is one fused epilogue (its coefficients differ from Mooee^-1 only);
// the factor (b + c K) before the first hop, and (b + c K^dag) after the last
// hop of the adjoint, are site-local kernels: three launches per M_pc.
#include "dwf_common.h"

namespace dwf {

static int two_step(dwf_ctx ctx, void *out, int prec_out, const void *in, void *t_e, int dagger, int prec,
                    hipStream_t st, double *norm_out = nullptr, long *nparts = nullptr,
                    const double *stop = nullptr) {
    const Geom &g = ctx->g;
    const DhopShape &sh = ctx->shape_schur[prec][dagger];
    if (!g.mobius) {
        DhopCall c1{in, t_e, nullptr, 0, dagger, EPI_M5INV, 1.0, 0.0, prec, prec};
        c1.stop = stop;
        int rc = launch_dhop(ctx, c1, sh, st);
        if (rc) return rc;
        DhopCall c2{t_e, out, in, 1, dagger, EPI_M5, -0.25, 0.0, prec, prec_out, norm_out, nparts};
        c2.stop = stop;
        return launch_dhop(ctx, c2, sh, st);
    }
    if (prec_out != prec) return fail(DWF_EUNSUP, "Moebius M_pc: output precision must equal the operator's");
    void *u = ctx->tmp[2];
    int rc;
    if (!dagger) {
        // u = (b + cK) in;  t = [Mooee^-1 (b + cK)] D^{e<-o} u;  out = Mooee in - 1/4 D^{o<-e} t
        if ((rc = launch_m5_op(g, u, in, g.b5, -g.c5, nullptr, 0.0, 0.0, 0, g.half, prec, st))) return rc;
        DhopCall c1{u, t_e, nullptr, 0, 0, EPI_M5INV, 1.0, 0.0, prec, prec};
        c1.schur_coef = true;
        c1.stop = stop;
        if ((rc = launch_dhop(ctx, c1, sh, st))) return rc;
        DhopCall c2{t_e, out, in, 1, 0, EPI_M5, -0.25, 0.0, prec, prec_out, norm_out, nparts};
        c2.stop = stop;
        return launch_dhop(ctx, c2, sh, st);
    }
    if (norm_out) return fail(DWF_EUNSUP, "Moebius M_pc^dag: no fused norm");
    // t = [Mooee^-dag (b + cK^dag)] D^dag{e<-o} in;  u = -1/4 D^dag{o<-e} t;
    // out = Mooee^dag in + (b + cK^dag) u
    DhopCall c1{in, t_e, nullptr, 0, 1, EPI_M5INV, 1.0, 0.0, prec, prec};
    c1.schur_coef = true;
    c1.stop = stop;
    if ((rc = launch_dhop(ctx, c1, sh, st))) return rc;
    DhopCall c2{t_e, u, nullptr, 1, 1, EPI_SCALE, -0.25, 0.0, prec, prec};
    c2.stop = stop;
    if ((rc = launch_dhop(ctx, c2, ctx->shape[prec][1], st))) return rc;
    return launch_m5_op(g, out, in, mooee_d(g), mooee_e(g), u, g.b5, -g.c5, 1, g.half, prec, st);
}

// With norm_out set, the workgroups of the second kernel also write partial sums
// of |M_pc in|^2 (count in *nparts).  With stop set, the hopping kernels do nothing
// when *stop is nonzero at their launch.
int op_mpc(dwf_ctx ctx, void *out, const void *in, int dagger, int prec, hipStream_t st, double *norm_out,
           long *nparts, const double *stop) {
    return two_step(ctx, out, prec, in, ctx->tmp[0], dagger, prec, st, norm_out, nparts, stop);
}

int op_mdagm(dwf_ctx ctx, void *out, const void *in, int prec, void *tmp_o, hipStream_t st) {
    int rc = two_step(ctx, tmp_o, prec, in, ctx->tmp[0], 0, prec, st);
    if (rc) return rc;
    return two_step(ctx, out, prec, tmp_o, ctx->tmp[0], 1, prec, st);
}

// One CG step on M_pc^dag M_pc with y = M_pc p already computed: the adjoint
// Schur complement of y is never stored, the second kernel's epilogue applies
// r -= alpha M_pc^dag y to r (prec_r) and writes partials of the new |r|^2.
// Moebius: M_pc^dag y is formed in ctx->tmp[2] and a streaming kernel updates r.
int op_mpcdag_cg(dwf_ctx ctx, void *r, int prec_r, const void *y, int prec, const double *cg_alpha,
                 const double *cg_live, double *partials, long *nparts, hipStream_t st, const double *stop) {
    const DhopShape &sh = ctx->shape_schur[prec][1];
    if (ctx->g.mobius) {
        int rc = two_step(ctx, ctx->tmp[2], prec, y, ctx->tmp[0], 1, prec, st, nullptr, nullptr, stop);
        if (rc) return rc;
        return launch_cg_residual(ctx, r, prec_r, ctx->tmp[2], prec, cg_alpha, cg_live, partials, nparts, st);
    }
    DhopCall c1{y, ctx->tmp[0], nullptr, 0, 1, EPI_M5INV, 1.0, 0.0, prec, prec};
    c1.stop = stop;
    int rc = launch_dhop(ctx, c1, sh, st);
    if (rc) return rc;
    DhopCall c2{ctx->tmp[0], r, y, 1, 1, EPI_CG, -0.25, 0.0, prec, prec_r, partials, nparts, cg_alpha, cg_live};
    return launch_dhop(ctx, c2, sh, st);
}

}  // namespace dwf
