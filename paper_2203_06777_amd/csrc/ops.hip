// Operators composed from the fused hopping kernels.
//
// Schur complement on the odd checkerboard, M_pc = M5op - 1/4 D_h^{o<-e} M5op^-1 D_h^{e<-o}:
//   t   = M5op^-1 (D_h^{e<-o} in)            one kernel (M5op^-1 fused as an LDS epilogue)
//   out = M5op in - 1/4 D_h^{o<-e} t          one kernel (M5op of the input fused)
// and the adjoint with every factor daggered.  M_pc^dag M_pc is four kernels.
#include "dwf_common.h"

namespace dwf {

static int two_step(dwf_ctx ctx, void *out, int prec_out, const void *in, void *t_e, int dagger, int prec,
                    hipStream_t st, double *norm_out = nullptr, long *nparts = nullptr) {
    const DhopShape &sh = ctx->shape_schur[prec][dagger];
    DhopCall c1{in, t_e, nullptr, 0, dagger, EPI_M5INV, 1.0, 0.0, prec, prec};
    int rc = launch_dhop(ctx, c1, sh, st);
    if (rc) return rc;
    DhopCall c2{t_e, out, in, 1, dagger, EPI_M5, -0.25, 0.0, prec, prec_out, norm_out, nparts};
    return launch_dhop(ctx, c2, sh, st);
}

// With norm_out set, the workgroups of the second kernel also write partial sums
// of |M_pc in|^2 (count in *nparts).
int op_mpc(dwf_ctx ctx, void *out, const void *in, int dagger, int prec, hipStream_t st, double *norm_out,
           long *nparts) {
    return two_step(ctx, out, prec, in, ctx->tmp[0], dagger, prec, st, norm_out, nparts);
}

int op_mdagm(dwf_ctx ctx, void *out, const void *in, int prec, void *tmp_o, hipStream_t st) {
    int rc = two_step(ctx, tmp_o, prec, in, ctx->tmp[0], 0, prec, st);
    if (rc) return rc;
    return two_step(ctx, out, prec, tmp_o, ctx->tmp[0], 1, prec, st);
}

// One CG step on M_pc^dag M_pc with y = M_pc p already computed: the adjoint
// Schur complement of y is never stored, the second kernel's epilogue applies
// r -= alpha M_pc^dag y to r (prec_r) and writes partials of the new |r|^2.
int op_mpcdag_cg(dwf_ctx ctx, void *r, int prec_r, const void *y, int prec, const double *cg_alpha,
                 const double *cg_live, double *partials, long *nparts, hipStream_t st) {
    const DhopShape &sh = ctx->shape_schur[prec][1];
    DhopCall c1{y, ctx->tmp[0], nullptr, 0, 1, EPI_M5INV, 1.0, 0.0, prec, prec};
    int rc = launch_dhop(ctx, c1, sh, st);
    if (rc) return rc;
    DhopCall c2{ctx->tmp[0], r, y, 1, 1, EPI_CG, -0.25, 0.0, prec, prec_r, partials, nparts, cg_alpha, cg_live};
    return launch_dhop(ctx, c2, sh, st);
}

}  // namespace dwf
