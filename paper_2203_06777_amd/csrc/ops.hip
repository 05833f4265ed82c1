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
    const DhopShape &sh = ctx->shape[prec][dagger];
    DhopCall c1{in, t_e, nullptr, 0, dagger, EPI_M5INV, 1.0, 0.0, prec, prec};
    int rc = launch_dhop(ctx, c1, sh, st);
    if (rc) return rc;
    DhopCall c2{t_e, out, in, 1, dagger, EPI_M5, -0.25, 0.0, prec, prec_out, norm_out, nparts};
    return launch_dhop(ctx, c2, sh, st);
}

int op_mpc(dwf_ctx ctx, void *out, const void *in, int dagger, int prec, hipStream_t st) {
    return two_step(ctx, out, prec, in, ctx->tmp[0], dagger, prec, st);
}

// With mp_norm set, the workgroups of the M_pc kernel also write partial sums of
// |M_pc in|^2 = <in, M_pc^dag M_pc in> (count in *nparts) for the solver.
int op_mdagm(dwf_ctx ctx, void *out, const void *in, int prec, void *tmp_o, hipStream_t st, double *mp_norm,
             long *nparts) {
    int rc = two_step(ctx, tmp_o, prec, in, ctx->tmp[0], 0, prec, st, mp_norm, nparts);
    if (rc) return rc;
    return two_step(ctx, out, prec, tmp_o, ctx->tmp[0], 1, prec, st);
}

// M_pc^dag M_pc with 16-bit (or FP32) intermediate fields and the final output
// written in prec_out (FP32 for the inner solver's A p).
int op_mdagm_mixed(dwf_ctx ctx, void *out, int prec_out, const void *in, int prec, hipStream_t st, double *mp_norm,
                   long *nparts) {
    int rc = two_step(ctx, ctx->tmp[1], prec, in, ctx->tmp[0], 0, prec, st, mp_norm, nparts);
    if (rc) return rc;
    return two_step(ctx, out, prec_out, ctx->tmp[1], ctx->tmp[0], 1, prec, st);
}

}  // namespace dwf
