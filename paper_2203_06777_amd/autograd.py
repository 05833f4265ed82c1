"""torch.autograd Functions over the C ABI.

DwfOp:      y = D_DW(U) x on full 5D fields.  Backward: grad_x = D_DW^dag grad_y
            (dwf_dw with dagger) and grad_U = -1/2 eta (M^dag + N) from the force
            kernel with (X, Y) = (x, grad_y), since dD_DW = -dD_h / 2.
DwfAction:  S(U, phi) = phi^dag (D_DW^dag D_DW)^-1 phi.  Forward solves D^dag Z = phi
            and D X = Z (so Y = D X = Z and S = |Z|^2); backward gives
            grad_phi = 2 X and grad_U = eta (M^dag + N)(X, Y), because
            dS = -2 Re(Y^dag dD X) = Re(Y^dag dD_h X).

Tensors are canonical complex128 CUDA tensors: U [Lt,Lz,Ly,Lx,4,3,3], fields
[Lt,Lz,Ly,Lx,Ls,4,3].  Gradients follow torch's convention for complex inputs
(delta L = Re sum conj(grad) delta z).  All arithmetic runs in libdwf.so.
"""

from __future__ import annotations

import torch

from . import dwf as D


def _shamir_only(op: D.Context):
    # the link gradient below differentiates D_h X; a Moebius operator hops (b + cK) X
    if op.mobius:
        raise NotImplementedError("autograd: the link gradient is implemented for the Shamir operator only")


class DwfOp(torch.autograd.Function):
    @staticmethod
    def forward(ctx, op: D.Context, U: torch.Tensor, x: torch.Tensor):
        _shamir_only(op)
        U = U.detach().to(torch.complex128).contiguous()
        op.set_gauge(U)
        xi = op.pack(x.detach(), 2, "f64")
        yi = op.field("f64", full=True)
        D.dwf_dw(op.handle, yi, xi, 0, "f64")
        ctx.op = op
        ctx.save_for_backward(U, xi)
        return op.unpack(yi, 2, "f64")

    @staticmethod
    def backward(ctx, gy):
        op = ctx.op
        U, xi = ctx.saved_tensors
        op.set_gauge(U)
        gi = op.pack(gy.contiguous(), 2, "f64")
        grad_x = grad_u = None
        if ctx.needs_input_grad[2]:
            gx = op.field("f64", full=True)
            D.dwf_dw(op.handle, gx, gi, 1, "f64")
            grad_x = op.unpack(gx, 2, "f64")
        if ctx.needs_input_grad[1]:
            grad_u = torch.empty_like(U)
            D.dwf_force(op.handle, grad_u, xi, gi, 0, -0.5)
        return None, grad_u, grad_x


class DwfAction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, op: D.Context, U: torch.Tensor, phi: torch.Tensor, tol: float = 1e-12, maxit: int = 100000,
                mode: int = 0):
        _shamir_only(op)
        U = U.detach().to(torch.complex128).contiguous()
        op.set_gauge(U)
        pi = op.pack(phi.detach(), 2, "f64")
        z = op.field("f64", full=True)
        x = op.field("f64", full=True)
        D.dwf_solve(op.handle, z, pi, 1, tol, maxit, mode)
        D.dwf_solve(op.handle, x, z, 0, tol, maxit, mode)
        s = D.dwf_norm2(op.handle, z, 1, "f64")
        ctx.op = op
        ctx.save_for_backward(U, x, z)
        return torch.tensor(s, dtype=torch.float64, device=phi.device)

    @staticmethod
    def backward(ctx, gs):
        op = ctx.op
        U, x, z = ctx.saved_tensors
        g = float(gs.item())
        grad_u = grad_phi = None
        if ctx.needs_input_grad[1]:
            op.set_gauge(U)
            grad_u = torch.empty_like(U)
            D.dwf_force(op.handle, grad_u, x, z, 0, g)
        if ctx.needs_input_grad[2]:
            gp = op.zeros("f64", full=True)
            D.dwf_axpy(op.handle, gp, 2.0 * g, x, 1, "f64")
            grad_phi = op.unpack(gp, 2, "f64")
        return None, grad_u, grad_phi, None, None, None


def dwf_op(op: D.Context, U: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    return DwfOp.apply(op, U, x)


def dwf_action(op: D.Context, U: torch.Tensor, phi: torch.Tensor, tol: float = 1e-12) -> torch.Tensor:
    return DwfAction.apply(op, U, phi, tol)
