"""Hybrid Monte Carlo with the domain-wall pseudofermion action on one GPU.

The molecular dynamics of S(U) = phi^dag (D^dag D)^-1 phi with momenta P
(traceless Hermitian, P = sum_a omega_a lambda_a / 2 with omega ~ N(0, 1), so
their Gaussian weight is exp(-sum tr P^2)):

    H = sum_links tr(P^2) + S(U),   dU/dtau = i P U,   dP/dtau = -K(U) / 2,

where K is the su(3) force of dwf_force (kind 1): under U -> exp(i eps Q) U
the action changes by eps sum tr(Q K).  A leapfrog trajectory takes a half
step of P, alternating full steps of U and P, and a closing half step of P;
it is reversible and conserves H up to O(eps^2) over a fixed trajectory length.

Every step runs in the library: two solves per force (dwf_solve with D^dag,
then with D), dwf_force, dwf_expi_links, dwf_gauge_axpy and dwf_gauge_norm2.
The fields U, P, phi are canonical complex128 tensors on the GPU; random
numbers (the pseudofermion noise, the momenta, the Metropolis uniform) are
passed in by the caller.  This module is not part of the paper, which treats
the operator only; it is the step that consumes the force kernel.
"""

from __future__ import annotations

import math

import torch

from . import dwf as D


def _shamir_only(op: D.Context):
    if op.mobius:
        raise NotImplementedError("hmc: the force is implemented for the Shamir operator only")


def pseudofermion(op: D.Context, U: torch.Tensor, eta: torch.Tensor) -> torch.Tensor:
    """phi = D^dag eta for Gaussian noise eta (full 5D canonical field): then phi has
    weight exp(-S(U)) at this U."""
    _shamir_only(op)
    op.set_gauge(U)
    ei = op.pack(eta, 2, "f64")
    pi = op.field("f64", full=True)
    D.dwf_dw(op.handle, pi, ei, 1, "f64")
    return op.unpack(pi, 2, "f64")


class _Work:
    """Internal fields reused over a trajectory."""

    def __init__(self, op: D.Context, phi: torch.Tensor):
        self.phi = op.pack(phi, 2, "f64")
        self.z = op.field("f64", full=True)
        self.x = op.field("f64", full=True)


def action_and_force(op: D.Context, U: torch.Tensor, w: _Work, K: torch.Tensor, tol: float, mode: int) -> float:
    """S(U) = |z|^2 with D^dag z = phi; K <- the su(3) force from X = D^-1 z = (D^dag D)^-1 phi
    and Y = D X = z."""
    op.set_gauge(U)
    D.dwf_solve(op.handle, w.z, w.phi, 1, tol, 100000, mode)
    D.dwf_solve(op.handle, w.x, w.z, 0, tol, 100000, mode)
    D.dwf_force(op.handle, K, w.x, w.z, 1, 1.0)
    return D.dwf_norm2(op.handle, w.z, 1, "f64")


def hamiltonian(op: D.Context, U: torch.Tensor, P: torch.Tensor, phi: torch.Tensor, tol: float = 1e-12,
                mode: int = 0) -> float:
    _shamir_only(op)
    w = _Work(op, phi)
    K = torch.empty_like(U)
    s = action_and_force(op, U, w, K, tol, mode)
    return D.dwf_gauge_norm2(op.handle, P) + s


def leapfrog(op: D.Context, U: torch.Tensor, P: torch.Tensor, phi: torch.Tensor, eps: float, nsteps: int,
             tol: float = 1e-12, mode: int = 0) -> float:
    """nsteps leapfrog steps, updating U and P in place.  Returns S at the final U."""
    _shamir_only(op)
    w = _Work(op, phi)
    K = torch.empty_like(U)
    action_and_force(op, U, w, K, tol, mode)
    D.dwf_gauge_axpy(op.handle, P, -0.25 * eps, K)
    s = 0.0
    for n in range(nsteps):
        D.dwf_expi_links(op.handle, U, P, eps)
        s = action_and_force(op, U, w, K, tol, mode)
        D.dwf_gauge_axpy(op.handle, P, -(0.5 * eps if n + 1 < nsteps else 0.25 * eps), K)
    return s


def trajectory(op: D.Context, U: torch.Tensor, P: torch.Tensor, phi: torch.Tensor, eps: float, nsteps: int,
               uniform: float, tol: float = 1e-12, mode: int = 0) -> dict:
    """One HMC trajectory from (U, P) with pseudofermion phi; accepts when
    uniform < exp(-(H_end - H_start)).  U is replaced by the end point if accepted
    and left bitwise unchanged otherwise; P is consumed."""
    _shamir_only(op)
    w = _Work(op, phi)
    K = torch.empty_like(U)
    h0 = D.dwf_gauge_norm2(op.handle, P) + action_and_force(op, U, w, K, tol, mode)
    U1 = U.clone()
    s1 = leapfrog(op, U1, P, phi, eps, nsteps, tol, mode)
    h1 = D.dwf_gauge_norm2(op.handle, P) + s1
    dh = h1 - h0
    accept = uniform < math.exp(-dh) if dh > 0 else True
    if accept:
        U.copy_(U1)
    op.set_gauge(U)
    return {"dH": dh, "accepted": bool(accept), "H0": h0, "H1": h1}
