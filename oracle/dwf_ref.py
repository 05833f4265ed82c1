"""numpy FP64 reference of the Shamir domain-wall fermion operator (test infrastructure only).

The paper names the domain-wall fermion (DWF) Dirac operator, built on the
node-local Wilson hopping matrix, as the kernel that dominates its run time
and that it profiles against memory bandwidth (Introduction; Performance
results, Nsight figures; Conclusion).  It does not print the operator, so this
module writes out the standard definitions with these fixed conventions:

* sites x = (x0,x1,x2,x3) = (x,y,z,t); mu = 0..3; arrays are indexed [t,z,y,x].
* Euclidean chiral gamma basis: gamma_mu = [[0, e_mu],[e_mu^dag, 0]] over the
  spin pairs (0,1),(2,3) with e_0 = -i sigma_1, e_1 = -i sigma_2,
  e_2 = -i sigma_3, e_3 = 1; gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3.
* hopping term  (D_h psi)(x,s) = sum_mu [ (1-gamma_mu) eta_mu(x) U_mu(x) psi(x+mu,s)
                                        + (1+gamma_mu) eta_mu(x-mu) U_mu(x-mu)^dag psi(x-mu,s) ]
  with eta_3(x) = -1 on the links leaving the last time slice (antiperiodic
  time), +1 otherwise; D_h^dag swaps (1-gamma) and (1+gamma).
* Wilson  D_W(m) = (4+m) - D_h/2.
* Shamir fifth-dimension term (M5op psi)(s) = (5-M5) psi(s) - P_- psi~(s+1) - P_+ psi~(s-1),
  psi~(Ls) = -mf psi(0), psi~(-1) = -mf psi(Ls-1), P_+- = (1 +- gamma_5)/2.
* full operator D_DW = M5op - D_h/2; Schur complement on the odd checkerboard
  M_pc = M5op - (1/4) D_h^{o<-e} M5op^-1 D_h^{e<-o}.
* Moebius (Cayley) generalisation with real b, c (Brower, Neff and Orginos;
  the paper does not treat it): with the fifth-dimension hop
  (K psi)(s) = P_- psi~(s+1) + P_+ psi~(s-1) and D_W = D_W(-M5),
  D_mob psi(s) = (b D_W + 1) psi(s) + (c D_W - 1) (K psi)(s),
  i.e. D_mob = D_W (b + c K) + 1 - K.  b = 1, c = 0 is Shamir.  Its site-local
  part is Mooee = [b (4-M5) + 1] - [1 - c (4-M5)] K and its hopping part
  -D_h (b + c K) / 2, so M_pc = Mooee - (1/4) D_h^{o<-e} (b + cK) Mooee^-1 D_h^{e<-o} (b + cK).

Everything is complex128 and written for readability, not speed.
"""

from __future__ import annotations

import numpy as np

# ----------------------------------------------------------------------------
# Gamma matrices (explicit 4x4; the definition, not a projection trick)
# ----------------------------------------------------------------------------
_E = [
    np.array([[0, -1j], [-1j, 0]]),
    np.array([[0, -1], [1, 0]], dtype=np.complex128),
    np.array([[-1j, 0], [0, 1j]]),
    np.eye(2, dtype=np.complex128),
]


def _gamma(e):
    g = np.zeros((4, 4), dtype=np.complex128)
    g[0:2, 2:4] = e
    g[2:4, 0:2] = e.conj().T
    return g


GAMMA = [_gamma(e) for e in _E]
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ID4 = np.eye(4, dtype=np.complex128)
P_PLUS = (ID4 + GAMMA5) / 2
P_MINUS = (ID4 - GAMMA5) / 2


def axis_of(mu: int) -> int:
    """Array axis of direction mu in a [t,z,y,x,...] array."""
    return 3 - mu


# ----------------------------------------------------------------------------
# Geometry
# ----------------------------------------------------------------------------
def dims_of(arr) -> tuple:
    """(Lx, Ly, Lz, Lt) of a canonical [t,z,y,x,...] array."""
    lt, lz, ly, lx = arr.shape[:4]
    return (lx, ly, lz, lt)


def coords(dims):
    """Integer coordinate arrays x0..x3, each shaped (Lt, Lz, Ly, Lx)."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return x, y, z, t


def lex_index(dims):
    x, y, z, t = coords(dims)
    lx, ly, lz, _ = dims
    return x + lx * (y + ly * (z + lz * t))


def parity(dims):
    x, y, z, t = coords(dims)
    return (x + y + z + t) % 2


def eta(dims, antiperiodic_t: bool = True):
    """Boundary phases eta_mu(x), shape (Lt, Lz, Ly, Lx, 4)."""
    lx, ly, lz, lt = dims
    e = np.ones((lt, lz, ly, lx, 4))
    if antiperiodic_t:
        e[lt - 1, :, :, :, 3] = -1.0
    return e


def full_to_cb(psi_full, par: int):
    """Rows of the given parity in lex order, which is checkerboard order c = lex >> 1."""
    dims = dims_of(psi_full)
    v = int(np.prod(dims))
    mask = (parity(dims) == par).reshape(v)
    return psi_full.reshape((v,) + psi_full.shape[4:])[mask].copy()


def cb_to_full(psi_cb, par: int, dims, other=None):
    """Embed a checkerboard field into a full field (zeros, or `other`, on the other parity)."""
    v = int(np.prod(dims))
    lx, ly, lz, lt = dims
    tail = psi_cb.shape[1:]
    out = np.zeros((v,) + tail, dtype=np.complex128)
    mask = (parity(dims) == par).reshape(v)
    out[mask] = psi_cb
    if other is not None:
        out[~mask] = other
    return out.reshape((lt, lz, ly, lx) + tail)


# ----------------------------------------------------------------------------
# Hopping term D_h (4D Wilson hopping applied at every s)
# ----------------------------------------------------------------------------
def _spin(mat, psi):
    """Apply a 4x4 spin matrix to [..., 4, 3]."""
    return np.einsum("ij,...ja->...ia", mat, psi)


def dhop(U, psi, dagger: bool = False, antiperiodic_t: bool = True):
    """D_h (or D_h^dag) on a full field psi of shape (Lt,Lz,Ly,Lx,Ls,4,3)."""
    dims = dims_of(U)
    et = eta(dims, antiperiodic_t)
    out = np.zeros_like(psi)
    sgn = 1.0 if dagger else -1.0  # forward hop uses (1 + sgn*gamma_mu)
    for mu in range(4):
        ax = axis_of(mu)
        w = U[..., mu, :, :] * et[..., mu, None, None]  # eta_mu(x) U_mu(x)
        fwd = np.roll(psi, -1, axis=ax)  # psi(x + mu)
        t = np.einsum("tzyxab,tzyxsib->tzyxsia", w, fwd)
        out += _spin(ID4 + sgn * GAMMA[mu], t)
        wb = np.roll(w, 1, axis=ax)  # eta_mu(x-mu) U_mu(x-mu)
        bwd = np.roll(psi, 1, axis=ax)  # psi(x - mu)
        t = np.einsum("tzyxba,tzyxsib->tzyxsia", wb.conj(), bwd)  # U^dag: (U^dag)_ab = conj(U_ba)
        out += _spin(ID4 - sgn * GAMMA[mu], t)
    return out


def dhop_cb(U, psi_cb, out_parity: int, dagger: bool = False, antiperiodic_t: bool = True):
    """Checkerboarded D_h^{p<-1-p}: embed the input on parity 1-p, apply D_h, keep parity p."""
    dims = dims_of(U)
    full = cb_to_full(psi_cb, 1 - out_parity, dims)
    return full_to_cb(dhop(U, full, dagger, antiperiodic_t), out_parity)


def site_of_cb(dims, par: int, c):
    """Coordinates of checkerboard row(s) c of parity par (vectorised)."""
    lx, ly, lz, lt = dims
    c = np.asarray(c)
    xh = c % (lx // 2)
    rest = c // (lx // 2)
    x1 = rest % ly
    x2 = (rest // ly) % lz
    x3 = rest // (ly * lz)
    x0 = 2 * xh + ((par + x1 + x2 + x3) % 2)
    return x0, x1, x2, x3


def dhop_sites(U, psi_cb, out_parity: int, rows, dagger: bool = False, antiperiodic_t: bool = True):
    """D_h^{p<-1-p} evaluated only at the listed output checkerboard rows.

    Works straight from the definition site by site (neighbour coordinates,
    links and gamma matrices), so it can sample outputs of lattices too large
    for the whole-lattice routine.  Returns shape (len(rows), Ls, 4, 3).
    """
    dims = dims_of(U)
    lx, ly, lz, lt = dims
    L = (lx, ly, lz, lt)
    x = list(site_of_cb(dims, out_parity, rows))
    ls = psi_cb.shape[1]
    out = np.zeros((len(rows), ls, 4, 3), dtype=np.complex128)
    sgn = 1.0 if dagger else -1.0

    def cbrow(c4):
        lex = c4[0] + lx * (c4[1] + ly * (c4[2] + lz * c4[3]))
        return lex // 2

    for mu in range(4):
        xf = list(x)
        xf[mu] = (x[mu] + 1) % L[mu]
        xb = list(x)
        xb[mu] = (x[mu] - 1) % L[mu]
        e_f = np.where((mu == 3) & (x[3] == lt - 1) & antiperiodic_t, -1.0, 1.0)
        e_b = np.where((mu == 3) & (xb[3] == lt - 1) & antiperiodic_t, -1.0, 1.0)
        uf = U[x[3], x[2], x[1], x[0], mu] * e_f[:, None, None]
        ub = U[xb[3], xb[2], xb[1], xb[0], mu] * e_b[:, None, None]
        pf = psi_cb[cbrow(xf)]
        pb = psi_cb[cbrow(xb)]
        out += _spin(ID4 + sgn * GAMMA[mu], np.einsum("nab,nsib->nsia", uf, pf))
        out += _spin(ID4 - sgn * GAMMA[mu], np.einsum("nba,nsib->nsia", ub.conj(), pb))
    return out


def wilson(U, psi4, m: float, antiperiodic_t: bool = True):
    """4D Wilson operator D_W(m) = (4+m) - D_h/2 on (Lt,Lz,Ly,Lx,4,3)."""
    p5 = psi4[..., None, :, :]
    return ((4.0 + m) * p5 - 0.5 * dhop(U, p5, False, antiperiodic_t))[..., 0, :, :]


# ----------------------------------------------------------------------------
# Fifth-dimension (Shamir) term
# ----------------------------------------------------------------------------
def m5op(psi, M5: float, mf: float, dagger: bool = False):
    """Shamir M5op (or its adjoint) on any field whose last three axes are (Ls, 4, 3)."""
    ls = psi.shape[-3]
    out = (5.0 - M5) * psi
    for s in range(ls):
        up = psi[..., s + 1, :, :] if s + 1 < ls else -mf * psi[..., 0, :, :]  # psi~(s+1)
        dn = psi[..., s - 1, :, :] if s >= 1 else -mf * psi[..., ls - 1, :, :]  # psi~(s-1)
        if not dagger:
            out[..., s, :, :] -= _spin(P_MINUS, up) + _spin(P_PLUS, dn)
        else:
            out[..., s, :, :] -= _spin(P_PLUS, up) + _spin(P_MINUS, dn)
    return out


def shift_matrix(ls: int, mf: float):
    """Ls x Ls matrix K with K[s, s+1] = 1 and the wrap K[Ls-1, 0] = -mf."""
    k = np.zeros((ls, ls))
    for s in range(ls):
        if s + 1 < ls:
            k[s, s + 1] += 1.0
        else:
            k[s, 0] += -mf
    return k


def m5_matrix(ls: int, M5: float, mf: float):
    """M5op as a dense (Ls*4) x (Ls*4) matrix over (s, spin), colour-blind."""
    k = shift_matrix(ls, mf)
    return (5.0 - M5) * np.eye(4 * ls) - np.kron(k, P_MINUS) - np.kron(k.T, P_PLUS)


def m5inv(psi, M5: float, mf: float, dagger: bool = False):
    """M5op^-1 (or M5op^-dag) by a dense LU solve of the (Ls*4) x (Ls*4) matrix."""
    ls = psi.shape[-3]
    m = m5_matrix(ls, M5, mf)
    if dagger:
        m = m.conj().T
    lead = psi.shape[:-3]
    flat = psi.reshape((-1, ls * 4, 3))  # rows ordered (s, spin)
    rhs = np.moveaxis(flat, 0, 1).reshape(ls * 4, -1)
    sol = np.linalg.solve(m, rhs)
    sol = np.moveaxis(sol.reshape(ls * 4, -1, 3), 1, 0)
    return sol.reshape(lead + (ls, 4, 3))


# ----------------------------------------------------------------------------
# Full operator and Schur form
# ----------------------------------------------------------------------------
def ddw(U, psi, M5: float, mf: float, dagger: bool = False, antiperiodic_t: bool = True):
    """D_DW = M5op - D_h/2 (or its adjoint) on a full 5D field."""
    return m5op(psi, M5, mf, dagger) - 0.5 * dhop(U, psi, dagger, antiperiodic_t)


def mpc(U, psi_o, M5, mf, dagger: bool = False, antiperiodic_t: bool = True):
    """M_pc = M5op - 1/4 D_h^{o<-e} M5op^-1 D_h^{e<-o} on the odd checkerboard (or M_pc^dag)."""
    t = dhop_cb(U, psi_o, 0, dagger, antiperiodic_t)
    t = m5inv(t, M5, mf, dagger)
    t = dhop_cb(U, t, 1, dagger, antiperiodic_t)
    return m5op(psi_o, M5, mf, dagger) - 0.25 * t


def mdagm(U, psi_o, M5, mf, antiperiodic_t: bool = True):
    return mpc(U, mpc(U, psi_o, M5, mf, False, antiperiodic_t), M5, mf, True, antiperiodic_t)


# ----------------------------------------------------------------------------
# Moebius (Cayley) generalisation
# ----------------------------------------------------------------------------
def k5(psi, mf: float, dagger: bool = False):
    """Fifth-dimension hop (K psi)(s) = P_- psi~(s+1) + P_+ psi~(s-1) (adjoint: P_+ and P_- swapped)."""
    ls = psi.shape[-3]
    out = np.zeros_like(psi)
    for s in range(ls):
        up = psi[..., s + 1, :, :] if s + 1 < ls else -mf * psi[..., 0, :, :]
        dn = psi[..., s - 1, :, :] if s >= 1 else -mf * psi[..., ls - 1, :, :]
        if not dagger:
            out[..., s, :, :] = _spin(P_MINUS, up) + _spin(P_PLUS, dn)
        else:
            out[..., s, :, :] = _spin(P_PLUS, up) + _spin(P_MINUS, dn)
    return out


def mobius_ddw(U, psi, M5, mf, b, c, dagger: bool = False, antiperiodic_t: bool = True):
    """Moebius D = (b D_W + 1) psi(s) + (c D_W - 1) (K psi)(s) with D_W = (4 - M5) - D_h/2.

    The adjoint is D^dag = (b + c K^dag) D_W^dag + 1 - K^dag.
    """
    def dw(f, dag):
        return (4.0 - M5) * f - 0.5 * dhop(U, f, dag, antiperiodic_t)

    if not dagger:
        kp = k5(psi, mf)
        return b * dw(psi, False) + psi + c * dw(kp, False) - kp
    w = dw(psi, True)
    return b * w + c * k5(w, mf, True) + psi - k5(psi, mf, True)


def mooee(psi, M5, mf, b, c, dagger: bool = False):
    """Site-local part of D_mob: [b (4-M5) + 1] psi - [1 - c (4-M5)] K psi (adjoint: K^dag)."""
    return (b * (4.0 - M5) + 1.0) * psi - (1.0 - c * (4.0 - M5)) * k5(psi, mf, dagger)


def mooee_inv(psi, M5, mf, b, c, dagger: bool = False):
    """Mooee^-1 (or Mooee^-dag) by a dense LU solve of the (Ls*4) x (Ls*4) matrix."""
    ls = psi.shape[-3]
    k = shift_matrix(ls, mf)
    kmat = np.kron(k, P_MINUS) + np.kron(k.T, P_PLUS)
    m = (b * (4.0 - M5) + 1.0) * np.eye(4 * ls) - (1.0 - c * (4.0 - M5)) * kmat
    if dagger:
        m = m.conj().T
    lead = psi.shape[:-3]
    flat = psi.reshape((-1, ls * 4, 3))
    rhs = np.moveaxis(flat, 0, 1).reshape(ls * 4, -1)
    sol = np.linalg.solve(m, rhs)
    sol = np.moveaxis(sol.reshape(ls * 4, -1, 3), 1, 0)
    return sol.reshape(lead + (ls, 4, 3))


def mobius_mpc(U, psi_o, M5, mf, b, c, dagger: bool = False, antiperiodic_t: bool = True):
    """Odd-checkerboard Schur complement of D_mob (or its adjoint).

    M_pc     = Mooee     - 1/4 D_h^{o<-e} (b + cK) Mooee^-1 D_h^{e<-o} (b + cK)
    M_pc^dag = Mooee^dag - 1/4 (b + cK^dag) D_h^dag{o<-e} Mooee^-dag (b + cK^dag) D_h^dag{e<-o}
    """
    if not dagger:
        u = b * psi_o + c * k5(psi_o, mf)
        t = dhop_cb(U, u, 0, False, antiperiodic_t)
        t = mooee_inv(t, M5, mf, b, c)
        t = b * t + c * k5(t, mf)
        t = dhop_cb(U, t, 1, False, antiperiodic_t)
        return mooee(psi_o, M5, mf, b, c) - 0.25 * t
    t = dhop_cb(U, psi_o, 0, True, antiperiodic_t)
    t = b * t + c * k5(t, mf, True)
    t = mooee_inv(t, M5, mf, b, c, True)
    t = dhop_cb(U, t, 1, True, antiperiodic_t)
    t = b * t + c * k5(t, mf, True)
    return mooee(psi_o, M5, mf, b, c, True) - 0.25 * t


def mobius_mdagm(U, psi_o, M5, mf, b, c, antiperiodic_t: bool = True):
    return mobius_mpc(U, mobius_mpc(U, psi_o, M5, mf, b, c, False, antiperiodic_t), M5, mf, b, c, True,
                      antiperiodic_t)


# ----------------------------------------------------------------------------
# Linear algebra: conjugate gradient and the Schur-preconditioned solve
# ----------------------------------------------------------------------------
def vdot(a, b) -> complex:
    return complex(np.vdot(a.ravel(), b.ravel()))


def norm2(a) -> float:
    return float(np.vdot(a.ravel(), a.ravel()).real)


def cg(apply_a, b, tol: float, maxit: int, x0=None):
    """Hestenes-Stiefel conjugate gradient for Hermitian positive-definite A.

    Stops when the recursively updated ||r||/||b|| <= tol, then recomputes the
    true residual b - A x and restarts from x if it is still above tol.
    Returns (x, iterations, true relative residual).
    """
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = np.sqrt(norm2(b))
    iters = 0
    while True:
        r = b - apply_a(x) if iters or x0 is not None else b.copy()
        rr = norm2(r)
        if np.sqrt(rr) / bnorm <= tol:
            return x, iters, np.sqrt(rr) / bnorm
        p = r.copy()
        while iters < maxit:
            ap = apply_a(p)
            alpha = rr / vdot(p, ap).real
            x = x + alpha * p
            r = r - alpha * ap
            rr_new = norm2(r)
            iters += 1
            if np.sqrt(rr_new) / bnorm <= tol:
                break
            p = r + (rr_new / rr) * p
            rr = rr_new
        true = np.sqrt(norm2(b - apply_a(x))) / bnorm
        if true <= tol or iters >= maxit:
            return x, iters, true


def solve_full(U, b, M5, mf, tol=1e-12, maxit=10000, antiperiodic_t=True):
    """Solve D_DW x = b through the odd-checkerboard Schur complement.

    b^_o = b_o + 1/2 D_h^{o<-e} M5op^-1 b_e;  M_pc^dag M_pc x_o = M_pc^dag b^_o;
    x_e = M5op^-1 (b_e + 1/2 D_h^{e<-o} x_o).
    """
    dims = dims_of(U)
    be, bo = full_to_cb(b, 0), full_to_cb(b, 1)
    bh = bo + 0.5 * dhop_cb(U, m5inv(be, M5, mf), 1, False, antiperiodic_t)
    rhs = mpc(U, bh, M5, mf, True, antiperiodic_t)
    xo, it, _ = cg(lambda v: mdagm(U, v, M5, mf, antiperiodic_t), rhs, tol, maxit)
    xe = m5inv(be + 0.5 * dhop_cb(U, xo, 0, False, antiperiodic_t), M5, mf)
    return cb_to_full(xo, 1, dims, other=xe), it


# ----------------------------------------------------------------------------
# Action and force
# ----------------------------------------------------------------------------
def action_dense(U, phi, M5, mf, antiperiodic_t=True):
    """S = phi^dag (D^dag D)^-1 phi by a dense solve (tiny lattices only)."""
    d = dense_operator(lambda v: ddw(U, v, M5, mf, False, antiperiodic_t), phi.shape)
    z = np.linalg.solve(d.conj().T, phi.ravel())
    return float(np.vdot(z, z).real)


def action_cg(U, phi, M5, mf, tol=1e-13, maxit=20000, antiperiodic_t=True):
    """S = phi^dag (D^dag D)^-1 phi with X from CG on the full normal operator.

    Uses the stationary estimator S = 2 Re(phi^dag X) - X^dag (D^dag D) X, whose
    error is quadratic in the solver error.  Returns (S, X).
    """
    def a(v):
        return ddw(U, ddw(U, v, M5, mf, False, antiperiodic_t), M5, mf, True, antiperiodic_t)

    x, _, _ = cg(a, phi, tol, maxit)
    s = 2.0 * vdot(phi, x).real - vdot(x, a(x)).real
    return s, x


def force_outer(U, X, Y, antiperiodic_t=True):
    """Colour outer products of the hopping term's link derivative.

    M_mu(x)_{ba} = sum_s sum_{ab spin} (1-gamma_mu)_{alpha beta} X(x+mu,s)_{beta b} conj(Y(x,s)_{alpha a})
    N_mu(x)_{ba} = sum_s sum            (1+gamma_mu)_{alpha beta} X(x,s)_{beta b}    conj(Y(x+mu,s)_{alpha a})
    Returns (M, N) shaped like U.
    """
    m = np.zeros_like(U)
    n = np.zeros_like(U)
    for mu in range(4):
        ax = axis_of(mu)
        xf = np.roll(X, -1, axis=ax)
        yf = np.roll(Y, -1, axis=ax)
        m[..., mu, :, :] = np.einsum("ij,tzyxsjb,tzyxsia->tzyxba", ID4 - GAMMA[mu], xf, Y.conj())
        n[..., mu, :, :] = np.einsum("ij,tzyxsjb,tzyxsia->tzyxba", ID4 + GAMMA[mu], X, yf.conj())
    return m, n


def force_euclid(U, X, Y, antiperiodic_t=True):
    """g_mu(x) = eta_mu(x) (M_mu(x)^dag + N_mu(x)).

    Gradient of Re(Y^dag D_h X) with respect to U in the convention
    delta f = Re sum conj(g) delta U.
    """
    m, n = force_outer(U, X, Y, antiperiodic_t)
    et = eta(dims_of(U), antiperiodic_t)[..., None, None]
    return et * (np.conj(np.swapaxes(m, -1, -2)) + n)


def force_su3(U, X, Y, antiperiodic_t=True):
    """K_mu(x): traceless part of (i/2)(G - G^dag), G = eta (U M - N U^dag).

    With X = (D^dag D)^-1 phi and Y = D X, dS/d(eps) = sum tr(Q K) for the
    perturbation U -> exp(i eps Q) U.
    """
    m, n = force_outer(U, X, Y, antiperiodic_t)
    et = eta(dims_of(U), antiperiodic_t)[..., None, None]
    udag = np.conj(np.swapaxes(U, -1, -2))
    g = et * (U @ m - n @ udag)
    k = 0.5j * (g - np.conj(np.swapaxes(g, -1, -2)))
    tr = np.trace(k, axis1=-2, axis2=-1)[..., None, None]
    return k - tr / 3.0 * np.eye(3)


# ----------------------------------------------------------------------------
# Hybrid Monte Carlo molecular dynamics with the pseudofermion action
# ----------------------------------------------------------------------------
def expi(q, eps):
    """exp(i eps Q) for Hermitian Q [..., 3, 3], by its eigen-decomposition."""
    w, v = np.linalg.eigh(q)
    return np.einsum("...ik,...k,...jk->...ij", v, np.exp(1j * eps * w), v.conj())


def action_and_force(U, phi, M5, mf, tol=1e-13, antiperiodic_t=True):
    """S = phi^dag (D^dag D)^-1 phi and its su(3) force K: under U -> exp(i eps Q) U the
    action changes by eps sum tr(Q K) + O(eps^2)."""
    s, x = action_cg(U, phi, M5, mf, tol=tol, antiperiodic_t=antiperiodic_t)
    y = ddw(U, x, M5, mf, False, antiperiodic_t)
    return s, force_su3(U, x, y, antiperiodic_t)


def hamiltonian(U, P, phi, M5, mf, tol=1e-13, antiperiodic_t=True):
    """H = sum_links tr(P^2) + S(U) for traceless Hermitian momenta P = sum_a omega_a lambda_a / 2,
    whose Gaussian weight exp(-sum omega^2 / 2) is exp(-sum tr P^2)."""
    s, _ = action_and_force(U, phi, M5, mf, tol, antiperiodic_t)
    return float(np.sum(np.einsum("...ij,...ji->...", P, P)).real) + s


def leapfrog(U, P, phi, M5, mf, eps, nsteps, tol=1e-13, antiperiodic_t=True):
    """nsteps leapfrog steps of the equations that conserve H: dU/dtau = i P U and
    dP/dtau = -K(U)/2 (d tr P^2 = -tr(P K) dtau cancels dS = tr(P K) dtau).  A half step
    of P, alternating full steps of U and P, and a closing half step of P.  Returns (U, P)."""
    _, k = action_and_force(U, phi, M5, mf, tol, antiperiodic_t)
    P = P - 0.25 * eps * k
    for n in range(nsteps):
        U = expi(P, eps) @ U
        _, k = action_and_force(U, phi, M5, mf, tol, antiperiodic_t)
        P = P - (0.5 * eps if n + 1 < nsteps else 0.25 * eps) * k
    return U, P


# ----------------------------------------------------------------------------
# Dense matrices (brute force on tiny lattices)
# ----------------------------------------------------------------------------
def dense_operator(apply, shape):
    """Dense matrix of a linear map on complex arrays of `shape`, column by column."""
    n = int(np.prod(shape))
    out = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1.0
        out[:, j] = apply(e.reshape(shape)).ravel()
        e[j] = 0.0
    return out
