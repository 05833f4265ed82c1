"""Pins of the CPU oracle against facts fixed by mathematics, not by the oracle itself.

Each test checks the numpy reference against something independent of its
own formulas: Clifford algebra, closed-form free-field spectra, brute-force
dense matrices, gauge covariance, finite differences, and a second
site-by-site evaluation.  A dropped term, a wrong sign or index, or a
transposed operand in the reference fails at least one of these.
"""

import itertools

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

from oracle import dwf_ref as R
from synth import fields as F

M5, MF = 1.8, 0.01


def _match(a, b):
    """Max distance of the best one-to-one matching of two complex multisets."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    assert a.size == b.size
    cost = np.abs(a[:, None] - b[None, :])
    i, j = linear_sum_assignment(cost)
    return cost[i, j].max()


def _momenta(dims, antiperiodic=True):
    lx, ly, lz, lt = dims
    ps = []
    for n in itertools.product(range(lx), range(ly), range(lz), range(lt)):
        p = [2 * np.pi * n[0] / lx, 2 * np.pi * n[1] / ly, 2 * np.pi * n[2] / lz,
             ((2 * n[3] + 1) if antiperiodic else 2 * n[3]) * np.pi / lt]
        ps.append(np.array(p))
    return ps


# ---------------------------------------------------------------------------
# Gamma matrices
# ---------------------------------------------------------------------------
def test_clifford_algebra_and_chirality():
    g = R.GAMMA
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            assert np.allclose(g[mu] @ g[nu] + g[nu] @ g[mu], 2.0 * (mu == nu) * np.eye(4))
        assert np.allclose(g[mu] @ R.GAMMA5 + R.GAMMA5 @ g[mu], 0)
    assert np.allclose(R.GAMMA5, np.diag([1, 1, -1, -1]))


# ---------------------------------------------------------------------------
# Generators
# ---------------------------------------------------------------------------
def test_generated_links_are_su3():
    u = F.gauge_field((4, 2, 2, 4), 0.5, seed=11).reshape(-1, 3, 3)
    eye = np.eye(3)
    assert np.abs(np.conj(np.swapaxes(u, 1, 2)) @ u - eye).max() < 1e-14
    assert np.abs(np.linalg.det(u) - 1).max() < 1e-14
    # exp(i eps H) with small eps stays close to the identity
    u_small = F.gauge_field((2, 2, 2, 2), 1e-3, seed=11).reshape(-1, 3, 3)
    assert np.abs(u_small - eye).max() < 1e-2


def test_generator_statistics_and_determinism():
    rng = np.random.Generator(np.random.PCG64(7))
    w = rng.standard_normal(200000)
    assert abs(w.mean()) < 0.01 and abs(w.var() - 1) < 0.02
    a = F.fermion_cb((4, 4, 4, 4), 8, seed=201)
    b = F.fermion_cb((4, 4, 4, 4), 8, seed=201)
    assert np.array_equal(a, b)
    assert abs(a.real.var() - 1) < 0.05 and abs(a.imag.var() - 1) < 0.05
    q = F.su3_directions((2, 2, 2, 2), 600)
    assert np.allclose(q, np.conj(np.swapaxes(q, -1, -2)))
    assert np.abs(np.trace(q, axis1=-2, axis2=-1)).max() < 1e-14


# ---------------------------------------------------------------------------
# Free-field closed forms (unit links)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dims", [(4, 2, 2, 4), (2, 4, 2, 2)])
def test_free_wilson_spectrum(dims):
    """Eigenvalues of D_W(m) at U = 1 are m + sum(1 - cos p) +- i sqrt(sum sin^2 p), 6-fold."""
    m = -0.3
    u = F.unit_gauge(dims)
    lx, ly, lz, lt = dims
    d = R.dense_operator(lambda v: R.wilson(u, v, m), (lt, lz, ly, lx, 4, 3))
    ev = np.linalg.eigvals(d)
    want = []
    for p in _momenta(dims):
        re = m + np.sum(1 - np.cos(p))
        im = np.sqrt(np.sum(np.sin(p) ** 2))
        want += [re + 1j * im] * 6 + [re - 1j * im] * 6
    assert _match(ev, want) < 1e-10


def test_free_wilson_spectrum_detects_periodic_time():
    """The antiperiodic time momenta are required: periodic ones do not fit."""
    dims = (2, 2, 2, 4)
    u = F.unit_gauge(dims)
    d = R.dense_operator(lambda v: R.wilson(u, v, 0.1), (4, 2, 2, 2, 4, 3))
    ev = np.linalg.eigvals(d)
    wrong = []
    for p in _momenta(dims, antiperiodic=False):
        re = 0.1 + np.sum(1 - np.cos(p))
        im = np.sqrt(np.sum(np.sin(p) ** 2))
        wrong += [re + 1j * im] * 6 + [re - 1j * im] * 6
    assert _match(ev, wrong) > 1e-2


@pytest.mark.parametrize("dims,ls,mf", [((4, 2, 2, 2), 4, 0.01), ((2, 2, 4, 2), 3, 0.2)])
def test_free_dwf_normal_spectrum(dims, ls, mf):
    """D^dag D at U = 1: eigenvalues sigma_k(A(p))^2 + sum sin^2 p, A = W - K, 12-fold.

    det A = W^Ls + mf fixes the sign of the mass wrap independently of the SVD.
    """
    u = F.unit_gauge(dims)
    lx, ly, lz, lt = dims
    shape = (lt, lz, ly, lx, ls, 4, 3)
    d = R.dense_operator(lambda v: R.ddw(u, v, M5, mf), shape)
    ev = np.linalg.eigvalsh(d.conj().T @ d)
    want = []
    k = np.zeros((ls, ls))
    for s in range(ls - 1):
        k[s, s + 1] = 1
    k[ls - 1, 0] = -mf
    for p in _momenta(dims):
        w = 1 - M5 + np.sum(1 - np.cos(p))
        a = w * np.eye(ls) - k
        assert abs(np.linalg.det(a) - (w ** ls + mf)) < 1e-12 * max(1.0, abs(w) ** ls)
        sv = np.linalg.svd(a, compute_uv=False)
        want += list(np.repeat(sv ** 2 + np.sum(np.sin(p) ** 2), 12))
    assert np.abs(np.sort(ev) - np.sort(want)).max() < 1e-10


def test_free_dwf_periodic_fifth_dimension_closed_form():
    """mf = -1 makes s periodic: singular values of A are |W - exp(i q)|, q = 2 pi k / Ls."""
    dims, ls = (2, 2, 2, 4), 4
    u = F.unit_gauge(dims)
    shape = (4, 2, 2, 2, ls, 4, 3)
    d = R.dense_operator(lambda v: R.ddw(u, v, M5, -1.0), shape)
    ev = np.linalg.eigvalsh(d.conj().T @ d)
    want = []
    for p in _momenta(dims):
        w = 1 - M5 + np.sum(1 - np.cos(p))
        for kq in range(ls):
            q = 2 * np.pi * kq / ls
            want += [abs(w - np.exp(1j * q)) ** 2 + np.sum(np.sin(p) ** 2)] * 12
    assert np.abs(np.sort(ev) - np.sort(want)).max() < 1e-10


def test_free_plane_wave_hopping():
    """D_h e^{ipx} chi = e^{ipx} sum_mu (2 cos p_mu - 2 i gamma_mu sin p_mu) chi, with p_t antiperiodic."""
    dims = (4, 4, 2, 4)
    u = F.unit_gauge(dims)
    x, y, z, t = R.coords(dims)
    rng = np.random.default_rng(3)
    chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    p = np.array([2 * np.pi / 4, 2 * np.pi * 3 / 4, np.pi, 3 * np.pi / 4])
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    psi = phase[..., None, None, None] * chi[None, None, None, None, None]
    got = R.dhop(u, psi)
    mom = sum(2 * np.cos(p[m]) * np.eye(4) - 2j * np.sin(p[m]) * R.GAMMA[m] for m in range(4))
    want = phase[..., None, None, None] * (mom @ chi)[None, None, None, None, None]
    assert np.abs(got - want).max() < 1e-13


# ---------------------------------------------------------------------------
# Adjoints, gamma5-hermiticity, brute force
# ---------------------------------------------------------------------------
def test_dense_adjoint_and_gamma5_hermiticity():
    dims, ls = (2, 2, 2, 2), 4
    u = F.gauge_field(dims, 0.5, 101)
    shape = (2, 2, 2, 2, ls, 4, 3)
    dh = R.dense_operator(lambda v: R.dhop(u, v), shape)
    dhd = R.dense_operator(lambda v: R.dhop(u, v, dagger=True), shape)
    assert np.abs(dhd - dh.conj().T).max() < 1e-13
    dd = R.dense_operator(lambda v: R.ddw(u, v, M5, MF), shape)
    ddd = R.dense_operator(lambda v: R.ddw(u, v, M5, MF, dagger=True), shape)
    assert np.abs(ddd - dd.conj().T).max() < 1e-13
    # D_h^dag = g5 D_h g5 ; D_DW^dag = Gamma5 D_DW Gamma5 with Gamma5 = g5 R5 (s -> Ls-1-s)
    g5 = np.kron(np.eye(16 * ls), np.kron(R.GAMMA5, np.eye(3)))
    assert np.abs(g5 @ dh @ g5 - dhd).max() < 1e-13
    r5 = np.kron(np.eye(16), np.kron(np.eye(ls)[::-1], np.eye(12)))
    G5 = g5 @ r5
    assert np.abs(G5 @ dd @ G5 - ddd).max() < 1e-13


def test_inner_product_adjoint_on_random_fields():
    dims, ls = (4, 4, 2, 4), 5
    u = F.gauge_field(dims, 0.5, 12)
    a = F.fermion_full(dims, ls, 1)
    b = F.fermion_full(dims, ls, 2)
    lhs = R.vdot(a, R.ddw(u, b, M5, MF))
    rhs = R.vdot(R.ddw(u, a, M5, MF, dagger=True), b)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("dagger", [False, True])
def test_gauge_covariance(dagger):
    dims, ls = (4, 2, 4, 2), 3
    u = F.gauge_field(dims, 0.7, 21)
    om = F.random_su3_field(dims, 22)
    psi = F.fermion_full(dims, ls, 23)
    up = np.empty_like(u)
    for mu in range(4):
        omf = np.roll(om, -1, axis=R.axis_of(mu))
        up[..., mu, :, :] = om @ u[..., mu, :, :] @ np.conj(np.swapaxes(omf, -1, -2))
    rot = np.einsum("tzyxab,tzyxsib->tzyxsia", om, psi)
    lhs = R.dhop(up, rot, dagger)
    rhs = np.einsum("tzyxab,tzyxsib->tzyxsia", om, R.dhop(u, psi, dagger))
    assert np.abs(lhs - rhs).max() < 1e-13


@pytest.mark.parametrize("par,dagger", [(0, False), (1, False), (0, True), (1, True)])
def test_sitewise_dhop_matches_whole_lattice(par, dagger):
    dims, ls = (6, 4, 2, 4), 3
    u = F.gauge_field(dims, 0.5, 31)
    psi = F.fermion_cb(dims, ls, 32)
    whole = R.dhop_cb(u, psi, par, dagger)
    rows = np.arange(psi.shape[0])
    assert np.abs(R.dhop_sites(u, psi, par, rows, dagger) - whole).max() < 1e-13


def test_checkerboard_blocks():
    dims, ls = (4, 2, 2, 2), 2
    u = F.gauge_field(dims, 0.5, 41)
    psi = F.fermion_full(dims, ls, 42)
    full = R.dhop(u, psi)
    for p in (0, 1):
        # D_h only couples opposite parities
        assert np.abs(R.full_to_cb(R.dhop(u, R.cb_to_full(R.full_to_cb(psi, p), p, dims)), p)).max() == 0
        got = R.dhop_cb(u, R.full_to_cb(psi, 1 - p), p)
        assert np.abs(got - R.full_to_cb(full, p)).max() < 1e-14


def test_hopping_is_diagonal_in_s():
    dims, ls = (2, 2, 2, 4), 3
    u = F.gauge_field(dims, 0.5, 45)
    psi = F.fermion_full(dims, ls, 46)
    out = R.dhop(u, psi)
    for s in range(ls):
        one = np.zeros_like(psi)
        one[..., s, :, :] = psi[..., s, :, :]
        d1 = R.dhop(u, one)
        assert np.abs(d1[..., s, :, :] - out[..., s, :, :]).max() < 1e-14
        d1[..., s, :, :] = 0
        assert np.abs(d1).max() == 0


# ---------------------------------------------------------------------------
# Fifth dimension
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ls", [1, 2, 5, 8])
def test_m5_loop_matches_matrix_and_inverse(ls):
    rng = np.random.default_rng(ls)
    psi = rng.standard_normal((7, ls, 4, 3)) + 1j * rng.standard_normal((7, ls, 4, 3))
    m = R.m5_matrix(ls, M5, MF)
    as_mat = np.einsum("ij,njc->nic", m, psi.reshape(7, ls * 4, 3)).reshape(psi.shape)
    assert np.abs(R.m5op(psi, M5, MF) - as_mat).max() < 1e-14
    as_mat_d = np.einsum("ij,njc->nic", m.conj().T, psi.reshape(7, ls * 4, 3)).reshape(psi.shape)
    assert np.abs(R.m5op(psi, M5, MF, dagger=True) - as_mat_d).max() < 1e-14
    for dag in (False, True):
        back = R.m5op(R.m5inv(psi, M5, MF, dag), M5, MF, dag)
        assert np.abs(back - psi).max() < 1e-13


def test_m5inv_geometric_closed_form():
    """(d - K)^-1 psi(s) = sum_n d^-(n+1) [wrap factor] psi(s+n) / (1 + mf d^-Ls) on spins 2,3."""
    ls = 6
    d = 5 - M5
    rng = np.random.default_rng(5)
    psi = rng.standard_normal((3, ls, 4, 3)) + 1j * rng.standard_normal((3, ls, 4, 3))
    got = R.m5inv(psi, M5, MF)
    want = np.zeros_like(psi)
    for s in range(ls):
        for n in range(ls):
            j = s + n
            f = 1.0 if j < ls else -MF
            want[:, s] += d ** (-(n + 1)) * f * psi[:, j % ls]
    want /= 1 + MF * d ** (-ls)
    assert np.abs(got[:, :, 2:4] - want[:, :, 2:4]).max() < 1e-14
    # spins 0,1 couple the other way round: s-n
    want_p = np.zeros_like(psi)
    for s in range(ls):
        for n in range(ls):
            j = s - n
            f = 1.0 if j >= 0 else -MF
            want_p[:, s] += d ** (-(n + 1)) * f * psi[:, j % ls]
    want_p /= 1 + MF * d ** (-ls)
    assert np.abs(got[:, :, 0:2] - want_p[:, :, 0:2]).max() < 1e-14


# ---------------------------------------------------------------------------
# Schur complement, CG, full solve
# ---------------------------------------------------------------------------
def test_schur_complement_matches_dense_blocks():
    dims, ls = (2, 2, 2, 2), 3
    u = F.gauge_field(dims, 0.5, 51)
    shape = (2, 2, 2, 2, ls, 4, 3)
    d = R.dense_operator(lambda v: R.ddw(u, v, M5, MF), shape)
    n = d.shape[0]
    par = np.repeat(R.parity(dims).reshape(-1), ls * 12)
    e, o = np.where(par == 0)[0], np.where(par == 1)[0]
    schur = d[np.ix_(o, o)] - d[np.ix_(o, e)] @ np.linalg.inv(d[np.ix_(e, e)]) @ d[np.ix_(e, o)]
    cbshape = (8, ls, 4, 3)
    mp = R.dense_operator(lambda v: R.mpc(u, v, M5, MF), cbshape)
    assert np.abs(mp - schur).max() < 1e-12
    mpd = R.dense_operator(lambda v: R.mpc(u, v, M5, MF, dagger=True), cbshape)
    assert np.abs(mpd - schur.conj().T).max() < 1e-12
    assert n == 16 * ls * 12


def test_cg_matches_dense_solve_and_full_solve():
    dims, ls = (2, 2, 2, 4), 4
    u = F.gauge_field(dims, 0.5, 61)
    b = F.fermion_cb(dims, ls, 62)
    x, it, res = R.cg(lambda v: R.mdagm(u, v, M5, MF), b, 1e-12, 2000)
    a = R.dense_operator(lambda v: R.mdagm(u, v, M5, MF), b.shape)
    xd = np.linalg.solve(a, b.ravel()).reshape(b.shape)
    assert res <= 1e-12
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-9
    # full 5D solve through the Schur complement satisfies D x = b
    bf = F.fermion_full(dims, ls, 63)
    xf, _ = R.solve_full(u, bf, M5, MF, tol=1e-12)
    r = R.ddw(u, xf, M5, MF) - bf
    assert np.linalg.norm(r) / np.linalg.norm(bf) < 1e-10


# ---------------------------------------------------------------------------
# Action and force
# ---------------------------------------------------------------------------
def _expi(q, eps):
    w, v = np.linalg.eigh(q)
    return np.einsum("...ik,...k,...jk->...ij", v, np.exp(1j * eps * w), v.conj())


def test_action_positive_and_consistent():
    dims, ls = (2, 2, 2, 2), 3
    u = F.gauge_field(dims, 0.5, 71)
    phi = F.fermion_full(dims, ls, 72)
    s_dense = R.action_dense(u, phi, M5, MF)
    s_cg, x = R.action_cg(u, phi, M5, MF)
    assert s_dense > 0
    assert abs(s_cg - s_dense) < 1e-10 * s_dense
    ax = R.ddw(u, R.ddw(u, x, M5, MF), M5, MF, dagger=True)
    assert abs(R.vdot(x, ax) - R.vdot(phi, x)) < 1e-10 * s_dense
    assert abs(R.vdot(phi, x).imag) < 1e-10 * s_dense


@pytest.mark.parametrize("seed", [600, 601])
def test_su3_force_matches_finite_difference(seed):
    dims, ls = (2, 2, 2, 4), 3
    u = F.gauge_field(dims, 0.5, 81)
    phi = F.fermion_full(dims, ls, 82)
    s0, x = R.action_cg(u, phi, M5, MF)
    y = R.ddw(u, x, M5, MF)
    k = R.force_su3(u, x, y)
    q = F.su3_directions(dims, seed)
    analytic = np.sum(np.einsum("...ij,...ji->...", q, k)).real
    h = 1e-5
    sp, _ = R.action_cg(_expi(q, h) @ u, phi, M5, MF)
    sm, _ = R.action_cg(_expi(q, -h) @ u, phi, M5, MF)
    fd = (sp - sm) / (2 * h)
    assert abs(fd - analytic) <= 1e-6 * abs(analytic)
    # K is traceless Hermitian
    assert np.abs(k - np.conj(np.swapaxes(k, -1, -2))).max() < 1e-12
    assert np.abs(np.trace(k, axis1=-2, axis2=-1)).max() < 1e-12


def test_euclidean_gradient_matches_finite_difference():
    """Re(Y^dag D_h X) is linear in U: its directional derivative is Re sum conj(g) dU exactly."""
    dims, ls = (2, 4, 2, 2), 2
    u = F.gauge_field(dims, 0.5, 91)
    x = F.fermion_full(dims, ls, 92)
    y = F.fermion_full(dims, ls, 93)
    g = R.force_euclid(u, x, y)
    rng = np.random.default_rng(94)
    du = rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape)

    def f(uu):
        return R.vdot(y, R.dhop(uu, x)).real

    h = 1e-3
    fd = (f(u + h * du) - f(u - h * du)) / (2 * h)
    an = np.sum(np.conj(g) * du).real
    assert abs(fd - an) < 1e-10 * abs(an)


# ---------------------------------------------------------------------------
# Moebius (Cayley) generalisation
# ---------------------------------------------------------------------------
B_MOB, C_MOB = 1.5, 0.5


def test_mobius_reduces_to_shamir():
    dims, ls = (2, 4, 2, 4), 5
    u = F.gauge_field(dims, 0.5, 131)
    psi = F.fermion_full(dims, ls, 132)
    po = F.fermion_cb(dims, ls, 133)
    for dag in (False, True):
        assert np.abs(R.mobius_ddw(u, psi, M5, MF, 1.0, 0.0, dag) - R.ddw(u, psi, M5, MF, dag)).max() < 1e-13
        assert np.abs(R.mooee(psi, M5, MF, 1.0, 0.0, dag) - R.m5op(psi, M5, MF, dag)).max() < 1e-13
        assert np.abs(R.mooee_inv(psi, M5, MF, 1.0, 0.0, dag) - R.m5inv(psi, M5, MF, dag)).max() < 1e-12
        assert np.abs(R.mobius_mpc(u, po, M5, MF, 1.0, 0.0, dag) - R.mpc(u, po, M5, MF, dag)).max() < 1e-12


def _mobius_dense(u, dims, ls, b, c):
    """The 5D Moebius matrix assembled block by block from a dense D_W, in (s, site, spin, colour)
    order: (b D_W + 1) on the diagonal, (c D_W - 1) P_- on (s, s+1) and (c D_W - 1) P_+ on
    (s, s-1), with -mf on the two wraps."""
    vol = int(np.prod(dims))
    dw = R.dense_operator(lambda v: R.wilson(u, v, -M5), tuple(dims[::-1]) + (4, 3))
    n4 = dw.shape[0]
    one = np.eye(n4)
    pm = np.kron(np.eye(vol), np.kron(R.P_MINUS, np.eye(3)))
    pp = np.kron(np.eye(vol), np.kron(R.P_PLUS, np.eye(3)))
    big = np.zeros((ls * n4, ls * n4), dtype=np.complex128)
    for s in range(ls):
        blk = slice(s * n4, (s + 1) * n4)
        big[blk, blk] += b * dw + one
        up, fu = (s + 1, 1.0) if s + 1 < ls else (0, -MF)
        dn, fd = (s - 1, 1.0) if s >= 1 else (ls - 1, -MF)
        big[blk, up * n4:(up + 1) * n4] += fu * (c * dw - one) @ pm
        big[blk, dn * n4:(dn + 1) * n4] += fd * (c * dw - one) @ pp
    return big


def test_mobius_matches_dense_bno_blocks():
    dims, ls = (2, 2, 2, 2), 3
    u = F.gauge_field(dims, 0.5, 141)
    big = _mobius_dense(u, dims, ls, B_MOB, C_MOB)
    psi = F.fermion_full(dims, ls, 142)
    v = np.moveaxis(psi, 4, 0).ravel()  # (s, site, spin, colour)
    for dag, m in ((False, big), (True, big.conj().T)):
        want = np.moveaxis((m @ v).reshape((ls,) + psi.shape[:4] + (4, 3)), 0, 4)
        got = R.mobius_ddw(u, psi, M5, MF, B_MOB, C_MOB, dag)
        assert np.abs(got - want).max() < 1e-12


def test_mobius_schur_complement_matches_dense_blocks():
    dims, ls = (2, 2, 2, 2), 3
    u = F.gauge_field(dims, 0.5, 151)
    shape = (2, 2, 2, 2, ls, 4, 3)
    d = R.dense_operator(lambda v: R.mobius_ddw(u, v, M5, MF, B_MOB, C_MOB), shape)
    par = np.repeat(R.parity(dims).reshape(-1), ls * 12)
    e, o = np.where(par == 0)[0], np.where(par == 1)[0]
    schur = d[np.ix_(o, o)] - d[np.ix_(o, e)] @ np.linalg.inv(d[np.ix_(e, e)]) @ d[np.ix_(e, o)]
    cbshape = (8, ls, 4, 3)
    mp = R.dense_operator(lambda v: R.mobius_mpc(u, v, M5, MF, B_MOB, C_MOB), cbshape)
    assert np.abs(mp - schur).max() < 1e-12
    mpd = R.dense_operator(lambda v: R.mobius_mpc(u, v, M5, MF, B_MOB, C_MOB, dagger=True), cbshape)
    assert np.abs(mpd - schur.conj().T).max() < 1e-12


def test_mobius_adjoints_on_random_fields():
    dims, ls = (4, 4, 2, 4), 5
    u = F.gauge_field(dims, 0.5, 161)
    a = F.fermion_full(dims, ls, 162)
    b = F.fermion_full(dims, ls, 163)
    for op, opd in ((lambda f: R.mobius_ddw(u, f, M5, MF, B_MOB, C_MOB),
                     lambda f: R.mobius_ddw(u, f, M5, MF, B_MOB, C_MOB, True)),
                    (lambda f: R.k5(f, MF), lambda f: R.k5(f, MF, True)),
                    (lambda f: R.mooee(f, M5, MF, B_MOB, C_MOB), lambda f: R.mooee(f, M5, MF, B_MOB, C_MOB, True))):
        lhs = R.vdot(a, op(b))
        rhs = R.vdot(opd(a), b)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("b,c", [(1.5, 0.5), (2.0, 1.0), (1.0, 0.0)])
def test_mooee_inverse_geometric_closed_form(b, c):
    # Mooee = alpha - beta K with K^Ls = -mf on each chirality, so
    # Mooee^-1 = (1/beta) sum_n d^-(n+1) K^n / (1 + mf d^-Ls), d = alpha / beta.
    ls = 6
    psi = F.fermion_full((2, 2, 2, 2), ls, 171)
    alpha, beta = b * (4.0 - M5) + 1.0, 1.0 - c * (4.0 - M5)
    d = alpha / beta
    for dag in (False, True):
        acc = np.zeros_like(psi)
        kp = psi.copy()
        for n in range(ls):
            acc += d ** -(n + 1) * kp
            kp = R.k5(kp, MF, dag)
        acc /= beta * (1.0 + MF * d ** -ls)
        assert np.abs(R.mooee_inv(psi, M5, MF, b, c, dag) - acc).max() < 1e-13
        assert np.abs(R.mooee(R.mooee_inv(psi, M5, MF, b, c, dag), M5, MF, b, c, dag) - psi).max() < 1e-13


# ---------------------------------------------------------------------------
# Hybrid Monte Carlo molecular dynamics
# ---------------------------------------------------------------------------
def test_expi_is_the_matrix_exponential_in_su3():
    from scipy.linalg import expm

    q = F.su3_directions((2, 2, 2, 2), 701)
    e = R.expi(q, 0.37)
    want = np.array([expm(0.37j * m) for m in q.reshape(-1, 3, 3)]).reshape(e.shape)
    assert np.abs(e - want).max() < 1e-14
    eye = np.eye(3)
    assert np.abs(np.conj(np.swapaxes(e, -1, -2)) @ e - eye).max() < 1e-14
    assert np.abs(np.linalg.det(e) - 1.0).max() < 1e-14


def _md_case():
    dims, ls = (2, 2, 2, 4), 3
    u = F.gauge_field(dims, 0.5, 711)
    phi = F.fermion_full(dims, ls, 712)
    p = F.su3_directions(dims, 713)
    return u, p, phi


def test_leapfrog_is_reversible():
    u, p, phi = _md_case()
    u1, p1 = R.leapfrog(u, p, phi, M5, MF, 0.1, 3)
    u2, p2 = R.leapfrog(u1, -p1, phi, M5, MF, 0.1, 3)
    assert np.abs(u2 - u).max() < 1e-10
    assert np.abs(-p2 - p).max() < 1e-10
    assert np.abs(u1 - u).max() > 1e-2  # it moved


def test_leapfrog_energy_violation_is_second_order():
    # over a fixed trajectory length the leapfrog error in H is O(eps^2)
    u, p, phi = _md_case()
    h0 = R.hamiltonian(u, p, phi, M5, MF)
    dh = []
    for eps, n in ((0.1, 4), (0.05, 8)):
        u1, p1 = R.leapfrog(u, p, phi, M5, MF, eps, n)
        dh.append(R.hamiltonian(u1, p1, phi, M5, MF) - h0)
    ratio = dh[0] / dh[1]
    assert 3.3 < ratio < 4.7, dh
    assert abs(dh[0]) < 1e-2 * abs(h0)
