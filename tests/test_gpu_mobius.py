"""GPU Moebius (Cayley) operator against the oracle: Mooee and its inverse,
M_pc, M_pc^dag M_pc, the full operator, CG in every mode and the full solve,
the switch back to Shamir, and the error paths of dwf_set_mobius."""

import numpy as np
import pytest
import torch

from oracle import dwf_ref as R
from synth import fields as F

from gpu_util import TOL, make, need_gpu, rel, to_dev

pytestmark = pytest.mark.gpu

M5, MF = 1.8, 0.01
B, C = 1.5, 0.5  # b - c = 1, b + c = 2


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def D():
    from paper_2203_06777_amd import dwf

    return dwf


def make_mob(dims, ls, seed_u, b=B, c=C):
    op, u = make(dims, ls, seed_u=seed_u)
    op.set_mobius(b, c)
    return op, u


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_mooee_family(prec):
    dims, ls = (4, 2, 2, 6), 7
    op, _ = make_mob(dims, ls, 201)
    psi = F.fermion_cb(dims, ls, 202)
    for dag in (0, 1):
        for inv in (0, 1):
            pin = op.pack(to_dev(psi), 0, prec)
            out = op.field(prec)
            D().dwf_m5(op.handle, out, pin, dag, inv, 0, prec)
            want = (R.mooee_inv if inv else R.mooee)(psi, M5, MF, B, C, bool(dag))
            assert rel(op.unpack(out, 0, prec).cpu().numpy(), want) <= TOL[prec]
            D().dwf_m5(op.handle, pin, pin, dag, inv, 0, prec)  # in place
            assert rel(op.unpack(pin, 0, prec).cpu().numpy(), want) <= TOL[prec]
    op.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_mobius_mpc_and_mdagm(prec):
    dims, ls = (4, 4, 4, 4), 8
    op, u = make_mob(dims, ls, 211)
    psi = F.fermion_cb(dims, ls, 212)
    pin = op.pack(to_dev(psi), 1, prec)
    out = op.field(prec)
    for dag in (0, 1):
        D().dwf_mpc(op.handle, out, pin, dag, prec)
        want = R.mobius_mpc(u, psi, M5, MF, B, C, bool(dag))
        assert rel(op.unpack(out, 1, prec).cpu().numpy(), want) <= TOL[prec]
    D().dwf_mdagm(op.handle, out, pin, prec)
    assert rel(op.unpack(out, 1, prec).cpu().numpy(), R.mobius_mdagm(u, psi, M5, MF, B, C)) <= TOL[prec]
    op.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dag", [0, 1])
def test_mobius_full_operator(prec, dag):
    dims, ls = (4, 2, 4, 2), 5
    op, u = make_mob(dims, ls, 221, b=2.0, c=1.0)
    psi = F.fermion_full(dims, ls, 222)
    pin = op.pack(to_dev(psi), 2, prec)
    out = op.field(prec, full=True)
    D().dwf_dw(op.handle, out, pin, dag, prec)
    want = R.mobius_ddw(u, psi, M5, MF, 2.0, 1.0, bool(dag))
    assert rel(op.unpack(out, 2, prec).cpu().numpy(), want) <= TOL[prec]
    op.close()


@pytest.fixture(scope="module")
def cg_case():
    """4^4 x 8 right-hand side and the oracle's FP64 CG solution (computed once)."""
    dims, ls = (4, 4, 4, 4), 8
    u = F.gauge_field(dims, 0.5, 231)
    b = F.fermion_cb(dims, ls, 232)
    want, _, res = R.cg(lambda v: R.mobius_mdagm(u, v, M5, MF, B, C), b, 1e-12, 5000)
    assert res <= 1e-12
    return dims, ls, u, b, want


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_mobius_cg_matches_oracle_cg(mode, cg_case):
    """Every mode reaches the oracle's FP64 CG solution of the Moebius normal equations."""
    dims, ls, u, b, want = cg_case
    op, _ = make_mob(dims, ls, 231)

    def a(v):
        return R.mobius_mdagm(u, v, M5, MF, B, C)

    bi = op.pack(to_dev(b), 1, "f64")
    x = op.zeros("f64")
    st = D().dwf_cg(op.handle, x, bi, 1e-10, 5000, mode)
    got = op.unpack(x, 1, "f64").cpu().numpy()
    assert st["true_rel_resid"] <= 1e-10
    assert np.linalg.norm(b - a(got)) / np.linalg.norm(b) <= 1.5e-10
    assert rel(got, want) <= 1e-8
    op.close()


@pytest.mark.parametrize("dag", [0, 1])
@pytest.mark.parametrize("mode", [0, 2])
def test_mobius_full_solve(dag, mode):
    dims, ls = (4, 4, 2, 4), 6
    op, u = make_mob(dims, ls, 241)
    b = F.fermion_full(dims, ls, 242)
    bi = op.pack(to_dev(b), 2, "f64")
    x = op.zeros("f64", full=True)
    D().dwf_solve(op.handle, x, bi, dag, 1e-11, 5000, mode)
    got = op.unpack(x, 2, "f64").cpu().numpy()
    r = R.mobius_ddw(u, got, M5, MF, B, C, bool(dag)) - b
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-9
    op.close()


def test_switch_back_to_shamir_is_bitwise_identical():
    dims, ls = (4, 4, 4, 4), 8
    psi = to_dev(F.fermion_cb(dims, ls, 252))
    ref, _ = make(dims, ls, seed_u=251)
    pin = ref.pack(psi, 1, "f32")
    want = ref.field("f32")
    D().dwf_mdagm(ref.handle, want, pin, "f32")
    op, _ = make_mob(dims, ls, 251)
    got = op.field("f32")
    D().dwf_mdagm(op.handle, got, pin, "f32")
    assert not torch.equal(got, want)
    op.set_mobius(1.0, 0.0)
    assert not op.mobius
    D().dwf_mdagm(op.handle, got, pin, "f32")
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    op.close()
    ref.close()


def test_set_mobius_errors_and_autograd_refusal():
    from paper_2203_06777_amd import autograd as AG

    dims, ls = (2, 2, 2, 2), 4
    op, u = make(dims, ls, seed_u=261)
    with pytest.raises(D().DwfError):
        D().dwf_set_mobius(op.handle, float("nan"), 0.0)
    with pytest.raises(D().DwfError):
        D().dwf_set_mobius(op.handle, 1.0, 1.0 / (4.0 - M5))  # e = 0
    assert D().dwf_get_mobius(op.handle) == (1.0, 0.0)
    op.set_mobius(B, C)
    assert D().dwf_get_mobius(op.handle) == (B, C) and op.mobius
    U = torch.from_numpy(u).cuda()
    x = to_dev(F.fermion_full(dims, ls, 262))
    with pytest.raises(NotImplementedError):
        AG.dwf_op(op, U, x)
    op.close()
