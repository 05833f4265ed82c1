"""GPU parity of the hopping term, the M5op family, the Schur operator and the
BLAS-1 reductions against the CPU oracle, through the C ABI."""

import numpy as np
import pytest
import torch

from oracle import coracle as C
from oracle import dwf_ref as R
from synth import fields as F

from gpu_util import TOL, make, need_gpu, rel, to_dev

pytestmark = pytest.mark.gpu

M5, MF = 1.8, 0.01


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def D():
    from paper_2203_06777_amd import dwf

    return dwf


# ---------------------------------------------------------------------------
# Hopping term
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("par,dag", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_dhop_4x4x4x4_ls8(prec, par, dag):
    w = F.WORKLOADS["dwf_4^4x8"]
    op, u = make(w["dims"], w["ls"], w["eps"], w["seed_u"])
    psi = F.fermion_cb(w["dims"], w["ls"], w["seed_psi"])
    pin = op.pack(to_dev(psi), 1 - par, prec)
    out = op.field(prec)
    D().dwf_dhop(op.handle, out, pin, par, dag, prec)
    got = op.unpack(out, par, prec).cpu().numpy()
    want = R.dhop_cb(u, psi, par, bool(dag))
    assert rel(got, want) <= TOL[prec]


@pytest.mark.parametrize("dims,ls", [((2, 2, 2, 2), 4), ((6, 4, 2, 8), 3), ((4, 2, 6, 2), 1), ((6, 6, 6, 6), 16),
                                     ((8, 8, 8, 8), 12), ((2, 4, 2, 2), 20), ((4, 4, 4, 4), 64)])
@pytest.mark.parametrize("dag", [0, 1])
def test_dhop_shapes_and_ragged_tails(dims, ls, dag):
    op, u = make(dims, ls, seed_u=7)
    psi = F.fermion_cb(dims, ls, 8)
    for par in (0, 1):
        pin = op.pack(to_dev(psi), 1 - par, "f64")
        out = op.field("f64")
        D().dwf_dhop(op.handle, out, pin, par, dag, "f64")
        got = op.unpack(out, par, "f64").cpu().numpy()
        assert rel(got, C.dhop_cb(u, psi, par, dag)) <= TOL["f64"]


def test_dhop_periodic_time_and_pack_roundtrip():
    dims, ls = (4, 4, 2, 6), 5
    op, u = make(dims, ls, seed_u=9, antiperiodic=False)
    psi = F.fermion_cb(dims, ls, 10)
    for prec in ("f64", "f32"):
        pin = op.pack(to_dev(psi), 0, prec)
        back = op.unpack(pin, 0, prec).cpu().numpy()
        assert rel(back, psi) <= (0 if prec == "f64" else 1e-7)
    pin = op.pack(to_dev(psi), 0, "f64")
    out = op.field("f64")
    D().dwf_dhop(op.handle, out, pin, 1, 0, "f64")
    got = op.unpack(out, 1, "f64").cpu().numpy()
    assert rel(got, R.dhop_cb(u, psi, 1, False, antiperiodic_t=False)) <= 1e-13
    full = F.fermion_full(dims, ls, 11)
    fi = op.pack(to_dev(full), 2, "f64")
    assert np.array_equal(op.unpack(fi, 2, "f64").cpu().numpy(), full)
    e, o = op.halves(fi)
    assert np.array_equal(op.unpack(e.contiguous(), 0, "f64").cpu().numpy(), R.full_to_cb(full, 0))
    assert np.array_equal(op.unpack(o.contiguous(), 1, "f64").cpu().numpy(), R.full_to_cb(full, 1))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_dhop_16x16x16x16_ls16(prec):
    w = F.WORKLOADS["dhop_16^4x16"]
    op, u = make(w["dims"], w["ls"], w["eps"], w["seed_u"])
    psi = F.fermion_cb(w["dims"], w["ls"], w["seed_psi"])
    for par, dag in ((0, 0), (1, 0), (1, 1)):
        pin = op.pack(to_dev(psi), 1 - par, prec)
        out = op.field(prec)
        D().dwf_dhop(op.handle, out, pin, par, dag, prec)
        got = op.unpack(out, par, prec).cpu().numpy()
        assert rel(got, C.dhop_cb(u, psi, par, dag)) <= TOL[prec]


@pytest.fixture(scope="module")
def headline_32():
    """The timed workload (32^4 x 16): context, links and input, plus sampled rows of both parities."""
    w = F.WORKLOADS["dhop_32^4x16"]
    dims, ls = w["dims"], w["ls"]
    op, u = make(dims, ls, w["eps"], w["seed_u"])
    psi = F.fermion_cb(dims, ls, w["seed_psi"])
    rng = np.random.default_rng(0)
    rows = np.unique(np.concatenate([rng.integers(0, psi.shape[0], 600), [0, psi.shape[0] - 1]]))
    want = {par: R.dhop_sites(u, psi, par, rows) for par in (0, 1)}
    yield op, psi, rows, want
    op.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["f32", "f64", "f16", "bf16"])
def test_dhop_32x32x32x32_ls16_sampled(headline_32, prec):
    """Headline shape, every precision, both output parities (the launches the bench times):
    sampled output rows against the site-wise oracle."""
    op, psi, rows, want = headline_32
    idx = torch.from_numpy(rows).cuda()
    for par in (0, 1):
        pin = op.pack(to_dev(psi), 1 - par, prec)
        out = op.field(prec)
        D().dwf_dhop(op.handle, out, pin, par, 0, prec)
        got = op.unpack(out, par, prec)[idx].cpu().numpy()
        assert rel(got, want[par]) <= TOL[prec], (prec, par)
        del pin, out


# ---------------------------------------------------------------------------
# M5op family, Schur operator, full operator
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("ls", [1, 5, 8, 12, 16])
def test_m5_family(prec, ls):
    dims = (4, 4, 2, 2)
    op, _ = make(dims, ls)
    psi = F.fermion_cb(dims, ls, 3)
    for dag in (0, 1):
        for inv in (0, 1):
            pin = op.pack(to_dev(psi), 0, prec)
            out = op.field(prec)
            D().dwf_m5(op.handle, out, pin, dag, inv, 0, prec)
            got = op.unpack(out, 0, prec).cpu().numpy()
            want = (R.m5inv if inv else R.m5op)(psi, M5, MF, bool(dag))
            assert rel(got, want) <= TOL[prec]
            # in place
            D().dwf_m5(op.handle, pin, pin, dag, inv, 0, prec)
            assert rel(op.unpack(pin, 0, prec).cpu().numpy(), want) <= TOL[prec]


def test_m5_full_field():
    dims, ls = (4, 2, 2, 4), 6
    op, _ = make(dims, ls)
    full = F.fermion_full(dims, ls, 4)
    fi = op.pack(to_dev(full), 2, "f64")
    out = op.field("f64", full=True)
    D().dwf_m5(op.handle, out, fi, 0, 1, 1, "f64")
    assert rel(op.unpack(out, 2, "f64").cpu().numpy(), R.m5inv(full, M5, MF)) <= 1e-13


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_mpc_and_mdagm(prec):
    dims, ls = (4, 4, 4, 4), 8
    op, u = make(dims, ls, seed_u=12)
    psi = F.fermion_cb(dims, ls, 13)
    pin = op.pack(to_dev(psi), 1, prec)
    out = op.field(prec)
    for dag in (0, 1):
        D().dwf_mpc(op.handle, out, pin, dag, prec)
        assert rel(op.unpack(out, 1, prec).cpu().numpy(), R.mpc(u, psi, M5, MF, bool(dag))) <= TOL[prec]
    D().dwf_mdagm(op.handle, out, pin, prec)
    assert rel(op.unpack(out, 1, prec).cpu().numpy(), R.mdagm(u, psi, M5, MF)) <= TOL[prec]


@pytest.mark.parametrize("dag", [0, 1])
def test_full_dwf_operator(dag):
    dims, ls = (4, 4, 2, 4), 6
    op, u = make(dims, ls, seed_u=14)
    full = F.fermion_full(dims, ls, 15)
    fi = op.pack(to_dev(full), 2, "f64")
    out = op.field("f64", full=True)
    D().dwf_dw(op.handle, out, fi, dag, "f64")
    assert rel(op.unpack(out, 2, "f64").cpu().numpy(), R.ddw(u, full, M5, MF, bool(dag))) <= 1e-13


# ---------------------------------------------------------------------------
# BLAS-1 and FP64 reductions
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_norm_dot_axpy(prec):
    dims, ls = (6, 4, 4, 2), 7
    op, _ = make(dims, ls)
    a = F.fermion_cb(dims, ls, 21)
    b = F.fermion_cb(dims, ls, 22)
    ai, bi = op.pack(to_dev(a), 0, prec), op.pack(to_dev(b), 0, prec)
    # exact reference: what the stored (rounded) values give in FP64
    ar = op.unpack(ai, 0, prec).cpu().numpy()
    br = op.unpack(bi, 0, prec).cpu().numpy()
    n2 = D().dwf_norm2(op.handle, ai, 0, prec)
    assert abs(n2 - np.vdot(ar, ar).real) <= 1e-12 * n2
    dt = D().dwf_cdot(op.handle, ai, bi, 0, prec)
    want = np.vdot(ar, br)
    assert abs(dt - want) <= 1e-12 * np.sqrt(n2 * np.vdot(br, br).real)
    # deterministic: bitwise identical on repeat
    assert D().dwf_norm2(op.handle, ai, 0, prec) == n2
    D().dwf_axpy(op.handle, bi, 0.3 - 0.7j, ai, 0, prec)
    got = op.unpack(bi, 0, prec).cpu().numpy()
    # one round-to-nearest of the FP32 result: |error| <= 2^-p |value| per element (p = 11 / 8
    # significand bits for FP16 / BF16), so the rel-L2 error is at most 2^-p
    assert rel(got, (0.3 - 0.7j) * ar + br) <= {"f64": 1e-15, "f32": 2e-7, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}[prec]
