"""GPU force kernel, autograd Functions and the batched graph launch against the oracle."""

import numpy as np
import pytest
import torch

from oracle import dwf_ref as R
from synth import fields as F

from gpu_util import make, need_gpu, rel, to_dev

pytestmark = pytest.mark.gpu

M5, MF = 1.8, 0.01


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def D():
    from paper_2203_06777_amd import dwf

    return dwf


# ---------------------------------------------------------------------------
# Force kernel
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("dims,ls", [((4, 4, 4, 4), 4), ((2, 4, 2, 6), 3), ((2, 2, 4, 2), 64)])
def test_force_kernel(kind, dims, ls):
    op, u = make(dims, ls, seed_u=51)
    x = F.fermion_full(dims, ls, 52)
    y = F.fermion_full(dims, ls, 53)
    xi, yi = op.pack(to_dev(x), 2, "f64"), op.pack(to_dev(y), 2, "f64")
    f = torch.empty(u.shape, dtype=torch.complex128, device="cuda")
    D().dwf_force(op.handle, f, xi, yi, kind, 0.7)
    want = 0.7 * (R.force_euclid(u, x, y) if kind == 0 else R.force_su3(u, x, y))
    assert rel(f.cpu().numpy(), want) <= 1e-13


# ---------------------------------------------------------------------------
# Autograd
# ---------------------------------------------------------------------------
def test_dwf_op_gradcheck():
    from paper_2203_06777_amd.autograd import dwf_op

    dims, ls = (2, 2, 2, 2), 4
    u0 = F.gauge_field(dims, 0.5, 61)
    op = D().Context(dims, ls, M5, MF)
    U = torch.from_numpy(u0).cuda().requires_grad_(True)
    x = torch.from_numpy(F.fermion_full(dims, ls, 62)).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: dwf_op(op, a, b), (U, x), eps=1e-6, atol=1e-7, rtol=1e-6,
                                    fast_mode=True)


def test_dwf_op_backward_matches_oracle():
    from paper_2203_06777_amd.autograd import dwf_op

    dims, ls = (4, 2, 2, 4), 3
    u0 = F.gauge_field(dims, 0.5, 63)
    x0 = F.fermion_full(dims, ls, 64)
    g0 = F.fermion_full(dims, ls, 65)
    op = D().Context(dims, ls, M5, MF)
    U = torch.from_numpy(u0).cuda().requires_grad_(True)
    x = torch.from_numpy(x0).cuda().requires_grad_(True)
    y = dwf_op(op, U, x)
    assert rel(y.detach().cpu().numpy(), R.ddw(u0, x0, M5, MF)) <= 1e-13
    y.backward(torch.from_numpy(g0).cuda())
    assert rel(x.grad.cpu().numpy(), R.ddw(u0, g0, M5, MF, dagger=True)) <= 1e-13
    assert rel(U.grad.cpu().numpy(), -0.5 * R.force_euclid(u0, x0, g0)) <= 1e-13


def test_dwf_action_gradcheck():
    from paper_2203_06777_amd.autograd import dwf_action

    dims, ls = (2, 2, 2, 2), 4
    op = D().Context(dims, ls, M5, MF)
    U = torch.from_numpy(F.gauge_field(dims, 0.5, 66)).cuda().requires_grad_(True)
    phi = torch.from_numpy(F.fermion_full(dims, ls, 67)).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: dwf_action(op, a, b, 1e-13), (U, phi), eps=1e-6, atol=1e-6,
                                    rtol=1e-5, fast_mode=True)


def test_action_force_matches_finite_differences_16x16x16x16_ls8():
    """dS/d(eps) along 16 random su(3) directions vs central differences (h = 1e-5).

    S is evaluated with the stationary estimator 2 Re(phi^dag X) - |D X|^2, whose
    error is quadratic in the solver residual, from FP64 solves at 1e-12.
    """
    from paper_2203_06777_amd.autograd import dwf_action

    w = F.WORKLOADS["force_16^4x8"]
    dims, ls, h = w["dims"], w["ls"], w["h"]
    u0 = F.gauge_field(dims, w["eps"], w["seed_u"])
    phi0 = F.fermion_full(dims, ls, w["seed_phi"])
    op = D().Context(dims, ls, w["M5"], w["mf"])
    U = torch.from_numpy(u0).cuda().requires_grad_(True)
    phi = torch.from_numpy(phi0).cuda()
    s = dwf_action(op, U, phi, 1e-12)
    s.backward()
    g = U.grad.detach()
    pi = op.pack(phi, 2, "f64")

    def action(uu):
        op.set_gauge(uu)
        z = op.field("f64", full=True)
        x = op.field("f64", full=True)
        D().dwf_solve(op.handle, z, pi, 1, 1e-12, 100000, 0)
        D().dwf_solve(op.handle, x, z, 0, 1e-12, 100000, 0)
        dx = op.field("f64", full=True)
        D().dwf_dw(op.handle, dx, x, 0, "f64")
        return 2 * D().dwf_cdot(op.handle, pi, x, 1, "f64").real - D().dwf_norm2(op.handle, dx, 1, "f64")

    worst = 0.0
    for seed in w["seed_dirs"]:
        q = F.su3_directions(dims, seed)
        wv, vv = np.linalg.eigh(q)
        ep = torch.from_numpy(np.einsum("...ik,...k,...jk->...ij", vv, np.exp(1j * h * wv), vv.conj())).cuda()
        em = torch.from_numpy(np.einsum("...ik,...k,...jk->...ij", vv, np.exp(-1j * h * wv), vv.conj())).cuda()
        fd = (action(ep @ U.detach()) - action(em @ U.detach())) / (2 * h)
        # analytic: dS/deps = Re sum conj(g) (i Q U)
        dU = 1j * torch.from_numpy(q).cuda() @ U.detach()
        an = float(torch.sum(torch.conj(g) * dU).real)
        worst = max(worst, abs(fd - an) / abs(an))
    assert worst <= 1e-6, worst


# ---------------------------------------------------------------------------
# Batched graph launch
# ---------------------------------------------------------------------------
def test_batched_mixed_lattices_match_single_applies_and_oracle():
    w = F.WORKLOADS["batch_mixed"]
    ctxs, ins, outs, us, psis = [], [], [], [], []
    nrhs = []
    for lat in w["lattices"]:  # 8^4, 12^4, 16^4, 20^4
        dims, ls = lat["dims"], lat["ls"]
        op, u = make(dims, ls, w["eps"], lat["seed_u"])
        ctxs.append(op)
        us.append(u)
        nrhs.append(len(lat["rhs_seeds"]))
        for sd in lat["rhs_seeds"]:
            p = F.fermion_cb(dims, ls, sd)
            psis.append(p)
            ins.append(op.pack(to_dev(p), 0, "f32"))
            outs.append(op.zeros("f32"))
    plan = D().dwf_batch_plan([c.handle for c in ctxs], nrhs, "f32", 0)
    try:
        D().dwf_batch_capture(plan, outs, ins, 1)
        for _ in range(3):  # replays give identical results
            D().dwf_batch_launch(plan)
        torch.cuda.synchronize()
        k = 0
        for li, op in enumerate(ctxs):
            for r in range(nrhs[li]):
                single = op.field("f32")
                D().dwf_dhop(op.handle, single, ins[k], 1, 0, "f32")
                got = op.unpack(outs[k], 1, "f32").cpu().numpy()
                assert rel(got, op.unpack(single, 1, "f32").cpu().numpy()) <= 1e-7
                if op.dims[0] <= 16:
                    if r == 0:
                        assert rel(got, R.dhop_cb(us[li], psis[k], 1)) <= 1e-6
                else:  # 20^4: sampled rows of every right-hand side
                    rows = np.random.default_rng(100 + r).integers(0, got.shape[0], 256)
                    assert rel(got[rows], R.dhop_sites(us[li], psis[k], 1, rows)) <= 1e-6
                k += 1
    finally:
        D().dwf_batch_free(plan)


@pytest.mark.parametrize("prec,dagger,lattices", [
    ("f64", 1, [((4, 4, 4, 4), 8, 2), ((6, 4, 4, 4), 12, 3)]),          # mixed Ls: generic-Ls row blocks
    ("f16", 0, [((4, 4, 4, 4), 8, 1), ((8, 4, 2, 6), 4, 2)]),
    ("bf16", 1, [((4, 4, 4, 4), 8, 2), ((64, 2, 2, 2), 20, 2)]),        # a 640-lane row: site fallback
])
def test_batched_precisions_mixed_ls_and_fallback_equal_single_applies(prec, dagger, lattices):
    """Every field of a batch equals the single-field dwf_dhop bit for bit (same arithmetic order)."""
    ctxs, ins, outs, nrhs = [], [], [], []
    for i, (dims, ls, nr) in enumerate(lattices):
        op, _ = make(dims, ls, 0.5, 900 + i)
        ctxs.append(op)
        nrhs.append(nr)
        for r in range(nr):
            ins.append(op.pack(to_dev(F.fermion_cb(dims, ls, 950 + 10 * i + r)), 1, prec))
            outs.append(op.zeros(prec))
    plan = D().dwf_batch_plan([c.handle for c in ctxs], nrhs, prec, dagger)
    try:
        D().dwf_batch_capture(plan, outs, ins, 0)
        D().dwf_batch_launch(plan)
        D().dwf_batch_launch(plan)
        torch.cuda.synchronize()
        k = 0
        for li, op in enumerate(ctxs):
            for _ in range(nrhs[li]):
                single = op.zeros(prec)
                D().dwf_dhop(op.handle, single, ins[k], 0, dagger, prec)
                torch.cuda.synchronize()
                assert torch.equal(outs[k], single), (li, k)
                assert float(outs[k].float().abs().sum()) > 0
                k += 1
    finally:
        D().dwf_batch_free(plan)


def test_batched_multi_rhs_sampled_32x32x32x32_ls12():
    """12 right-hand sides on 32^4 x 12 (the batched workload): sampled rows of each RHS vs the oracle."""
    w = F.WORKLOADS["batch_32^4x12x12"]
    dims, ls = w["dims"], w["ls"]
    op, u = make(dims, ls, w["eps"], w["seed_u"])
    ins, outs, rows_want = [], [], []
    rng = np.random.default_rng(5)
    rows = rng.integers(0, 32 ** 4 // 2, 64)
    for sd in w["rhs_seeds"]:
        p = F.fermion_cb(dims, ls, sd)
        ins.append(op.pack(to_dev(p), 1, "f32"))
        outs.append(op.field("f32"))
        rows_want.append(R.dhop_sites(u, p, 0, rows))
        del p
    plan = D().dwf_batch_plan([op.handle], [len(ins)], "f32", 0)
    try:
        D().dwf_batch_capture(plan, outs, ins, 0)
        D().dwf_batch_launch(plan)
        torch.cuda.synchronize()
        idx = torch.from_numpy(rows).cuda()
        for k in range(len(ins)):
            got = op.unpack(outs[k], 0, "f32")[idx].cpu().numpy()
            assert rel(got, rows_want[k]) <= 1e-6
    finally:
        D().dwf_batch_free(plan)
    del ins, outs
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# ABI behaviour
# ---------------------------------------------------------------------------
def test_abi_errors_and_no_allocation_in_dhop():
    dims, ls = (4, 4, 4, 4), 8
    dw = D()
    with pytest.raises(dw.DwfError) as e:
        dw.dwf_create((4, 4, 3, 4), 8)
    assert e.value.code == -1
    with pytest.raises(dw.DwfError):
        dw.dwf_create((4, 4, 4, 4), 0)
    op = dw.Context(dims, ls)
    f = op.zeros("f32")
    g = op.zeros("f32")
    with pytest.raises(dw.DwfError) as e:  # gauge not set yet
        dw.dwf_dhop(op.handle, g, f, 0, 0, "f32")
    assert e.value.code == -6
    op.set_gauge(torch.from_numpy(F.unit_gauge(dims)).cuda())
    with pytest.raises(dw.DwfError):
        dw.dwf_dhop(op.handle, f, f, 0, 0, "f32")  # aliasing
    with pytest.raises(dw.DwfError):
        dw.dwf_dhop(op.handle, g, f, 2, 0, "f32")  # parity
    with pytest.raises(dw.DwfError):
        dw.dwf_dhop(op.handle, g, f, 0, 0, 7)  # precision
    with pytest.raises(dw.DwfError):
        dw.dwf_dhop(op.handle, g, 0, 0, 0, "f32")  # null
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(5):
        dw.dwf_dhop(op.handle, g, f, 1, 0, "f32")
        dw.dwf_mdagm(op.handle, g, f, "f32")
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free0 == free1


def test_tuner_keeps_results_identical():
    dims, ls = (8, 8, 8, 8), 16
    op, u = make(dims, ls, seed_u=71)
    p = F.fermion_cb(dims, ls, 72)
    pin = op.pack(to_dev(p), 0, "f32")
    a, b = op.field("f32"), op.field("f32")
    D().dwf_dhop(op.handle, a, pin, 1, 0, "f32")
    us = D().dwf_tune(op.handle, "f32", 0)
    assert us > 0
    D().dwf_dhop(op.handle, b, pin, 1, 0, "f32")
    assert torch.equal(a, b)


@pytest.mark.parametrize("prec", ["f64", "f16"])
def test_tuner_keeps_schur_operator_and_cg_identical(prec):
    """The fused Schur kernels get their own tuned shape; M_pc^dag M_pc and a CG solve are bitwise
    unchanged by tuning (every candidate shape is checked to give the same bits)."""
    dims, ls = (8, 8, 4, 8), 12
    op, u = make(dims, ls, seed_u=73)
    p = F.fermion_cb(dims, ls, 74)
    pin = op.pack(to_dev(p), 1, prec)
    a, b = op.field(prec), op.field(prec)
    D().dwf_mdagm(op.handle, a, pin, prec)
    bsrc = op.pack(to_dev(p), 1, "f64")
    x0 = op.zeros("f64")
    mode = 0 if prec == "f64" else 2
    D().dwf_cg(op.handle, x0, bsrc, 1e-10, 5000, mode)
    for dag in (0, 1):
        assert D().dwf_tune(op.handle, prec, dag) > 0
    D().dwf_mdagm(op.handle, b, pin, prec)
    x1 = op.zeros("f64")
    D().dwf_cg(op.handle, x1, bsrc, 1e-10, 5000, mode)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # CG: partial sums are per workgroup, so a different shape may reorder the FP64 reductions;
    # the solution must still agree to the solver tolerance
    d = op.field("f64")
    d.copy_(x1)
    D().dwf_axpy(op.handle, d, -1.0, x0, 0, "f64")
    assert np.sqrt(D().dwf_norm2(op.handle, d, 0, "f64") / D().dwf_norm2(op.handle, x0, 0, "f64")) <= 1e-8
