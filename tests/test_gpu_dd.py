"""GPU domain-decomposed hopping term (faces of every cut direction assembled in one kernel,
exchange, interior-only launch, exterior sites computed from the faces) against dwf_dhop (bit
for bit) and the oracle, all precisions, both parities and daggers, each single cut, the
2x2x2x1 split (x, y, z cut) and all four cuts, ragged shapes, extent-2 directions, repeated
calls, and the argument checks."""

import numpy as np
import pytest
import torch

from oracle import dwf_ref as R
from synth import fields as F

from gpu_util import TOL, make, need_gpu, rel, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def D():
    from paper_2203_06777_amd import dwf

    return dwf


CUTS = ["x", "y", "z", "t", "xyz", "xyzt"]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("cuts", CUTS)
@pytest.mark.parametrize("dims,ls", [((4, 4, 2, 6), 5), ((8, 4, 4, 8), 8)])
def test_dd_dhop_equals_dhop_and_oracle(prec, cuts, dims, ls):
    op, u = make(dims, ls, seed_u=901)
    dd = D().dwf_dd_create(op.handle, prec, cuts)
    for par in (0, 1):
        psi = F.fermion_cb(dims, ls, 902 + par)
        pin = op.pack(to_dev(psi), 1 - par, prec)
        for dag in (0, 1):
            want = op.zeros(prec)
            got = op.zeros(prec)
            D().dwf_dhop(op.handle, want, pin, par, dag, prec)
            D().dwf_dd_dhop(dd, got, pin, par, dag)
            torch.cuda.synchronize()
            # same projections, link multiplies and accumulation order as dwf_dhop
            assert torch.equal(got, want), (prec, cuts, par, dag)
            assert rel(op.unpack(got, par, prec).cpu().numpy(), R.dhop_cb(u, psi, par, bool(dag))) <= TOL[prec]
    D().dwf_dd_destroy(dd)
    op.close()


@pytest.mark.parametrize("cuts", ["xyzt", "xz"])
@pytest.mark.parametrize("dims,ls", [((2, 2, 2, 2), 4), ((2, 6, 2, 4), 3), ((6, 2, 4, 2), 1)])
def test_dd_extent_two_and_ragged(cuts, dims, ls):
    """Directions of extent 2 (every site on both faces of that cut), odd Ls, Ls = 1."""
    op, u = make(dims, ls, seed_u=905)
    dd = D().dwf_dd_create(op.handle, "f64", cuts)
    for par in (0, 1):
        psi = F.fermion_cb(dims, ls, 906 + par)
        pin = op.pack(to_dev(psi), 1 - par, "f64")
        for dag in (0, 1):
            want, got = op.zeros("f64"), op.zeros("f64")
            D().dwf_dhop(op.handle, want, pin, par, dag, "f64")
            D().dwf_dd_dhop(dd, got, pin, par, dag)
            torch.cuda.synchronize()
            assert torch.equal(got, want)
            assert rel(op.unpack(got, par, "f64").cpu().numpy(), R.dhop_cb(u, psi, par, bool(dag))) <= 1e-13
    D().dwf_dd_destroy(dd)
    op.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("cuts", ["t", "xyzt"])
def test_dd_rows_too_long_for_the_row_kernel(prec, cuts):
    """x-rows of 32 sites x Ls 17 (544 lanes) exceed a row workgroup: every boundary site goes to
    the site kernel, which reads the FP32 / FP64 faces from the ghost sites."""
    dims, ls = (64, 2, 2, 4), 17
    op, u = make(dims, ls, seed_u=907)
    dd = D().dwf_dd_create(op.handle, prec, cuts)
    for par in (0, 1):
        psi = F.fermion_cb(dims, ls, 908 + par)
        pin = op.pack(to_dev(psi), 1 - par, prec)
        for dag in (0, 1):
            want, got = op.zeros(prec), op.zeros(prec)
            D().dwf_dhop(op.handle, want, pin, par, dag, prec)
            D().dwf_dd_dhop(dd, got, pin, par, dag)
            torch.cuda.synchronize()
            assert torch.equal(got, want), (prec, cuts, par, dag)
            assert rel(op.unpack(got, par, prec).cpu().numpy(), R.dhop_cb(u, psi, par, bool(dag))) <= TOL[prec]
    D().dwf_dd_destroy(dd)
    op.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("cuts", ["t", "yz", "yzt"])
def test_dd_whole_row_interior(prec, cuts):
    """x-rows of 16 sites x Ls 16 (one row per workgroup) and no x cut: the interior launch that
    stores every site of the rows it keeps."""
    dims, ls = (32, 4, 2, 4), 16
    op, u = make(dims, ls, seed_u=911)
    dd = D().dwf_dd_create(op.handle, prec, cuts)
    for par in (0, 1):
        psi = F.fermion_cb(dims, ls, 912 + par)
        pin = op.pack(to_dev(psi), 1 - par, prec)
        for dag in (0, 1):
            want, got = op.zeros(prec), op.zeros(prec)
            D().dwf_dhop(op.handle, want, pin, par, dag, prec)
            D().dwf_dd_dhop(dd, got, pin, par, dag)
            torch.cuda.synchronize()
            assert torch.equal(got, want), (prec, cuts, par, dag)
            assert rel(op.unpack(got, par, prec).cpu().numpy(), R.dhop_cb(u, psi, par, bool(dag))) <= TOL[prec]
    D().dwf_dd_destroy(dd)
    op.close()


def test_dd_repeated_calls_and_errors():
    dims, ls = (4, 4, 4, 4), 4
    op, u = make(dims, ls, seed_u=911)
    dd = D().dwf_dd_create(op.handle, "f32", "xyz")
    outs, ins = [], []
    for k in range(3):  # back-to-back calls reuse the face buffers
        psi = F.fermion_cb(dims, ls, 912 + k)
        ins.append(psi)
        pin = op.pack(to_dev(psi), 0, "f32")
        out = op.field("f32")
        D().dwf_dd_dhop(dd, out, pin, 1, k % 2)
        outs.append(out)
    for k in range(3):
        got = op.unpack(outs[k], 1, "f32").cpu().numpy()
        assert rel(got, R.dhop_cb(u, ins[k], 1, bool(k % 2))) <= 1e-6
    x = op.field("f32")
    with pytest.raises(D().DwfError):
        D().dwf_dd_dhop(dd, x, x, 0, 0)
    with pytest.raises(D().DwfError):
        D().dwf_dd_dhop(dd, op.field("f32"), x, 2, 0)
    with pytest.raises(D().DwfError):
        D().dwf_dd_faces(dd, x, 3, 0)
    D().dwf_dd_faces(dd, x, 1, 0)
    torch.cuda.synchronize()
    D().dwf_dd_destroy(dd)
    for bad in (0, 16, -1):
        with pytest.raises(D().DwfError):
            D().dwf_dd_create(op.handle, "f32", bad)
    op.close()


def test_dd_follows_a_gauge_change():
    """The plan reads the context's links at every apply: a new gauge needs no new plan."""
    dims, ls = (4, 4, 2, 4), 4
    op, _ = make(dims, ls, seed_u=915)
    dd = D().dwf_dd_create(op.handle, "f64", "xt")
    u2 = F.gauge_field(dims, 0.5, 916)
    op.set_gauge(to_dev(u2))
    psi = F.fermion_cb(dims, ls, 917)
    pin = op.pack(to_dev(psi), 0, "f64")
    got = op.zeros("f64")
    D().dwf_dd_dhop(dd, got, pin, 1, 0)
    assert rel(op.unpack(got, 1, "f64").cpu().numpy(), R.dhop_cb(u2, psi, 1)) <= 1e-13
    D().dwf_dd_destroy(dd)
    op.close()


@pytest.mark.parametrize("cuts", ["t", "xyz"])
def test_dd_32x32x32x32_ls16_f32(cuts):
    """The timed shape and launch configuration: the decomposed apply equals dwf_dhop bit for bit
    and, on sampled rows including every face of the 2x2x2x1 split, the site-wise oracle."""
    w = F.WORKLOADS["dhop_32^4x16"]
    dims, ls = w["dims"], w["ls"]
    op, u = make(dims, ls, w["eps"], w["seed_u"])
    psi = F.fermion_cb(dims, ls, w["seed_psi"])
    S = psi.shape[0] // dims[3]
    rng = np.random.default_rng(1)
    # sampled rows: random, the t = 0 and t = Lt-1 slices, and rows with y or z on a face
    yz_face = [c for c in rng.integers(0, psi.shape[0], 4000)
               if (c // 16) % 32 in (0, 31) or (c // (16 * 32)) % 32 in (0, 31)][:150]
    x_face = [c for c in rng.integers(0, psi.shape[0] // 16, 200) * 16 + rng.choice([0, 15], 200)][:100]
    rows = np.unique(np.concatenate([rng.integers(0, psi.shape[0], 200), rng.integers(0, S, 60),
                                     rng.integers(psi.shape[0] - S, psi.shape[0], 60), yz_face, x_face]))
    pin = op.pack(to_dev(psi), 0, "f32")
    dd = D().dwf_dd_create(op.handle, "f32", cuts)
    got, want = op.zeros("f32"), op.zeros("f32")
    D().dwf_dd_dhop(dd, got, pin, 1, 0)
    D().dwf_dhop(op.handle, want, pin, 1, 0, "f32")
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    sel = op.unpack(got, 1, "f32")[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert rel(sel, R.dhop_sites(u, psi, 1, rows)) <= TOL["f32"]
    D().dwf_dd_destroy(dd)
    del pin, got, want
    torch.cuda.empty_cache()
    op.close()
