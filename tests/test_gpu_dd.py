"""GPU domain-decomposed hopping term (t-direction faces, exchange, interior /
exterior split) against dwf_dhop and the oracle, all precisions, both parities
and daggers, ragged shapes, Lt = 2, repeated calls, and the argument checks."""

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


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("dims,ls", [((4, 4, 2, 6), 5), ((4, 2, 2, 2), 3), ((8, 4, 4, 8), 8)])
def test_dd_dhop_equals_dhop_and_oracle(prec, dims, ls):
    op, u = make(dims, ls, seed_u=901)
    dd = D().dwf_dd_create(op.handle, prec)
    for par in (0, 1):
        psi = F.fermion_cb(dims, ls, 902 + par)
        pin = op.pack(to_dev(psi), 1 - par, prec)
        for dag in (0, 1):
            want = op.field(prec)
            got = op.field(prec)
            D().dwf_dhop(op.handle, want, pin, par, dag, prec)
            D().dwf_dd_dhop(dd, got, pin, par, dag)
            g = op.unpack(got, par, prec).cpu().numpy()
            w = op.unpack(want, par, prec).cpu().numpy()
            # only the boundary sites' last addition differs (for 16-bit storage also the
            # rounding of the interior result before it)
            assert rel(g, w) <= {"f64": 1e-15, "f32": 1e-6}.get(prec, TOL[prec])
            assert rel(g, R.dhop_cb(u, psi, par, bool(dag))) <= TOL[prec]
    D().dwf_dd_destroy(dd)
    op.close()


def test_dd_repeated_calls_and_errors():
    dims, ls = (4, 4, 4, 4), 4
    op, u = make(dims, ls, seed_u=911)
    dd = D().dwf_dd_create(op.handle, "f32")
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
    D().dwf_dd_faces(dd, x, 0)
    torch.cuda.synchronize()
    D().dwf_dd_destroy(dd)
    op.close()


def test_dd_32x32x32x32_ls16_f32_sampled():
    """The timed shape: the decomposed apply equals dwf_dhop and, on sampled rows (including
    both boundary slices), the site-wise oracle."""
    w = F.WORKLOADS["dhop_32^4x16"]
    dims, ls = w["dims"], w["ls"]
    op, u = make(dims, ls, w["eps"], w["seed_u"])
    psi = F.fermion_cb(dims, ls, w["seed_psi"])
    S = psi.shape[0] // dims[3]
    rng = np.random.default_rng(1)
    rows = np.unique(np.concatenate([rng.integers(0, psi.shape[0], 300), rng.integers(0, S, 100),
                                     rng.integers(psi.shape[0] - S, psi.shape[0], 100)]))
    pin = op.pack(to_dev(psi), 0, "f32")
    dd = D().dwf_dd_create(op.handle, "f32")
    got, want = op.field("f32"), op.field("f32")
    D().dwf_dd_dhop(dd, got, pin, 1, 0)
    D().dwf_dhop(op.handle, want, pin, 1, 0, "f32")
    g = op.unpack(got, 1, "f32")
    assert rel(g.cpu().numpy(), op.unpack(want, 1, "f32").cpu().numpy()) <= 1e-6
    sel = g[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert rel(sel, R.dhop_sites(u, psi, 1, rows)) <= TOL["f32"]
    D().dwf_dd_destroy(dd)
    del pin, got, want, g
    torch.cuda.empty_cache()
    op.close()
