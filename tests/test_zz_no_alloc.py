"""The no-allocation reduction entry point (static device scratch) against dwf_cdot and
dwf_norm2, through the C ABI: two calls in a row, the second on a smaller field."""

import numpy as np
import pytest
import torch

from synth import fields as F

from gpu_util import make, need_gpu, to_dev

pytestmark = pytest.mark.gpu


def D():
    from paper_2203_06777_amd import dwf

    return dwf


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_cdot_noalloc_equals_cdot_and_norm2(prec):
    need_gpu()
    res = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    # the second call works on a smaller field than the first (the static partials are reused)
    for dims, ls, seed, full in (((8, 8, 4, 4), 8, 61, 1), ((4, 4, 2, 2), 4, 62, 0)):
        op, _ = make(dims, ls, seed_u=seed)
        par = 2 if full else 0
        mk = F.fermion_full if full else F.fermion_cb
        x = op.pack(to_dev(mk(dims, ls, seed + 100)), par, prec)
        y = op.pack(to_dev(mk(dims, ls, seed + 200)), par, prec)
        want = D().dwf_cdot(op.handle, x, y, full, prec)
        res.fill_(float("nan"))
        D().dwf_cdot_noalloc(op.handle, res, x, y, full, prec)
        torch.cuda.synchronize()
        got = res.cpu().numpy()
        assert got[0] == want.real and got[1] == want.imag, (got, want)
        n2 = D().dwf_norm2(op.handle, x, full, prec)
        res.fill_(float("nan"))
        D().dwf_cdot_noalloc(op.handle, res, x, None, full, prec)
        torch.cuda.synchronize()
        got = res.cpu().numpy()
        assert got[0] == n2 and got[1] == 0.0, (got, n2)
        # and both agree with the FP64 inner product of the stored values
        xr = op.unpack(x, par, prec).cpu().numpy()
        yr = op.unpack(y, par, prec).cpu().numpy()
        ref = np.vdot(xr, yr)
        assert abs(complex(want) - ref) <= 1e-12 * np.linalg.norm(xr) * np.linalg.norm(yr)
        op.close()


def test_cdot_noalloc_rejects_bad_arguments():
    need_gpu()
    dims, ls = (4, 4, 2, 2), 4
    op, _ = make(dims, ls, seed_u=63)
    x = op.zeros("f32")
    res = torch.zeros(2, dtype=torch.float64, device="cuda")
    lib = D().lib()
    assert lib.dwf_cdot_noalloc(op.handle, None, x.data_ptr(), None, 0, 1, None) == -1
    assert lib.dwf_cdot_noalloc(op.handle, res.data_ptr(), None, None, 0, 1, None) == -1
    assert lib.dwf_cdot_noalloc(op.handle, res.data_ptr(), x.data_ptr(), None, 0, 7, None) == -1
    assert lib.dwf_cdot_noalloc(op.handle, res.data_ptr(), x.data_ptr(), None, 3, 1, None) == -1
    assert lib.dwf_cdot_noalloc(None, res.data_ptr(), x.data_ptr(), None, 0, 1, None) == -1
    op.close()
