"""GPU solvers against the oracle: FP64 CG and defect-correction CG on
M_pc^dag M_pc, the Schur-preconditioned full solve, determinism, error codes."""

import numpy as np
import pytest
import torch

from oracle import coracle as C
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


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_cg_small_matches_oracle_cg(mode):
    """4^4 x 8: every mode reaches the oracle's FP64 CG solution (rel <= 1e-8 at tol 1e-10)."""
    dims, ls = (4, 4, 4, 4), 8
    op, u = make(dims, ls, seed_u=31)
    b = F.fermion_cb(dims, ls, 32)
    want, _, res = R.cg(lambda v: R.mdagm(u, v, M5, MF), b, 1e-12, 5000)
    assert res <= 1e-12
    bi = op.pack(to_dev(b), 1, "f64")
    x = op.zeros("f64")
    st = D().dwf_cg(op.handle, x, bi, 1e-10, 5000, mode)
    got = op.unpack(x, 1, "f64").cpu().numpy()
    assert st["true_rel_resid"] <= 1e-10
    # the library's own residual claim, recomputed by the oracle
    r = b - C.mdagm(u, got, M5, MF)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.5e-10
    assert rel(got, want) <= 1e-8
    if mode:
        assert st["outer_iters"] >= 2


def test_cg_tiny_lattice_dense_solve():
    dims, ls = (2, 2, 2, 2), 4
    op, u = make(dims, ls, seed_u=33)
    b = F.fermion_cb(dims, ls, 34)
    a = R.dense_operator(lambda v: R.mdagm(u, v, M5, MF), b.shape)
    xd = np.linalg.solve(a, b.ravel()).reshape(b.shape)
    bi = op.pack(to_dev(b), 1, "f64")
    x = op.zeros("f64")
    D().dwf_cg(op.handle, x, bi, 1e-12, 2000, 0)
    assert rel(op.unpack(x, 1, "f64").cpu().numpy(), xd) <= 1e-10


def test_cg_is_deterministic_and_warm_starts():
    dims, ls = (4, 4, 4, 4), 8
    op, u = make(dims, ls, seed_u=35)
    b = F.fermion_cb(dims, ls, 36)
    bi = op.pack(to_dev(b), 1, "f64")
    x1, x2 = op.zeros("f64"), op.zeros("f64")
    s1 = D().dwf_cg(op.handle, x1, bi, 1e-10, 5000, 1)
    s2 = D().dwf_cg(op.handle, x2, bi, 1e-10, 5000, 1)
    assert torch.equal(x1, x2)
    assert s1["inner_iters"] == s2["inner_iters"]
    s3 = D().dwf_cg(op.handle, x1, bi, 1e-10, 5000, 0)  # warm start at the solution
    assert s3["inner_iters"] <= 2


def test_cg_error_codes():
    dims, ls = (4, 4, 2, 2), 4
    op, u = make(dims, ls, seed_u=37)
    b = F.fermion_cb(dims, ls, 38)
    bi = op.pack(to_dev(b), 1, "f64")
    x = op.zeros("f64")
    st = D().dwf_cg(op.handle, x, bi, 1e-14, 3, 0, raise_on_noconv=False)
    assert st["status"] == -4 and st["inner_iters"] >= 3
    bad = b.copy()
    bad[0, 0, 0, 0] = np.nan
    bn = op.pack(to_dev(bad), 1, "f64")
    with pytest.raises(D().DwfError) as e:
        D().dwf_cg(op.handle, x, bn, 1e-10, 100, 0)
    assert e.value.code == -5
    with pytest.raises(D().DwfError) as e:
        D().dwf_cg(op.handle, x, bi, -1.0, 100, 0)
    assert e.value.code == -1
    with pytest.raises(D().DwfError):
        D().dwf_cg(op.handle, x, x, 1e-8, 100, 0)
    # zero right-hand side: zero solution
    z = op.zeros("f64")
    D().dwf_cg(op.handle, x, z, 1e-10, 10, 0)
    assert not x.any()


@pytest.mark.parametrize("dagger", [0, 1])
@pytest.mark.parametrize("mode", [0, 2])
def test_full_solve(dagger, mode):
    dims, ls = (4, 4, 2, 4), 6
    op, u = make(dims, ls, seed_u=39)
    b = F.fermion_full(dims, ls, 40)
    bi = op.pack(to_dev(b), 2, "f64")
    x = op.field("f64", full=True)
    D().dwf_solve(op.handle, x, bi, dagger, 1e-12, 5000, mode)
    got = op.unpack(x, 2, "f64").cpu().numpy()
    r = R.ddw(u, got, M5, MF, bool(dagger)) - b
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-9
    if not dagger:
        want, _ = R.solve_full(u, b, M5, MF, tol=1e-13)
        assert rel(got, want) <= 1e-9


@pytest.fixture(scope="module")
def cg_workload():
    """The CG workload (24^4 x 12, eps 0.3, tol 1e-10): context, source, the FP64 solution and its
    iteration count."""
    w = F.WORKLOADS["cg_24^4x12"]
    dims, ls = w["dims"], w["ls"]
    op, u = make(dims, ls, w["eps"], w["seed_u"], w["M5"], w["mf"])
    b = F.fermion_cb(dims, ls, w["seed_psi"])
    bi = op.pack(to_dev(b), 1, "f64")
    x = op.zeros("f64")
    st = D().dwf_cg(op.handle, x, bi, w["tol"], 20000, 0)
    assert st["true_rel_resid"] <= w["tol"]
    x64 = op.unpack(x, 1, "f64").cpu().numpy()
    yield w, op, u, b, bi, x64, st["inner_iters"]
    op.close()
    torch.cuda.empty_cache()


def test_cg_24x24x24x24_fp64_residual_by_oracle(cg_workload):
    """The FP64 solver's solution, its residual recomputed by the C oracle."""
    w, op, u, b, bi, x64, _ = cg_workload
    r = b - C.mdagm(u, x64, w["M5"], w["mf"])
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 2e-10


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_cg_24x24x24x24_mixed_agrees_with_fp64(cg_workload, mode):
    """The CG workload, defect correction with FP32 / FP16 / BF16 inner solves: the true residual
    reaches 1e-10 (recomputed by the oracle) and the solution agrees with FP64 CG to 1e-8."""
    w, op, u, b, bi, x64, fp64_iters = cg_workload
    x = op.zeros("f64")
    st = D().dwf_cg(op.handle, x, bi, w["tol"], 20000, mode)
    assert st["true_rel_resid"] <= w["tol"]
    assert st["outer_iters"] >= 2
    got = op.unpack(x, 1, "f64").cpu().numpy()
    assert rel(got, x64) <= 1e-8
    r = b - C.mdagm(u, got, w["M5"], w["mf"])
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 2e-10
    if mode == 1:
        # the FP32 inner iteration keeps its search direction across the FP64 residual
        # refreshes: its iteration count stays within a few percent of FP64 CG's
        assert st["inner_iters"] <= 1.03 * fp64_iters


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_cg_from_a_nonzero_start(mode):
    """A random initial guess: the first residual is b - A x0 (not b), and the solve still
    reaches the oracle's solution."""
    dims, ls = (4, 4, 4, 4), 8
    op, u = make(dims, ls, seed_u=41)
    b = F.fermion_cb(dims, ls, 42)
    x0 = F.fermion_cb(dims, ls, 43)
    want, _, res = R.cg(lambda v: R.mdagm(u, v, M5, MF), b, 1e-12, 5000)
    bi = op.pack(to_dev(b), 1, "f64")
    x = op.pack(to_dev(x0), 1, "f64")
    st = D().dwf_cg(op.handle, x, bi, 1e-10, 5000, mode)
    got = op.unpack(x, 1, "f64").cpu().numpy()
    r = b - C.mdagm(u, got, M5, MF)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.5e-10
    assert rel(got, want) <= 1e-8
    assert st["true_rel_resid"] <= 1e-10
    op.close()
