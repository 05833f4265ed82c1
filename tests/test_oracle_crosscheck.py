"""The plain C oracle agrees with the pinned numpy oracle (FP64, round-off only)."""

import numpy as np
import pytest

from oracle import coracle as C
from oracle import dwf_ref as R
from synth import fields as F

M5, MF = 1.8, 0.01


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("dims,ls", [((4, 4, 4, 4), 8), ((2, 2, 2, 2), 4), ((6, 4, 2, 8), 3), ((4, 2, 6, 2), 1)])
@pytest.mark.parametrize("par,dag", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_c_dhop_matches_numpy(dims, ls, par, dag):
    u = F.gauge_field(dims, 0.5, 101)
    psi = F.fermion_cb(dims, ls, 201)
    assert rel(C.dhop_cb(u, psi, par, dag), R.dhop_cb(u, psi, par, dag)) < 1e-14
    assert rel(C.dhop_cb(u, psi, par, dag, antiperiodic_t=False), R.dhop_cb(u, psi, par, dag, False)) < 1e-14


def test_c_dhop_row_range():
    dims, ls = (4, 4, 4, 4), 4
    u = F.gauge_field(dims, 0.5, 1)
    psi = F.fermion_cb(dims, ls, 2)
    full = C.dhop_cb(u, psi, 1)
    part = C.dhop_cb(u, psi, 1, rows=(10, 37))
    assert np.array_equal(part[10:37], full[10:37])
    assert not part[:10].any() and not part[37:].any()


@pytest.mark.parametrize("ls", [1, 4, 8, 12])
@pytest.mark.parametrize("dag", [0, 1])
def test_c_m5_family_matches_numpy(ls, dag):
    psi = F.fermion_cb((4, 4, 2, 2), ls, 5)
    assert rel(C.m5op(psi, M5, MF, dag), R.m5op(psi, M5, MF, dag)) < 1e-14
    assert rel(C.m5inv(psi, M5, MF, dag), R.m5inv(psi, M5, MF, dag)) < 1e-13


def test_c_schur_matches_numpy():
    dims, ls = (4, 4, 2, 4), 6
    u = F.gauge_field(dims, 0.5, 7)
    psi = F.fermion_cb(dims, ls, 8)
    for dag in (0, 1):
        assert rel(C.mpc(u, psi, M5, MF, dag), R.mpc(u, psi, M5, MF, dag)) < 1e-13
    assert rel(C.mdagm(u, psi, M5, MF), R.mdagm(u, psi, M5, MF)) < 1e-13
