"""Helpers shared by the GPU tests: seeded inputs, a context per lattice, rel-L2."""

import numpy as np
import pytest
import torch

from synth import fields as F

# rel-L2 per operator application against the FP64 oracle.  16-bit storage (FP16 and BF16) is
# held to 5e-3; measured on every configuration the tests use: FP16 <= 4.4e-4, BF16 <= 3.4e-3
# (the Moebius M_pc^dag M_pc, with four rounded intermediates, is the largest).
TOL = {"f64": 1e-13, "f32": 1e-6, "f16": 5e-3, "bf16": 5e-3}


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def make(dims, ls, eps=0.5, seed_u=101, M5=1.8, mf=0.01, antiperiodic=True):
    """(Context with gauge set, numpy U)."""
    from paper_2203_06777_amd import dwf as D

    u = F.gauge_field(dims, eps, seed_u)
    op = D.Context(dims, ls, M5, mf, antiperiodic)
    op.set_gauge(torch.from_numpy(u).cuda())
    return op, u


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()
