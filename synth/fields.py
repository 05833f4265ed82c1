"""Seeded generators for gauge links and fermion fields in the canonical layouts.

Canonical layouts (complex128, numpy, interleaved re/im in memory):

* gauge ``U``: ``(Lt, Lz, Ly, Lx, 4, 3, 3)``, ``U[t,z,y,x,mu,a,b]`` is the colour
  matrix on the link from x to x + mu_hat, mu = 0..3 = x, y, z, t.
* full fermion: ``(Lt, Lz, Ly, Lx, Ls, 4, 3)`` (spin, colour innermost).
* checkerboard fermion: ``(V/2, Ls, 4, 3)``, row c(x) = lex(x) >> 1 with
  lex(x) = x0 + Lx*(x1 + Ly*(x2 + Lz*x3)).

Every random stream is numpy's PCG64 seeded by an integer, so a workload is
reproduced exactly from its seed on any host.
"""

from __future__ import annotations

import numpy as np

# Gell-Mann matrices lambda_1..lambda_8 (the standard su(3) basis).
_GM = np.zeros((8, 3, 3), dtype=np.complex128)
_GM[0][0, 1] = _GM[0][1, 0] = 1
_GM[1][0, 1], _GM[1][1, 0] = -1j, 1j
_GM[2][0, 0], _GM[2][1, 1] = 1, -1
_GM[3][0, 2] = _GM[3][2, 0] = 1
_GM[4][0, 2], _GM[4][2, 0] = -1j, 1j
_GM[5][1, 2] = _GM[5][2, 1] = 1
_GM[6][1, 2], _GM[6][2, 1] = -1j, 1j
_GM[7][0, 0] = _GM[7][1, 1] = 1 / np.sqrt(3)
_GM[7][2, 2] = -2 / np.sqrt(3)


def lattice_volume(dims) -> int:
    return int(np.prod(dims))


def _check_dims(dims):
    dims = tuple(int(d) for d in dims)
    if len(dims) != 4 or any(d < 2 or d % 2 for d in dims):
        raise ValueError(f"lattice extents must be four even numbers >= 2, got {dims}")
    return dims


def _reunitarise(u: np.ndarray) -> np.ndarray:
    """Project batched 3x3 matrices onto SU(3) by row Gram-Schmidt.

    Row 0 is normalised, row 1 is orthogonalised against row 0 and normalised,
    and row 2 is conj(row0 x row1), which makes the determinant exactly 1 up to
    rounding.
    """
    r0 = u[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = u[..., 1, :]
    r1 = r1 - np.sum(r0.conj() * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.cross(r0, r1).conj()
    return np.stack([r0, r1, r2], axis=-2)


def _su3_from_omega(omega: np.ndarray, eps: float) -> np.ndarray:
    """exp(i eps H) with H = sum_a omega_a lambda_a / 2, via eigh, reunitarised."""
    h = np.einsum("...a,aij->...ij", omega, _GM) * 0.5
    w, v = np.linalg.eigh(h)
    u = np.einsum("...ik,...k,...jk->...ij", v, np.exp(1j * eps * w), v.conj())
    return _reunitarise(u)


def gauge_field(dims, eps: float, seed: int, chunk_links: int = 1 << 19) -> np.ndarray:
    """Random SU(3) links U = exp(i eps H), H Gaussian traceless Hermitian.

    omega in R^8 is drawn N(0,1) per link in canonical order (t, z, y, x, mu),
    all at once, so chunked processing never changes the stream.
    """
    dims = _check_dims(dims)
    lx, ly, lz, lt = dims
    nlinks = lattice_volume(dims) * 4
    rng = np.random.Generator(np.random.PCG64(seed))
    omega = rng.standard_normal((nlinks, 8))
    out = np.empty((nlinks, 3, 3), dtype=np.complex128)
    for a in range(0, nlinks, chunk_links):
        b = min(nlinks, a + chunk_links)
        out[a:b] = _su3_from_omega(omega[a:b], eps)
    return out.reshape(lt, lz, ly, lx, 4, 3, 3)


def unit_gauge(dims) -> np.ndarray:
    """Free field: every link is the 3x3 identity."""
    lx, ly, lz, lt = _check_dims(dims)
    u = np.zeros((lt, lz, ly, lx, 4, 3, 3), dtype=np.complex128)
    for a in range(3):
        u[..., a, a] = 1.0
    return u


def _gaussian_complex(rng, shape) -> np.ndarray:
    z = rng.standard_normal(tuple(shape) + (2,))
    return z.view(np.complex128).reshape(shape)


def fermion_full(dims, ls: int, seed: int) -> np.ndarray:
    """Full 5D fermion field, re and im iid N(0,1), canonical order."""
    lx, ly, lz, lt = _check_dims(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    return _gaussian_complex(rng, (lt, lz, ly, lx, ls, 4, 3))


def fermion_cb(dims, ls: int, seed: int) -> np.ndarray:
    """One-checkerboard 5D fermion field (V/2, Ls, 4, 3), re and im iid N(0,1)."""
    dims = _check_dims(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    return _gaussian_complex(rng, (lattice_volume(dims) // 2, ls, 4, 3))


def random_su3_field(dims, seed: int, eps: float = 3.0) -> np.ndarray:
    """One SU(3) matrix per site, shape (Lt, Lz, Ly, Lx, 3, 3) (gauge transforms)."""
    lx, ly, lz, lt = _check_dims(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    omega = rng.standard_normal((lattice_volume(dims), 8))
    return _su3_from_omega(omega, eps).reshape(lt, lz, ly, lx, 3, 3)


def su3_directions(dims, seed: int) -> np.ndarray:
    """Gaussian su(3) direction Q_mu(x) = sum_a omega_a lambda_a / 2 per link.

    Shape (Lt, Lz, Ly, Lx, 4, 3, 3), Hermitian and traceless.
    """
    lx, ly, lz, lt = _check_dims(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    omega = rng.standard_normal((lt, lz, ly, lx, 4, 8))
    return np.einsum("...a,aij->...ij", omega, _GM) * 0.5


# Named workloads: shapes, parameters and seeds of the measured and tested cases.
WORKLOADS = {
    # Dhop + M5 parity case (FP64).
    "dwf_4^4x8": dict(dims=(4, 4, 4, 4), ls=8, M5=1.8, mf=0.01, eps=0.5, seed_u=101, seed_psi=201),
    # Checkerboarded Dhop, FP64 and FP32; the headline is 32^4 x 16.
    "dhop_16^4x16": dict(dims=(16, 16, 16, 16), ls=16, M5=1.8, mf=0.01, eps=0.5, seed_u=102, seed_psi=202),
    "dhop_32^4x16": dict(dims=(32, 32, 32, 32), ls=16, M5=1.8, mf=0.01, eps=0.5, seed_u=102, seed_psi=202),
    # Mixed-precision defect-correction CG on the Schur normal operator.
    "cg_24^4x12": dict(dims=(24, 24, 24, 24), ls=12, M5=1.8, mf=0.01, eps=0.3, seed_u=103, seed_psi=303,
                       tol=1e-10),
    # Batched multi-RHS: 32^4 x 12 with 12 right-hand sides (seed 2040 + r) ...
    "batch_32^4x12x12": dict(dims=(32, 32, 32, 32), ls=12, M5=1.8, mf=0.01, eps=0.5, seed_u=104,
                             rhs_seeds=[2040 + r for r in range(12)]),
    # ... and a mixed batch of four lattices (Ls = 8, 4 RHS each; U seed 100+L, RHS 1000*L+r).
    "batch_mixed": dict(lattices=[dict(dims=(L, L, L, L), ls=8, seed_u=100 + L,
                                       rhs_seeds=[1000 * L + r for r in range(4)]) for L in (8, 12, 16, 20)],
                        M5=1.8, mf=0.01, eps=0.5),
    # Differentiable action S = phi^dag (D^dag D)^-1 phi.
    "force_16^4x8": dict(dims=(16, 16, 16, 16), ls=8, M5=1.8, mf=0.01, eps=0.5, seed_u=105, seed_phi=505,
                         seed_dirs=list(range(600, 616)), h=1e-5),
}
