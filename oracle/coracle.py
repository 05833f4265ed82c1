"""ctypes loader for the plain C/OpenMP oracle (liboracle_dwf.so) — test infrastructure only.

The library is compiled from dwf_oracle.c next to this file by the package
build step; every function takes numpy complex128 arrays in the canonical
layouts and returns new arrays.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle_dwf.so")
SRC_PATH = os.path.join(_HERE, "dwf_oracle.c")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, OpenMP)."""
    import subprocess

    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall",
                               SRC_PATH, "-o", LIB_PATH + ".tmp"])
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        l = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i, lng, d = ctypes.c_int, ctypes.c_long, ctypes.c_double
        l.oracle_dhop_cb.argtypes = [P, P, P, P, i, i, i, i, lng, lng]
        l.oracle_m5op.argtypes = [P, P, lng, i, d, d, i]
        l.oracle_m5inv.argtypes = [P, P, lng, i, d, d, i]
        l.oracle_mpc.argtypes = [P, P, P, P, i, d, d, i, i]
        l.oracle_mdagm.argtypes = [P, P, P, P, i, d, d, i]
        l.oracle_num_threads.restype = ctypes.c_int
        l.oracle_set_num_threads.argtypes = [i]
        _lib = l
    return _lib


def _c(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _dims(U):
    lt, lz, ly, lx = U.shape[:4]
    d = np.array([lx, ly, lz, lt], dtype=np.int32)
    return d, d.ctypes.data_as(ctypes.c_void_p)


def dhop_cb(U, psi_cb, out_parity, dagger=False, antiperiodic_t=True, rows=None):
    """D_h^{p<-1-p}; with rows=(begin, end) only that row range is computed (others left zero)."""
    U, pu = _c(U)
    psi, pp = _c(psi_cb)
    d, pd = _dims(U)
    out = np.zeros_like(psi)
    b, e = (0, psi.shape[0]) if rows is None else rows
    lib().oracle_dhop_cb(pu, pp, out.ctypes.data_as(ctypes.c_void_p), pd, psi.shape[1], int(out_parity),
                         int(bool(dagger)), int(bool(antiperiodic_t)), int(b), int(e))
    return out


def m5op(psi, M5, mf, dagger=False):
    psi, pp = _c(psi)
    ls = psi.shape[-3]
    out = np.empty_like(psi)
    lib().oracle_m5op(pp, out.ctypes.data_as(ctypes.c_void_p), psi.size // (ls * 12), ls, M5, mf, int(dagger))
    return out


def m5inv(psi, M5, mf, dagger=False):
    psi, pp = _c(psi)
    ls = psi.shape[-3]
    out = np.empty_like(psi)
    lib().oracle_m5inv(pp, out.ctypes.data_as(ctypes.c_void_p), psi.size // (ls * 12), ls, M5, mf, int(dagger))
    return out


def mpc(U, psi_o, M5, mf, dagger=False, antiperiodic_t=True):
    U, pu = _c(U)
    psi, pp = _c(psi_o)
    d, pd = _dims(U)
    out = np.empty_like(psi)
    lib().oracle_mpc(pu, pp, out.ctypes.data_as(ctypes.c_void_p), pd, psi.shape[1], M5, mf, int(dagger),
                     int(bool(antiperiodic_t)))
    return out


def mdagm(U, psi_o, M5, mf, antiperiodic_t=True):
    U, pu = _c(U)
    psi, pp = _c(psi_o)
    d, pd = _dims(U)
    out = np.empty_like(psi)
    lib().oracle_mdagm(pu, pp, out.ctypes.data_as(ctypes.c_void_p), pd, psi.shape[1], M5, mf,
                       int(bool(antiperiodic_t)))
    return out


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_num_threads(n: int) -> None:
    lib().oracle_set_num_threads(int(n))
