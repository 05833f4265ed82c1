"""ctypes binding of libdwf.so: the C ABI's entry points under the same names.

Arguments are marshalled only: torch tensors (device memory owned by the
caller) become raw pointers, the stream is torch's current HIP stream, and a
non-zero status becomes a DwfError carrying dwf_last_error().  Every
operation runs in the library's HIP kernels; if the library is missing this
module raises at import of the first call instead of falling back to anything.
"""

from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdwf.so")

DWF_F64, DWF_F32, DWF_F16, DWF_BF16 = 0, 1, 2, 3
PRECS = {"f64": DWF_F64, "f32": DWF_F32, "f16": DWF_F16, "bf16": DWF_BF16}
STATUS = {0: "DWF_OK", -1: "DWF_EINVAL", -2: "DWF_ENOMEM", -3: "DWF_EHIP", -4: "DWF_ENOCONV", -5: "DWF_ENAN",
          -6: "DWF_EUNSUP"}


class DwfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class dwf_geom(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("Ls", ctypes.c_int), ("M5", ctypes.c_double),
                ("mf", ctypes.c_double), ("antiperiodic_t", ctypes.c_int)]


class dwf_cg_stats(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int), ("inner_iters", ctypes.c_int),
                ("true_rel_resid", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class dwf_cache_stats(ctypes.Structure):
    _fields_ = [("watermark", ctypes.c_size_t), ("resident_bytes", ctypes.c_size_t),
                ("held_bytes", ctypes.c_size_t), ("entries", ctypes.c_longlong),
                ("h2d_count", ctypes.c_longlong), ("d2h_count", ctypes.c_longlong),
                ("evictions", ctypes.c_longlong), ("h2d_bytes", ctypes.c_ulonglong),
                ("d2h_bytes", ctypes.c_ulonglong)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


DWF_CPU_READ, DWF_CPU_WRITE, DWF_ACC_READ, DWF_ACC_WRITE = 0, 1, 2, 3
DWF_ST_EMPTY, DWF_ST_CPU_DIRTY, DWF_ST_ACC_DIRTY, DWF_ST_CONSISTENT = 0, 1, 2, 3
DWF_ADVISE_NORMAL, DWF_ADVISE_INFREQUENT = 0, 1
DWF_CACHE_DEVICE, DWF_CACHE_HOST_SIM = 0, 1

_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_SIGS = {
    "dwf_create": [ctypes.POINTER(dwf_geom), ctypes.POINTER(_P)],
    "dwf_destroy": [_P],
    "dwf_field_bytes": [_P, _I, _I, ctypes.POINTER(ctypes.c_size_t)],
    "dwf_set_gauge": [_P, _P, _P],
    "dwf_set_mobius": [_P, _D, _D],
    "dwf_expi_links": [_P, _P, _P, _D, _P],
    "dwf_dd_create": [_P, _I, _I, ctypes.POINTER(_P)],
    "dwf_dd_dhop": [_P, _P, _P, _I, _I, _P],
    "dwf_dd_faces": [_P, _P, _I, _I, _P],
    "dwf_dd_destroy": [_P],
    "dwf_gauge_axpy": [_P, _P, _D, _P, _P],
    "dwf_gauge_norm2": [_P, ctypes.POINTER(_D), _P, _P],
    "dwf_get_mobius": [_P, ctypes.POINTER(_D), ctypes.POINTER(_D)],
    "dwf_pack": [_P, _P, _P, _I, _I, _P],
    "dwf_unpack": [_P, _P, _P, _I, _I, _P],
    "dwf_convert": [_P, _P, _I, _P, _I, _I, _P],
    "dwf_dhop": [_P, _P, _P, _I, _I, _I, _P],
    "dwf_m5": [_P, _P, _P, _I, _I, _I, _I, _P],
    "dwf_mpc": [_P, _P, _P, _I, _I, _P],
    "dwf_mdagm": [_P, _P, _P, _I, _P],
    "dwf_dw": [_P, _P, _P, _I, _I, _P],
    "dwf_norm2": [_P, ctypes.POINTER(_D), _P, _I, _I, _P],
    "dwf_cdot": [_P, ctypes.POINTER(_D), _P, _P, _I, _I, _P],
    "dwf_cdot_noalloc": [_P, _P, _P, _P, _I, _I, _P],
    "dwf_axpy": [_P, _P, _D, _D, _P, _I, _I, _P],
    "dwf_cg": [_P, _P, _P, _D, _I, _I, ctypes.POINTER(dwf_cg_stats), _P],
    "dwf_cg_set_inner": [_P, _D, _I],
    "dwf_solve": [_P, _P, _P, _I, _D, _I, _I, ctypes.POINTER(dwf_cg_stats), _P],
    "dwf_force": [_P, _P, _P, _P, _I, _D, _P],
    "dwf_batch_plan": [ctypes.POINTER(_P), _I, ctypes.POINTER(_I), _I, _I, ctypes.POINTER(_P)],
    "dwf_batch_capture": [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), _I, _P],
    "dwf_batch_launch": [_P, _P],
    "dwf_batch_free": [_P],
    "dwf_tune": [_P, _I, _I, ctypes.POINTER(_D), _P],
    "dwf_cache_create": [ctypes.c_size_t, _I, ctypes.POINTER(_P)],
    "dwf_cache_open": [_P, _P, ctypes.c_size_t, _I, ctypes.POINTER(_P), _P],
    "dwf_cache_close": [_P, _P],
    "dwf_cache_advise": [_P, _P, _I],
    "dwf_cache_release": [_P, _P, _P],
    "dwf_cache_flush": [_P, _P],
    "dwf_cache_query": [_P, _P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)],
    "dwf_cache_get_stats": [_P, ctypes.POINTER(dwf_cache_stats)],
    "dwf_cache_destroy": [_P, _P],
}


def lib():
    """Load libdwf.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() (hipcc, gfx950)")
        l = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(l, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        l.dwf_last_error.restype = ctypes.c_char_p
        l.dwf_last_error.argtypes = []
        _lib = l
    return _lib


def _check(rc: int):
    if rc != 0:
        raise DwfError(rc, lib().dwf_last_error().decode())


def _ptr(t) -> int:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("fields must be device tensors")
    if not t.is_contiguous():
        raise ValueError("fields must be contiguous")
    return t.data_ptr()


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _prec(p) -> int:
    return PRECS[p] if isinstance(p, str) else int(p)


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ---------------------------------------------------------------------------
def dwf_create(dims, Ls, M5=1.8, mf=0.01, antiperiodic_t=True) -> int:
    g = dwf_geom((ctypes.c_int * 4)(*[int(d) for d in dims]), int(Ls), float(M5), float(mf), int(bool(antiperiodic_t)))
    h = _P()
    _check(lib().dwf_create(ctypes.byref(g), ctypes.byref(h)))
    return h.value


def dwf_destroy(ctx: int):
    _check(lib().dwf_destroy(ctx))


def dwf_field_bytes(ctx, prec, full=0) -> int:
    n = ctypes.c_size_t()
    _check(lib().dwf_field_bytes(ctx, _prec(prec), int(full), ctypes.byref(n)))
    return n.value


def dwf_set_mobius(ctx, b, c):
    _check(lib().dwf_set_mobius(ctx, float(b), float(c)))


def dwf_get_mobius(ctx):
    b, c = _D(), _D()
    _check(lib().dwf_get_mobius(ctx, ctypes.byref(b), ctypes.byref(c)))
    return b.value, c.value


DWF_CUT = {"x": 1, "y": 2, "z": 4, "t": 8}


def dwf_dd_create(ctx, prec, cuts="t"):
    """cuts: a mask of DWF_CUT values or a string of the cut axes, e.g. "xyz" (the 2x2x2x1 split)."""
    mask = cuts if isinstance(cuts, int) else sum(DWF_CUT[a] for a in set(cuts))
    d = _P()
    _check(lib().dwf_dd_create(ctx, _prec(prec), int(mask), ctypes.byref(d)))
    return d


def dwf_dd_dhop(dd, out, inp, out_parity, dagger, stream=None):
    _check(lib().dwf_dd_dhop(dd, _ptr(out), _ptr(inp), int(out_parity), int(dagger), _stream(stream)))


def dwf_dd_faces(dd, inp, out_parity, dagger, stream=None):
    _check(lib().dwf_dd_faces(dd, _ptr(inp), int(out_parity), int(dagger), _stream(stream)))


def dwf_dd_destroy(dd):
    _check(lib().dwf_dd_destroy(dd))


def dwf_expi_links(ctx, U, P, eps, stream=None):
    _check(lib().dwf_expi_links(ctx, _ptr(U), _ptr(P), float(eps), _stream(stream)))


def dwf_gauge_axpy(ctx, Y, a, X, stream=None):
    _check(lib().dwf_gauge_axpy(ctx, _ptr(Y), float(a), _ptr(X), _stream(stream)))


def dwf_gauge_norm2(ctx, X, stream=None) -> float:
    r = _D()
    _check(lib().dwf_gauge_norm2(ctx, ctypes.byref(r), _ptr(X), _stream(stream)))
    return r.value


def dwf_set_gauge(ctx, U, stream=None):
    _check(lib().dwf_set_gauge(ctx, _ptr(U), _stream(stream)))


def dwf_pack(ctx, internal, canonical, parity, prec, stream=None):
    _check(lib().dwf_pack(ctx, _ptr(internal), _ptr(canonical), int(parity), _prec(prec), _stream(stream)))


def dwf_unpack(ctx, canonical, internal, parity, prec, stream=None):
    _check(lib().dwf_unpack(ctx, _ptr(canonical), _ptr(internal), int(parity), _prec(prec), _stream(stream)))


def dwf_convert(ctx, out, out_prec, inp, in_prec, full=0, stream=None):
    _check(lib().dwf_convert(ctx, _ptr(out), _prec(out_prec), _ptr(inp), _prec(in_prec), int(full),
                             _stream(stream)))


def dwf_dhop(ctx, out, inp, out_parity, dagger, prec, stream=None):
    _check(lib().dwf_dhop(ctx, _ptr(out), _ptr(inp), int(out_parity), int(dagger), _prec(prec), _stream(stream)))


def dwf_m5(ctx, out, inp, dagger, inverse, full, prec, stream=None):
    _check(lib().dwf_m5(ctx, _ptr(out), _ptr(inp), int(dagger), int(inverse), int(full), _prec(prec),
                        _stream(stream)))


def dwf_mpc(ctx, out, inp, dagger, prec, stream=None):
    _check(lib().dwf_mpc(ctx, _ptr(out), _ptr(inp), int(dagger), _prec(prec), _stream(stream)))


def dwf_mdagm(ctx, out, inp, prec, stream=None):
    _check(lib().dwf_mdagm(ctx, _ptr(out), _ptr(inp), _prec(prec), _stream(stream)))


def dwf_dw(ctx, out, inp, dagger, prec, stream=None):
    _check(lib().dwf_dw(ctx, _ptr(out), _ptr(inp), int(dagger), _prec(prec), _stream(stream)))


def dwf_norm2(ctx, x, full, prec, stream=None) -> float:
    r = _D()
    _check(lib().dwf_norm2(ctx, ctypes.byref(r), _ptr(x), int(full), _prec(prec), _stream(stream)))
    return r.value


def dwf_cdot(ctx, x, y, full, prec, stream=None) -> complex:
    r = (_D * 2)()
    _check(lib().dwf_cdot(ctx, r, _ptr(x), _ptr(y), int(full), _prec(prec), _stream(stream)))
    return complex(r[0], r[1])


def dwf_cdot_noalloc(ctx, result, x, y, full, prec, stream=None):
    """<x, y> (y given) or |x|^2 (y None) into result[0], result[1] (a device FP64 tensor of >= 2
    elements); enqueued on the stream, no synchronisation, no allocation."""
    if result.dtype != torch.float64 or result.numel() < 2 or not result.is_cuda:
        raise ValueError("dwf_cdot_noalloc: result must be a device float64 tensor of >= 2 elements")
    _check(lib().dwf_cdot_noalloc(ctx, _ptr(result), _ptr(x), _ptr(y), int(full), _prec(prec), _stream(stream)))


def dwf_axpy(ctx, y, a, x, full, prec, stream=None):
    a = complex(a)
    _check(lib().dwf_axpy(ctx, _ptr(y), a.real, a.imag, _ptr(x), int(full), _prec(prec), _stream(stream)))


def dwf_cg_set_inner(ctx, inner_tol=0.0, inner_maxit=0):
    _check(lib().dwf_cg_set_inner(ctx, float(inner_tol), int(inner_maxit)))


def dwf_cg(ctx, x, b, tol, maxit, mode=0, stream=None, raise_on_noconv=True) -> dict:
    st = dwf_cg_stats()
    rc = lib().dwf_cg(ctx, _ptr(x), _ptr(b), float(tol), int(maxit), int(mode), ctypes.byref(st), _stream(stream))
    if rc != 0 and (raise_on_noconv or rc != -4):
        _check(rc)
    d = st.as_dict()
    d["status"] = rc
    return d


def dwf_solve(ctx, x, b, dagger, tol, maxit, mode=0, stream=None) -> dict:
    st = dwf_cg_stats()
    _check(lib().dwf_solve(ctx, _ptr(x), _ptr(b), int(dagger), float(tol), int(maxit), int(mode),
                           ctypes.byref(st), _stream(stream)))
    return st.as_dict()


def dwf_force(ctx, F, X, Y, kind, scale=1.0, stream=None):
    _check(lib().dwf_force(ctx, _ptr(F), _ptr(X), _ptr(Y), int(kind), float(scale), _stream(stream)))


def dwf_batch_plan(ctxs, nrhs, prec, dagger=0) -> int:
    n = len(ctxs)
    arr = (_P * n)(*ctxs)
    rh = (_I * n)(*[int(r) for r in nrhs])
    h = _P()
    _check(lib().dwf_batch_plan(arr, n, rh, _prec(prec), int(dagger), ctypes.byref(h)))
    return h.value


def dwf_batch_capture(plan, outs, ins, out_parity, stream=None):
    n = len(outs)
    o = (_P * n)(*[_ptr(t) for t in outs])
    i = (_P * n)(*[_ptr(t) for t in ins])
    _check(lib().dwf_batch_capture(plan, o, i, int(out_parity), _stream(stream)))


def dwf_batch_launch(plan, stream=None):
    _check(lib().dwf_batch_launch(plan, _stream(stream)))


def dwf_batch_free(plan):
    _check(lib().dwf_batch_free(plan))


def dwf_tune(ctx, prec, dagger=0, stream=None) -> float:
    us = _D()
    _check(lib().dwf_tune(ctx, _prec(prec), int(dagger), ctypes.byref(us), _stream(stream)))
    return us.value


# ---------------------------------------------------------------------------
# Convenience: a context object that allocates caller-owned fields with torch
# ---------------------------------------------------------------------------
class Context:
    """One lattice: geometry, gauge links and helpers that allocate internal fields."""

    def __init__(self, dims, Ls, M5=1.8, mf=0.01, antiperiodic_t=True, device=None):
        if device is not None:
            torch.cuda.set_device(device)
        self.dims = tuple(int(d) for d in dims)
        self.Ls = int(Ls)
        self.M5, self.mf = float(M5), float(mf)
        self.handle = dwf_create(self.dims, self.Ls, M5, mf, antiperiodic_t)
        lx, ly, lz, lt = self.dims
        self.vol = lx * ly * lz * lt

    def close(self):
        if self.handle:
            dwf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def field(self, prec="f64", full=False) -> torch.Tensor:
        return torch.empty(dwf_field_bytes(self.handle, prec, int(full)), dtype=torch.uint8, device="cuda")

    def zeros(self, prec="f64", full=False) -> torch.Tensor:
        return torch.zeros(dwf_field_bytes(self.handle, prec, int(full)), dtype=torch.uint8, device="cuda")

    def halves(self, full_field: torch.Tensor):
        """Views of the even and odd checkerboards of a full internal field."""
        n = full_field.numel() // 2
        return full_field[:n], full_field[n:]

    def set_mobius(self, b: float, c: float):
        """Moebius coefficients (b = 1, c = 0 is Shamir, the default)."""
        dwf_set_mobius(self.handle, b, c)

    @property
    def mobius(self) -> bool:
        b, c = dwf_get_mobius(self.handle)
        return not (b == 1.0 and c == 0.0)

    def set_gauge(self, U: torch.Tensor):
        dwf_set_gauge(self.handle, U.to(torch.complex128).contiguous())

    def pack(self, canonical: torch.Tensor, parity: int, prec="f64") -> torch.Tensor:
        out = self.field(prec, parity == 2)
        dwf_pack(self.handle, out, canonical.to(torch.complex128).contiguous(), parity, prec)
        return out

    def unpack(self, internal: torch.Tensor, parity: int, prec="f64") -> torch.Tensor:
        lx, ly, lz, lt = self.dims
        if parity == 2:
            shape = (lt, lz, ly, lx, self.Ls, 4, 3)
        else:
            shape = (self.vol // 2, self.Ls, 4, 3)
        out = torch.empty(shape, dtype=torch.complex128, device="cuda")
        dwf_unpack(self.handle, out, internal, parity, prec)
        return out


# ---- software-managed device cache (host buffers: CPU tensors or addresses) ----

def _hptr(t) -> int:
    if isinstance(t, int):
        return t
    if t.is_cuda:
        raise ValueError("the cache keeps HOST buffers: pass a CPU tensor")
    if not t.is_contiguous():
        raise ValueError("host buffers must be contiguous")
    return t.data_ptr()


def _cstream(stream):
    """torch's current stream when a GPU is present; the host stand-in backend needs none."""
    if stream is None:
        return torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None
    return _stream(stream)


def dwf_cache_create(watermark_bytes, backend=DWF_CACHE_DEVICE) -> int:
    c = _P()
    _check(lib().dwf_cache_create(int(watermark_bytes), int(backend), ctypes.byref(c)))
    return c.value


def dwf_cache_open(cache, host, nbytes, intent, stream=None) -> int:
    """Address of the view: device memory for DWF_ACC_*, the host buffer for DWF_CPU_*."""
    v = _P()
    _check(lib().dwf_cache_open(cache, _hptr(host), int(nbytes), int(intent), ctypes.byref(v), _cstream(stream)))
    return v.value


def dwf_cache_close(cache, host):
    _check(lib().dwf_cache_close(cache, _hptr(host)))


def dwf_cache_advise(cache, host, advice):
    _check(lib().dwf_cache_advise(cache, _hptr(host), int(advice)))


def dwf_cache_release(cache, host, stream=None):
    _check(lib().dwf_cache_release(cache, _hptr(host), _cstream(stream)))


def dwf_cache_flush(cache, stream=None):
    _check(lib().dwf_cache_flush(cache, _cstream(stream)))


def dwf_cache_query(cache, host):
    """(state DWF_ST_*, open views, resident on the device)."""
    st, refs, res = _I(), _I(), _I()
    _check(lib().dwf_cache_query(cache, _hptr(host), ctypes.byref(st), ctypes.byref(refs), ctypes.byref(res)))
    return st.value, refs.value, bool(res.value)


def dwf_cache_get_stats(cache) -> dict:
    st = dwf_cache_stats()
    _check(lib().dwf_cache_get_stats(cache, ctypes.byref(st)))
    return st.as_dict()


def dwf_cache_destroy(cache, stream=None):
    _check(lib().dwf_cache_destroy(cache, _cstream(stream)))
