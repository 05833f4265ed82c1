"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point that include/dwf.h declares, and rejects invalid arguments
before touching a device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dwf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dwf_[a-z0-9_]+)\s*\(", text)))


def lib():
    from paper_2203_06777_amd import dwf

    try:
        return dwf.lib()
    except RuntimeError as e:
        pytest.skip(f"libdwf.so not built: {e}")


def test_header_declares_the_hot_path_entry_points():
    names = declared_functions()
    for must in ("dwf_dhop", "dwf_m5", "dwf_mdagm", "dwf_cg", "dwf_force", "dwf_create", "dwf_destroy",
                 "dwf_set_gauge", "dwf_pack", "dwf_unpack", "dwf_batch_plan", "dwf_batch_capture",
                 "dwf_batch_launch", "dwf_tune", "dwf_solve", "dwf_norm2", "dwf_cdot", "dwf_axpy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    l = lib()
    missing = [n for n in declared_functions() if not hasattr(l, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2203_06777_amd import dwf

    names = [n for n in declared_functions() if n != "dwf_last_error"]
    assert all(hasattr(dwf, n) for n in names), [n for n in names if not hasattr(dwf, n)]


@pytest.mark.parametrize("dims,ls", [((4, 4, 3, 4), 8), ((4, 4, 4, 0), 8), ((4, 4, 4, 4), 0), ((4, 4, 4, 4), 65),
                                     ((1, 4, 4, 4), 4)])
def test_create_rejects_bad_geometry_without_a_device(dims, ls):
    from paper_2203_06777_amd import dwf

    lib()
    with pytest.raises(dwf.DwfError) as e:
        dwf.dwf_create(dims, ls)
    assert e.value.code == -1
    assert "dwf_create" in str(e.value)


@pytest.mark.parametrize("dims,ls,M5,mf,what", [
    ((256, 256, 256, 2), 8, 1.8, 0.01, "too large"),        # V/2 = 2^24 sites
    ((4, 4, 4, 4), 8, 5.0, 0.01, "singular"),                # 5 - M5 = 0
    ((4, 4, 4, 4), 2, 3.0, -4.0, "singular"),                # 1 + mf (5 - M5)^-Ls = 0
    ((4, 4, 4, 4), 8, 1.8, float("nan"), "finite"),
    ((4, 4, 4, 4), 8, float("inf"), 0.01, "finite"),
])
def test_create_rejects_degenerate_parameters_without_a_device(dims, ls, M5, mf, what):
    from paper_2203_06777_amd import dwf

    lib()
    with pytest.raises(dwf.DwfError) as e:
        dwf.dwf_create(dims, ls, M5, mf)
    assert e.value.code == -1
    assert what in str(e.value)


def test_null_context_is_an_error():
    from paper_2203_06777_amd import dwf

    l = lib()
    rc = l.dwf_dhop(None, None, None, 0, 0, 1, None)
    assert rc == -1
    assert b"null context" in l.dwf_last_error()
    n = ctypes.c_size_t()
    assert l.dwf_field_bytes(None, 1, 0, ctypes.byref(n)) == -1
    assert l.dwf_batch_launch(None, None) == -1
    assert l.dwf_batch_free(None) == 0
    assert l.dwf_destroy(None) == 0
    l.dwf_cdot_noalloc.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    assert l.dwf_cdot_noalloc(None, None, None, None, 0, 1, None) == -1
    assert b"null context" in l.dwf_last_error()


def test_null_handles_of_the_extensions_are_errors():
    """Moebius, HMC and domain-decomposition entry points reject null handles without a device."""
    l = lib()
    l.dwf_set_mobius.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double]
    assert l.dwf_set_mobius(None, 1.5, 0.5) == -1
    assert b"null context" in l.dwf_last_error()
    b, c = ctypes.c_double(), ctypes.c_double()
    assert l.dwf_get_mobius(None, ctypes.byref(b), ctypes.byref(c)) == -1
    l.dwf_expi_links.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]
    assert l.dwf_expi_links(None, None, None, 0.1, None) == -1
    l.dwf_gauge_axpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
    assert l.dwf_gauge_axpy(None, None, 1.0, None, None) == -1
    r = ctypes.c_double()
    assert l.dwf_gauge_norm2(None, ctypes.byref(r), None, None) == -1
    d = ctypes.c_void_p()
    assert l.dwf_dd_create(None, 1, 8, ctypes.byref(d)) == -1
    assert l.dwf_dd_dhop(None, None, None, 0, 0, None) == -1
    assert b"null plan" in l.dwf_last_error()
    assert l.dwf_dd_faces(None, None, 0, 0, None) == -1
    assert l.dwf_dd_destroy(None) == 0
