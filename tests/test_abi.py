"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments before touching a device (CPU-only checks, no compute calls)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nncp.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(nncp[a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


def _lib():
    from paper_1806_07985_amd import native
    if not os.path.exists(native.LIB_PATH):
        pytest.skip("library not built")
    return native.lib()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ["nncp", "nncp_workspace_bytes", "nncp_strerror", "nncp_plan_create", "nncp_plan_run",
                     "nncp_partial_mttkrp", "nncp_mttv", "nncp_mttkrp", "nncp_gram", "nncp_nls_update",
                     "nncp_quantize", "nncp_norm_sq"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_strerror_and_version():
    L = _lib()
    assert L.nncp_strerror(0) == b"ok"
    assert L.nncp_strerror(-1) == b"invalid argument"
    assert L.nncp_version() >= 100


def test_workspace_bytes_validation():
    from paper_1806_07985_amd import native
    _lib()
    assert native.workspace_bytes([60, 50, 40], 5) > 0
    assert native.workspace_bytes([128, 128, 128, 128], 32, split=2) > 4 * 16384 * 32
    L = native.lib()
    o = native.Options()
    bad = [
        ([5], 3, 0),            # N < 2
        ([5, 0, 3], 3, 0),      # zero extent
        ([5, 4, 3], 0, 0),      # R < 1
        ([5, 4, 3], 1000, 0),   # R too large
        ([5, 4, 3], 3, 7),      # unknown dtype
    ]
    for dims, R, dt in bad:
        assert L.nncp_workspace_bytes(len(dims), native._dims(dims), R, dt, ctypes.byref(o)) == 0
    o.split = 3
    assert L.nncp_workspace_bytes(3, native._dims([5, 4, 3]), 3, 0, ctypes.byref(o)) == 0


def test_entry_points_reject_bad_arguments_without_a_device():
    from paper_1806_07985_amd import native
    L = _lib()
    dims = native._dims([4, 4, 4])
    o = native.Options()
    lam = (ctypes.c_double * 2)(1.0, 1.0)
    # NULL tensor / factor pointers and a bad update code are rejected up front
    assert L.nncp(None, 0, 3, dims, 2, 1, 0, None, lam, None, None, None, 0, ctypes.byref(o), None) == -1
    H = (native.c_vp * 3)(None, None, None)
    assert L.nncp(ctypes.c_void_p(16), 0, 3, dims, 2, 1, 0, H, lam, None, None, None, 0, ctypes.byref(o),
                  None) == -1
    assert L.nncp_quantize(None, None, 1, 10, None) == -1
    assert L.nncp_quantize(ctypes.c_void_p(16), ctypes.c_void_p(16), 0, 10, None) == -1
    assert L.nncp_mttv(None, 2, dims, 0, None, 2, None, None) == -1
    assert L.nncp_partial_mttkrp(None, 0, 3, dims, 1, 0, None, 2, None, None) == -1
    assert L.nncp_nls_update(None, None, 4, 2, None, None, 0, None, None) == -1
    assert L.nncp_gram(None, 4, 2, None, None) == -1


def test_inner_sweeps_option_layout_and_limit():
    """The options struct keeps its size (inner_sweeps and inner_tol took reserved
    slots) and a sweep count above the maximum or a bad tolerance is rejected
    before any device work."""
    from paper_1806_07985_amd import native
    L = _lib()
    assert ctypes.sizeof(native.Options) == 56
    assert native.Options.inner_sweeps.offset == 32
    dims = native._dims([4, 4, 4])
    lam = (ctypes.c_double * 2)(1.0, 1.0)
    H = (native.c_vp * 3)(ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16))
    o = native.Options(inner_sweeps=100001)
    assert L.nncp(ctypes.c_void_p(16), 0, 3, dims, 2, 1, 0, H, lam, None, None, None, 0, ctypes.byref(o),
                  None) == -1
    # inner_tol must be finite and >= 0
    assert native.Options.inner_tol.offset == 40
    for bad in (-1e-9, float("nan"), float("inf")):
        o = native.Options(inner_sweeps=10, inner_tol=bad)
        assert L.nncp(ctypes.c_void_p(16), 0, 3, dims, 2, 1, 0, H, lam, None, None, None, 0, ctypes.byref(o),
                      None) == -1
    # the block solve entry point checks its sweep count and tolerance
    p16 = ctypes.c_void_p(16)
    assert L.nncp_nls_solve(p16, p16, 4, 2, p16, p16, 0, 0, 0.0, None, p16, None) == -1
    assert L.nncp_nls_solve(p16, p16, 4, 2, p16, p16, 0, 100001, 0.0, None, p16, None) == -1
    assert L.nncp_nls_solve(p16, p16, 4, 2, p16, p16, 0, 10, -1.0, None, p16, None) == -1


def test_autotune_split_rejects_bad_arguments_without_a_device():
    from paper_1806_07985_amd import native
    L = _lib()
    dims = native._dims([4, 4, 4])
    best = ctypes.c_int(0)
    H = (native.c_vp * 3)(ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16))
    assert L.nncp_autotune_split(None, 0, 3, dims, 2, H, None, 3, ctypes.byref(best), None, None) == -1
    assert L.nncp_autotune_split(ctypes.c_void_p(16), 0, 3, dims, 2, H, None, 0, ctypes.byref(best), None,
                                 None) == -1
    assert L.nncp_autotune_split(ctypes.c_void_p(16), 0, 1, dims, 2, H, None, 3, ctypes.byref(best), None,
                                 None) == -1
    assert L.nncp_autotune_split(ctypes.c_void_p(16), 0, 3, dims, 2, H, None, 3, None, None, None) == -1


def test_last_device_error_is_callable():
    from paper_1806_07985_amd import native
    code, where = native.last_device_error()
    assert isinstance(code, int) and isinstance(where, int)
    assert (code == 0) == (where == 0)
