"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/sylt.h declares, and rejects invalid arguments with
the documented status before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sylt.h")


@pytest.fixture(scope="module")
def L():
    from paper_2412_15840_amd import sylt
    return sylt.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sylt_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_five_calls():
    names = declared_functions()
    for f in ("sylt_schur_factor", "sylt_transform", "sylt_sweep", "sylt_solve",
              "sylt_solve_backward"):
        assert f in names


def test_every_declared_symbol_is_exported(L):
    missing = [f for f in declared_functions() if not hasattr(L, f)]
    assert not missing, missing


def test_status_strings(L):
    for code in range(0, -8, -1):
        s = L.sylt_status_string(code)
        assert s and s != b"unknown status"
    assert L.sylt_status_string(5) == b"unknown status"
    assert L.sylt_version() == 200


def _dims(n):
    return (ctypes.c_int64 * max(1, len(n)))(*n)


@pytest.mark.parametrize("N,n,code", [
    (0, [], -1),               # no modes
    (33, [2] * 33, -6),        # more modes than supported
    (2, [3, 0], -1),           # empty extent
    (2, [257, 2], -6),         # extent above 256
    (2, [-1, 2], -1),
    (31, [64] * 31, -6),       # prod n_k overflows 2^62
])
def test_schur_factor_rejects_bad_shapes(L, N, n, code):
    h = ctypes.c_void_p(1234)
    dummy = (ctypes.c_void_p * max(1, N))(*([8] * max(1, N)))
    r = L.sylt_schur_factor(N, _dims(n), ctypes.cast(dummy, ctypes.c_void_p), None, ctypes.byref(h))
    assert r == code
    assert not h.value


def test_null_pointers_rejected(L):
    h = ctypes.c_void_p()
    assert L.sylt_schur_factor(2, _dims([2, 2]), None, None, ctypes.byref(h)) == -1
    arr = (ctypes.c_void_p * 2)(8, None)
    assert L.sylt_schur_factor(2, _dims([2, 2]), ctypes.cast(arr, ctypes.c_void_p), None,
                               ctypes.byref(h)) == -1
    assert L.sylt_schur_factor(2, _dims([2, 2]), ctypes.cast(arr, ctypes.c_void_p), None, None) == -1
    assert L.sylt_plan_from_factors(2, _dims([2, 2]), None, None, None, None, ctypes.byref(h)) == -1
    assert L.sylt_transform(None, 0, 0, None, None) == -1
    assert L.sylt_sweep(None, 0, 0, None, None) == -1
    assert L.sylt_solve(None, None, None, None, None, 0, None, None) == -1
    assert L.sylt_solve_backward(None, None, None, None, None, None, 0, None) == -1
    assert L.sylt_residual(None, None, None, None, None, None) == -1
    assert L.sylt_plan_destroy(None) == -1
    assert L.sylt_workspace_bytes(None, 0) == -1
    assert L.sylt_plan_separation(None, None) == -1
    assert L.sylt_plan_get_factors(None, 0, None, None, None) == -1
    assert L.sylt_evolve(None, ctypes.c_double(0.1), None, None, None, None, 0, None) == -1
    L.sylt_evolve_workspace_bytes.restype = ctypes.c_int64
    assert L.sylt_evolve_workspace_bytes(None) == -1
    assert L.sylt_schur_factor_ex(2, _dims([2, 2]), None, 1, None, ctypes.byref(h)) == -1
    blocks = (ctypes.c_int * 2)(2, 2)
    assert L.sylt_plan_set_sweep_blocks(None, 2, blocks) == -1


def test_info_struct_layout_matches_header():
    """sylt_info as declared in the header and as marshalled by the binding."""
    from paper_2412_15840_amd import sylt
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\} sylt_info;", text).group(1)
    names = re.findall(r"([a-z_]+)\s*[,;]", body)
    assert [f[0] for f in sylt._Info._fields_] == names
    assert ctypes.sizeof(sylt._Info) == 40


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2412_15840_amd import sylt
    monkeypatch.setattr(sylt, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(sylt, "_LIB", None)
    with pytest.raises(RuntimeError, match="not found"):
        sylt.lib()
