"""The C-ABI library loads and exports every symbol include/pvjp.h declares;
host-side validation rejects bad arguments before any launch.  No GPU needed:
nothing here launches a kernel."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pvjp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pvjp_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def capi():
    from paper_2202_10297_amd import build, capi as c

    if not os.path.exists(c.LIB_PATH):
        build.build()
    return c


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ["pvjp_linrec_scan", "pvjp_linrec_scan_vjp", "pvjp_reduce", "pvjp_reduce_vjp", "pvjp_hist",
                 "pvjp_hist_vjp", "pvjp_scatter", "pvjp_scatter_vjp", "pvjp_map", "pvjp_map_vjp"]:
        assert must in names


def test_every_declared_symbol_is_exported(capi):
    lib = ctypes.CDLL(capi.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", capi.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\b(pvjp_[a-z0-9_]+)\b", out))
    assert set(declared_functions()) <= exported


def test_binding_covers_header(capi):
    assert set(capi.SIGNATURES) == set(declared_functions())


def test_validation_before_launch(capi):
    L = capi.lib()
    assert L.pvjp_linrec_scan(7, None, None, 10, None, None, None, None, 0, None) == capi.PVJP_EINVAL
    assert "dtype" in capi.last_error()
    assert L.pvjp_linrec_scan(capi.F64, 8, 8, -1, None, None, None, None, 0, None) == capi.PVJP_EINVAL
    # workspace too small
    assert L.pvjp_linrec_scan(capi.F64, 8, 8, 100, 8, 8, None, 256, 1, None) == capi.PVJP_ENOMEM
    assert L.pvjp_hist(0, 0, None, None, 10, 0, None, None, None, None, None, None, 0, None) == capi.PVJP_EINVAL
    assert L.pvjp_hist(capi.MAX, 0, 8, 8, 10, 4, 8, None, None, None, None, 256, 1 << 20, None) == capi.PVJP_EINVAL
    assert "winner" in capi.last_error()
    assert L.pvjp_reduce(9, 0, None, 1, None, None, None, None, None, 0, None) == capi.PVJP_EINVAL
    assert L.pvjp_map(42, 0, 8, 1, 8, None) == capi.PVJP_EINVAL
    # empty inputs are valid and launch nothing
    assert L.pvjp_linrec_scan(capi.F32, None, None, 0, None, None, None, None, 0, None) == capi.PVJP_OK
    assert L.pvjp_scatter(capi.F32, None, 0, None, None, 0, None, None) == capi.PVJP_OK


def test_workspace_queries(capi):
    L = capi.lib()
    assert L.pvjp_linrec_ckpt_len(0) == 0
    assert L.pvjp_linrec_ckpt_len(1) == 1 and L.pvjp_linrec_ckpt_len(1025) == 2
    assert L.pvjp_linrec_scan_ws_bytes(capi.F64, 65536) >= 256 + 32 * 64
    # bins that fit LDS: per-block partials, independent of n beyond the grid
    small = L.pvjp_hist_ws_bytes(capi.ADD, capi.F32, 1 << 26, 1 << 10)
    assert 8 << 10 <= small <= 64 << 20
    # FP32 + beyond LDS: a value and a bin slot (4 + 4 bytes) per element,
    # plus per-tile offsets and per-item partials
    n = 1 << 26
    big = L.pvjp_hist_ws_bytes(capi.ADD, capi.F32, n, 1 << 20)
    assert 8 * n <= big <= 10 * n
    # FP64 has no partitioned path: the direct-mapped cache needs no partials
    assert L.pvjp_hist_ws_bytes(capi.ADD, capi.F64, n, 1 << 20) < 64 << 20
    assert L.pvjp_reduce_ws_bytes(capi.ADD, capi.F32, 0) > 0


def test_generic_reduce_validation(capi):
    L = capi.lib()
    assert [L.pvjp_gop_components(k) for k in range(4)] == [1, 2, 4, 0]
    # three 32-byte slots per tile and per group of 64 tiles, each array
    # rounded to 256 bytes
    assert L.pvjp_reduce_generic_ws_bytes(capi.GOP_LOGADDEXP, capi.F32, 2048 * 100) == 3 * 3328 + 3 * 256
    assert L.pvjp_reduce_generic_ws_bytes(capi.GOP_MAT2, capi.F64, 1024 * 8 + 1) == 3 * 512 + 3 * 256
    # 2^26 FP32: 32768 tiles in 512 groups
    assert L.pvjp_reduce_generic_ws_bytes(capi.GOP_LINREC, capi.F32, 1 << 26) == 3 * 32768 * 32 + 3 * 512 * 32
    assert L.pvjp_reduce_generic_ws_bytes(7, capi.F32, 10) == 0
    one = capi.ptr_array([256])
    assert L.pvjp_reduce_generic_ckpt_bytes(capi.GOP_LINREC, capi.F32, (1 << 26) + 1) == 32769 * 32
    assert L.pvjp_reduce_generic(7, capi.F32, one, 10, one, None, 256, 1 << 20, None) == capi.PVJP_EINVAL
    assert "operator" in capi.last_error()
    assert L.pvjp_reduce_generic(capi.GOP_LOGADDEXP, 5, one, 10, one, None, 256, 1 << 20, None) == capi.PVJP_EINVAL
    assert L.pvjp_reduce_generic(capi.GOP_LOGADDEXP, capi.F32, one, 10, one, None, 256, 16, None) == capi.PVJP_ENOMEM
    assert L.pvjp_reduce_generic(capi.GOP_LOGADDEXP, capi.F32, one, 10, one, None, 100, 1 << 20,
                                 None) == capi.PVJP_EINVAL
    assert "aligned" in capi.last_error()
    assert L.pvjp_reduce_generic(capi.GOP_LOGADDEXP, capi.F32, one, 10, one, 8, 256, 1 << 20, None) == capi.PVJP_EINVAL
    assert "ckpt" in capi.last_error()
    two = capi.ptr_array([256, None])
    assert L.pvjp_reduce_generic(capi.GOP_LINREC, capi.F64, two, 10, two, None, 256, 1 << 20,
                                 None) == capi.PVJP_EINVAL
    assert "component 1" in capi.last_error()
    assert L.pvjp_reduce_generic_vjp(capi.GOP_LOGADDEXP, capi.F32, one, 10, None, None, one, 0, 256, 1 << 20,
                                     None) == capi.PVJP_EINVAL
    misaligned = capi.ptr_array([258])
    assert L.pvjp_reduce_generic_vjp(capi.GOP_LOGADDEXP, capi.F32, one, 10, None, one, misaligned, 0, 256, 1 << 20,
                                     None) == capi.PVJP_EINVAL
    assert "misaligned" in capi.last_error()
