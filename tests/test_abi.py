"""The C-ABI library loads and exports every entry point include/mcd.h declares
(no GPU work: only calls that return before touching the device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcd.h")
LIB = os.path.join(ROOT, "paper_2509_22975_amd", "libmcd.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mcd_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("mcd_basis_build", "mcd_op_create", "mcd_hamiltonian_apply", "mcd_lanczos_ground",
              "mcd_band_lanczos_green", "mcd_last_error", "mcd_op_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libmcd.so not built: run python -m paper_2509_22975_amd.build")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_argument_errors_without_device_work():
    import paper_2509_22975_amd as mcd
    L = mcd.lib()
    assert L.mcd_version() >= 10000
    # NULL output handle is rejected before any HIP call
    rc = L.mcd_op_create(None, None, 0, 0, 0, None, None, None)
    assert rc == -1
    assert b"NULL" in L.mcd_last_error()
    rc = L.mcd_lanczos_ground(None, None, None, None, None, None, None, None, None, None)
    assert rc == -1


def test_kept_band_run_entry_points_reject_null_handles():
    import paper_2509_22975_amd as mcd
    L = mcd.lib()
    L.mcd_band_keep_destroy(None)   # NULL is ignored
    fwd = [None, None, 0, None, 0.0, 0, None, None, 0, None, None, None, None, None, None, None,
           None]
    assert L.mcd_band_lanczos_green_keep(*fwd, None) == -1
    assert b"keep_out" in L.mcd_last_error()
    vjp = [None, None, 0, None, 0.0, 0, None, None, 0, None, None, None, 0.0, 0.0, 0, None,
           None, None, None, None, None]
    assert L.mcd_band_green_vjp_keep(*vjp, None) == -1
    assert b"keep" in L.mcd_last_error()


def test_workspace_handle_bookkeeping_without_device_work():
    """mcd_ws_create only records the caller's range (no device access): a
    handle over a stand-in address, its statistics, and the argument checks."""
    import paper_2509_22975_amd as mcd
    L = mcd.lib()
    h = ctypes.c_void_p()
    assert L.mcd_ws_create(ctypes.c_void_p(1 << 20), 1 << 20, ctypes.byref(h)) == 0
    sz, used, high, need = (ctypes.c_size_t() for _ in range(4))
    assert L.mcd_ws_stats(h, ctypes.byref(sz), ctypes.byref(used), ctypes.byref(high),
                          ctypes.byref(need)) == 0
    assert (sz.value, used.value, high.value, need.value) == (1 << 20, 0, 0, 0)
    L.mcd_ws_destroy(h)
    L.mcd_ws_destroy(None)
    # misaligned base, NULL output
    assert L.mcd_ws_create(ctypes.c_void_p((1 << 20) + 8), 4096, ctypes.byref(h)) == -1
    assert L.mcd_ws_create(ctypes.c_void_p(1 << 20), 4096, None) == -1
    # size queries that need no device: on-the-fly operator, Lanczos on a NULL op
    bq = ctypes.c_size_t()
    assert L.mcd_lanczos_workspace_size(None, None, ctypes.byref(bq)) == -1
