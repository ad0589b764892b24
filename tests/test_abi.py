"""The C ABI library loads and exports every entry point include/fdbscan.h
declares; host-side argument checks and workspace sizing need no GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdbscan.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fdb_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared()
    for must in ("fdb_create", "fdb_destroy", "fdb_workspace_bytes", "fdb_dbscan", "fdb_last_info",
                 "fdb_last_status", "fdb_status_string", "fdb_set_timing", "fdb_stage_times", "fdb_dbscan_batched",
                 "fdb_tune", "fdb_tune_batched", "fdb_tuned_options"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2103_05162_amd import _lib
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (fdb_\w+)", out))
    assert set(_declared()) <= exported


def test_status_strings():
    from paper_2103_05162_amd import _lib
    assert _lib.status_string(0) == "ok"
    assert "invalid" in _lib.status_string(1)
    assert _lib.status_string(99) == "unknown status"


def test_workspace_is_linear_in_n_and_rejects_bad_arguments():
    from paper_2103_05162_amd import _lib
    for algo in ("fdbscan", "densebox"):
        for d in (2, 3):
            a = _lib.workspace_bytes(1 << 20, d, algo)
            b = _lib.workspace_bytes(1 << 21, d, algo)
            c = _lib.workspace_bytes(1 << 22, d, algo)
            assert a < b < c
            per_point = (c - b) / (1 << 21)
            assert abs((b - a) / (1 << 20) - per_point) < 1.0
            assert per_point < 400
    lib = _lib.load()
    out = ctypes.c_size_t(0)
    assert lib.fdb_workspace_bytes(10, 4, None, ctypes.byref(out)) == _lib.FDB_ERR_INVALID
    assert lib.fdb_workspace_bytes(-1, 3, None, ctypes.byref(out)) == _lib.FDB_ERR_INVALID
    assert lib.fdb_workspace_bytes(1 << 30, 3, None, ctypes.byref(out)) == _lib.FDB_ERR_INVALID
    bad = _lib.make_options("fdbscan", "canonical", leaf_size=-1)
    assert lib.fdb_workspace_bytes(10, 3, ctypes.byref(bad), ctypes.byref(out)) == _lib.FDB_ERR_INVALID
    bad = _lib.make_options("fdbscan", "canonical", block_size=100)
    assert lib.fdb_workspace_bytes(10, 3, ctypes.byref(bad), ctypes.byref(out)) == _lib.FDB_ERR_INVALID
    for tile in (-1, 4, 65):
        bad = _lib.make_options("densebox", "canonical", tile=tile)
        assert lib.fdb_workspace_bytes(10, 3, ctypes.byref(bad), ctypes.byref(out)) == _lib.FDB_ERR_INVALID
    bad = _lib.make_options("densebox", "canonical", flags=4)  # no such flag
    assert lib.fdb_workspace_bytes(10, 3, ctypes.byref(bad), ctypes.byref(out)) == _lib.FDB_ERR_INVALID
    for ok in (_lib.make_options("densebox", tile=8), _lib.make_options("densebox", tile=64, graph=True)):
        assert lib.fdb_workspace_bytes(10, 3, ctypes.byref(ok), ctypes.byref(out)) == 0
    assert lib.fdb_workspace_bytes(0, 2, None, ctypes.byref(out)) == 0


def test_options_struct_matches_the_header():
    """fdb_options is six 32-bit fields in the header's order (the binding mirrors it)."""
    import re as _re
    from paper_2103_05162_amd import _lib
    text = open(HEADER).read()
    body = _re.search(r"typedef struct \{(.*?)\} fdb_options;", text, flags=_re.S).group(1)
    body = _re.sub(r"/\*.*?\*/", "", body, flags=_re.S)
    fields = _re.findall(r"(?:int32_t|uint32_t)\s+(\w+);", body)
    assert fields == [f for f, _ in _lib.FdbOptions._fields_]
    assert ctypes.sizeof(_lib.FdbOptions) == 24


def test_tune_and_status_arguments_are_checked_before_any_gpu_call():
    from paper_2103_05162_amd import _lib
    lib = _lib.load()
    best = _lib.FdbOptions()
    ms = (ctypes.c_double * 2)()
    assert lib.fdb_tune(None, None, 10, 3, ctypes.c_float(0.1), 5, None, 3, None, None, None, 0, None,
                        ctypes.byref(best), ms) == _lib.FDB_ERR_INVALID
    assert lib.fdb_tune_batched(None, None, 10, None, 1, 3, None, None, None, 3, None, None, None, None, 0, None,
                                ctypes.byref(best), ms) == _lib.FDB_ERR_INVALID
    assert lib.fdb_tuned_options(None, 10, 3, 5, 0, None, ctypes.byref(best)) == _lib.FDB_ERR_INVALID
    v = ctypes.c_uint32(0)
    assert lib.fdb_last_status(None, None, ctypes.byref(v)) == _lib.FDB_ERR_INVALID
    assert "another thread" in _lib.status_string(_lib.FDB_ERR_BUSY)


def test_null_handle_is_rejected_before_any_gpu_call():
    from paper_2103_05162_amd import _lib
    lib = _lib.load()
    assert lib.fdb_dbscan(None, None, 0, 3, ctypes.c_float(0.1), 5, None, None, None, None, None, 0,
                          None) == _lib.FDB_ERR_INVALID
    lib.fdb_destroy(None)
    assert lib.fdb_create(None, 0) == _lib.FDB_ERR_INVALID


def test_batched_and_server_arguments_are_checked_before_any_gpu_call():
    from paper_2103_05162_amd import _lib
    lib = _lib.load()
    out = ctypes.c_size_t(0)
    assert lib.fdb_workspace_bytes_batched(100, 0, 3, None, ctypes.byref(out)) == _lib.FDB_ERR_INVALID
    assert lib.fdb_workspace_bytes_batched(100, 4, 5, None, ctypes.byref(out)) == _lib.FDB_ERR_INVALID
    assert lib.fdb_workspace_bytes_batched(100, 4, 3, None, ctypes.byref(out)) == 0
    one = out.value
    assert lib.fdb_workspace_bytes_batched(100, 4096, 3, None, ctypes.byref(out)) == 0
    assert out.value > one  # per-cloud arrays grow with the number of clouds
    srv = ctypes.c_void_p()
    opt = _lib.make_options("densebox")
    assert lib.fdb_server_create(0, 1 << 30, 16, 7, ctypes.byref(opt), ctypes.byref(srv)) == _lib.FDB_ERR_INVALID
    assert lib.fdb_server_create(0, 1 << 30, 0, 0, ctypes.byref(opt), ctypes.byref(srv)) == _lib.FDB_ERR_INVALID
    assert lib.fdb_server_create(0, 1000, 16, 0, ctypes.byref(opt), ctypes.byref(srv)) == _lib.FDB_ERR_INVALID
    bad = _lib.make_options("fdbscan", "canonical", leaf_size=-1)
    assert lib.fdb_server_create(0, 1 << 30, 16, 0, ctypes.byref(bad), ctypes.byref(srv)) == _lib.FDB_ERR_INVALID
    assert lib.fdb_server_create(0, 1 << 30, 16, 0, None, None) == _lib.FDB_ERR_INVALID
    job = _lib.FdbJob(None, 0, 3, ctypes.c_float(0.1), 3, None, None)
    t = ctypes.c_int64(0)
    assert lib.fdb_server_submit(None, ctypes.byref(job), ctypes.byref(t)) == _lib.FDB_ERR_INVALID
    assert lib.fdb_server_poll(None, 0, None) == _lib.FDB_ERR_INVALID
    assert lib.fdb_server_drain(None) == _lib.FDB_ERR_INVALID
    lib.fdb_server_destroy(None)


def test_out_of_core_arguments_are_checked_before_any_gpu_call():
    import numpy as np
    from paper_2103_05162_amd import _lib
    lib = _lib.load()
    offs = np.array([0, 3, 5], np.int64)
    eps = np.array([0.1, 0.1], np.float32)
    mp = np.array([2, 2], np.int32)
    pts = np.zeros((5, 3), np.float32)
    lab = np.zeros(5, np.int32)
    k = np.zeros(2, np.int32)
    args = [pts.ctypes.data, offs.ctypes.data, 2, 3, eps.ctypes.data, mp.ctypes.data, None, 1 << 30,
            lab.ctypes.data, None, k.ctypes.data]
    assert lib.fdb_dbscan_batched_host(None, *args) == _lib.FDB_ERR_INVALID  # no handle
