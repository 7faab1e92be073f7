"""The C ABI library loads and exports every symbol its header declares, and
argument checks that need no device behave as documented (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1208_3933_amd import fspbb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if f.endswith(".h"):
            text = open(os.path.join(inc, f)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(fsp_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_symbols()
    for want in ["fsp_create_instance", "fsp_destroy_instance", "fsp_bound_pool", "fsp_pool_status"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    L = fspbb.lib()
    missing = [n for n in declared_symbols() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings():
    for code in [0, -1, -2, -3, -4, -5, -6, 1]:
        assert fspbb.status_string(code).startswith("FSP_")


@pytest.mark.parametrize("n,m,bad", [(0, 5, None), (5, 1, None), (513, 5, None), (5, 33, None),
                                     (4, 3, (1, 2, -7))])
def test_create_instance_rejects_bad_arguments(n, m, bad):
    L = fspbb.lib()
    p = np.ones((max(n, 1), max(m, 1)), np.int32)
    if bad:
        p[bad[0], bad[1]] = bad[2]
    h = ctypes.c_void_p()
    st = L.fsp_create_instance(p.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n, m, ctypes.byref(h))
    assert st == fspbb.E_INVAL and not h.value


def test_create_instance_rejects_overflow():
    L = fspbb.lib()
    p = np.full((100, 20), 30_000_000, np.int32)
    h = ctypes.c_void_p()
    st = L.fsp_create_instance(p.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 100, 20, ctypes.byref(h))
    assert st == fspbb.E_RANGE


def test_null_arguments():
    L = fspbb.lib()
    assert L.fsp_create_instance(None, 3, 3, None) == fspbb.E_INVAL
    assert L.fsp_bound_pool(None, None, None, 0, None, None) == fspbb.E_INVAL
    assert L.fsp_destroy_instance(None) == fspbb.OK
    assert L.fsp_get_instance_info(None, None) == fspbb.E_INVAL
    assert L.fsp_pool_status(None, None, None) == fspbb.E_INVAL
    assert L.fsp_release_cached() == fspbb.OK  # nothing allocated in this process
    rate = ctypes.c_double()
    assert L.fsp_probe_peak(fspbb.PROBE_VALU16, 0, None, None, None) == fspbb.E_INVAL
    for kind, nbytes in [(-1, 1 << 20), (4, 1 << 20), (fspbb.PROBE_HBM, 1 << 19), (fspbb.PROBE_HBM, (1 << 20) + 8)]:
        assert L.fsp_probe_peak(kind, nbytes, None, ctypes.byref(rate), None) == fspbb.E_INVAL


def test_tuning_table_roundtrip(tmp_path):
    assert fspbb.tune_get(37, 7)[1] is False
    w0, _ = fspbb.tune_get(37, 7)
    assert w0 in (1, 2, 4, 8, 16)
    fspbb.tune_set(37, 7, 4)
    assert fspbb.tune_get(37, 7) == (4, True)
    path = str(tmp_path / "tune.txt")
    assert fspbb.tune_get_form(37, 7) == fspbb.FORM_GRID
    fspbb.tune_set_form(37, 7, fspbb.FORM_PERSISTENT)
    fspbb.tune_save(path)
    fspbb.tune_set(37, 7, 16)
    fspbb.tune_set_form(37, 7, fspbb.FORM_GRID)
    fspbb.tune_load(path)
    assert fspbb.tune_get(37, 7) == (4, True)
    assert fspbb.tune_get_form(37, 7) == fspbb.FORM_PERSISTENT
    with pytest.raises(fspbb.FspError):
        fspbb.tune_set_form(37, 7, 2)
    with pytest.raises(fspbb.FspError):
        fspbb.tune_set(37, 7, 3)


def test_rule_of_thumb_schedules():
    # about four machine pairs per wave and chain, at most 16 waves per group
    assert fspbb.tune_get(200, 20)[0] == 16   # 190 pairs
    assert fspbb.tune_get(50, 10)[0] == 8     # 45 pairs
    assert fspbb.tune_get(20, 5)[0] == 2      # 10 pairs
    assert fspbb.tune_get(9, 2)[0] == 1       # 1 pair


def test_create_instance_pairs_rejects_bad_pair_lists():
    L = fspbb.lib()
    p = np.ones((6, 4), np.int32)
    pp = p.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    for pairs in [[], [(0, 0)], [(2, 1)], [(0, 4)], [(-1, 2)], [(0, 3), (0, 3)], [(0, 3)] * 7, [(0, 1), (1, 2)]]:
        a = np.asarray(pairs, np.int32).reshape(-1, 2)
        h = ctypes.c_void_p()
        st = L.fsp_create_instance_pairs(pp, 6, 4, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(pairs), 0,
                                         ctypes.byref(h))
        assert st == fspbb.E_INVAL and not h.value, pairs
    assert L.fsp_create_instance_pairs(pp, 6, 4, None, 1, 0, ctypes.byref(ctypes.c_void_p())) == fspbb.E_INVAL


def test_binding_fails_loudly_without_the_library(monkeypatch):
    """With no built library every call raises: there is no fallback path."""
    monkeypatch.setattr(fspbb, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libfspbb.so"))
    monkeypatch.setattr(fspbb, "_lib", None)
    with pytest.raises(RuntimeError, match="is missing"):
        fspbb.lib()
    with pytest.raises(RuntimeError, match="is missing"):
        fspbb.create_instance(np.ones((5, 3), np.int32))


def test_noalloc_entry_points_reject_a_null_instance():
    # argument checks only: nothing reaches a device
    L = fspbb.lib()
    assert L.fsp_noalloc_max_nodes(None) == -1
    assert L.fsp_bound_pool_noalloc(None, None, None, 1, None, None) == fspbb.E_INVAL
