"""ctypes wrapper around the C oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py, never by the library.  The oracle shares no code
with the GPU path; only the seeded input generator is common to both.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")
INVALID = -1

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


class Counts(ctypes.Structure):
    _fields_ = [("ptm", ctypes.c_int64), ("lm", ctypes.c_int64), ("rm", ctypes.c_int64),
                ("qm", ctypes.c_int64), ("mm", ctypes.c_int64)]


class BnbResult(ctypes.Structure):
    _fields_ = [("ub", ctypes.c_int32), ("proven", ctypes.c_int32),
                ("nodes_bounded", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("improvements", ctypes.c_int64), ("max_stack", ctypes.c_int64),
                ("seconds_total", ctypes.c_double), ("seconds_bound", ctypes.c_double)]


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so (plain -O2, no vectorising tricks)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-o", tmp, SRC_PATH])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_makespan.restype = ctypes.c_int32
        L.orc_makespan.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int]
        L.orc_bound.restype = ctypes.c_int32
        L.orc_bound.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int]
        L.orc_bound_tie.restype = ctypes.c_int32
        L.orc_bound_tie.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int,
                                    _i32p, ctypes.c_int]
        L.orc_bound_counted.restype = ctypes.c_int32
        L.orc_bound_counted.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int,
                                        ctypes.POINTER(Counts)]
        L.orc_pair_scan.restype = ctypes.c_int32
        L.orc_pair_scan.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, _i64p, _i64p]
        L.orc_bound_pool.restype = ctypes.c_int64
        L.orc_bound_pool.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, _i32p, _i32p,
                                     ctypes.c_int64, _i32p]
        L.orc_bound_heads.restype = ctypes.c_int32
        L.orc_bound_heads.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int]
        L.orc_bound_pool_mode.restype = ctypes.c_int64
        L.orc_bound_pool_mode.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, _i32p, _i32p,
                                          ctypes.c_int64, _i32p, ctypes.c_int]
        L.orc_brute.restype = ctypes.c_int32
        L.orc_brute.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int]
        L.orc_neh.restype = ctypes.c_int32
        L.orc_neh.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, _i32p]
        L.orc_bnb_best_first.restype = ctypes.c_int
        L.orc_bnb_best_first.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int32, _i32p,
                                         ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                         ctypes.POINTER(BnbResult), _i32p, _i64p, ctypes.c_int64, ctypes.c_int]
        L.orc_bnb.restype = ctypes.c_int
        L.orc_bnb.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int32, _i32p,
                              ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                              ctypes.POINTER(BnbResult), _i32p, _i64p, ctypes.c_int64, ctypes.c_int]
        L.orc_bound_pool_pairs.restype = ctypes.c_int64
        L.orc_bound_pool_pairs.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, _i32p, _i32p,
                                           ctypes.c_int64, _i32p, ctypes.c_int, _i32p, ctypes.c_int]
        L.orc_bnb_pairs.restype = ctypes.c_int
        L.orc_bnb_pairs.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int32, _i32p,
                                    ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                    ctypes.POINTER(BnbResult), _i32p, _i64p, ctypes.c_int64, ctypes.c_int,
                                    ctypes.c_int, _i32p, ctypes.c_int]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_i32p)


def _mat(p):
    p = np.ascontiguousarray(p, dtype=np.int32)
    assert p.ndim == 2
    return p, p.shape[0], p.shape[1]


def _seq(s):
    return np.ascontiguousarray(np.asarray(s, dtype=np.int32).reshape(-1))


def makespan(p, seq) -> int:
    p, n, m = _mat(p)
    s = _seq(seq)
    return int(lib().orc_makespan(_p(p), n, m, _p(s), len(s)))


def bound(p, prefix) -> int:
    p, n, m = _mat(p)
    s = _seq(prefix)
    buf = np.zeros(max(n, 1), np.int32)
    buf[:len(s)] = s
    return int(lib().orc_bound(_p(p), n, m, _p(buf), len(s)))


def bound_heads(p, prefix) -> int:
    """The bound with the heads variant of the machine releases."""
    p, n, m = _mat(p)
    s = _seq(prefix)
    buf = np.zeros(max(n, 1), np.int32)
    buf[:len(s)] = s
    return int(lib().orc_bound_heads(_p(p), n, m, _p(buf), len(s)))


def bound_tie(p, prefix, tiekey, eq_in_s2: bool) -> int:
    p, n, m = _mat(p)
    s = _seq(prefix)
    buf = np.zeros(max(n, 1), np.int32)
    buf[:len(s)] = s
    t = _seq(tiekey)
    return int(lib().orc_bound_tie(_p(p), n, m, _p(buf), len(s), _p(t), int(eq_in_s2)))


def bound_counted(p, prefix):
    p, n, m = _mat(p)
    s = _seq(prefix)
    buf = np.zeros(max(n, 1), np.int32)
    buf[:len(s)] = s
    c = Counts()
    v = lib().orc_bound_counted(_p(p), n, m, _p(buf), len(s), ctypes.byref(c))
    return int(v), {f: getattr(c, f) for f, _ in Counts._fields_}


def pair_scan(p, prefix, k: int, l: int):
    """(finishing time on machine l after the scan of pair (k,l), tail of machine l)."""
    p, n, m = _mat(p)
    s = _seq(prefix)
    buf = np.zeros(max(n, 1), np.int32)
    buf[:len(s)] = s
    t2, q = ctypes.c_int64(), ctypes.c_int64()
    rc = lib().orc_pair_scan(_p(p), n, m, _p(buf), len(s), k, l, ctypes.byref(t2), ctypes.byref(q))
    if rc != 0:
        raise ValueError("invalid node or pair")
    return int(t2.value), int(q.value)


def _pairs(pairs):
    """The pair subset as a contiguous (P, 2) int32 array, or None for every pair."""
    if pairs is None:
        return None
    a = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    assert a.shape[0] >= 1
    return a


def bound_pool(p, prefixes, depths, heads: bool = False, pairs=None) -> np.ndarray:
    """Bounds of a pool (heads: the heads variant; pairs: the maximum over
    these machine pairs (k, l) only, else over every pair)."""
    p, n, m = _mat(p)
    pre = np.ascontiguousarray(prefixes, dtype=np.int32).reshape(-1, n)
    dep = np.ascontiguousarray(depths, dtype=np.int32).reshape(-1)
    assert pre.shape[0] == dep.shape[0]
    out = np.empty(dep.shape[0], np.int32)
    pr = _pairs(pairs)
    if pr is not None:
        lib().orc_bound_pool_pairs(_p(p), n, m, _p(pre), _p(dep), dep.shape[0], _p(out), int(heads), _p(pr),
                                   pr.shape[0])
    elif heads:
        lib().orc_bound_pool_mode(_p(p), n, m, _p(pre), _p(dep), dep.shape[0], _p(out), 1)
    else:
        lib().orc_bound_pool(_p(p), n, m, _p(pre), _p(dep), dep.shape[0], _p(out))
    return out


def brute(p, prefix=()) -> int:
    p, n, m = _mat(p)
    s = _seq(prefix)
    buf = np.zeros(max(n, 1), np.int32)
    buf[:len(s)] = s
    return int(lib().orc_brute(_p(p), n, m, _p(buf), len(s)))


def neh(p):
    p, n, m = _mat(p)
    perm = np.empty(n, np.int32)
    ms = lib().orc_neh(_p(p), n, m, _p(perm))
    return int(ms), perm


def bnb(p, ub0: int, incumbent0=None, pool_cap: int = 1 << 18, node_budget: int = 1 << 62,
        strict_gt: bool = False, steplog_cap: int = 0, heads: bool = False, best_first: bool = False,
        pairs=None):
    """Pool-synchronous branch-and-bound, depth-first or best-first (heads:
    the heads variant of the bound; pairs: the bound over these machine
    pairs only).  Returns a dict; for best-first, max_stack is the largest
    frontier."""
    p, n, m = _mat(p)
    res = BnbResult()
    inc = np.empty(n, np.int32)
    inc0 = None if incumbent0 is None else _seq(incumbent0)
    log = np.zeros((max(steplog_cap, 1), 6), np.int64)
    pr = _pairs(pairs)
    args = (_p(p), n, m, int(ub0), None if inc0 is None else _p(inc0), int(pool_cap), int(node_budget),
            int(strict_gt), ctypes.byref(res), _p(inc), log.ctypes.data_as(_i64p), int(steplog_cap), int(heads))
    if pr is not None:
        rc = lib().orc_bnb_pairs(*args, int(best_first), _p(pr), pr.shape[0])
    else:
        rc = (lib().orc_bnb_best_first if best_first else lib().orc_bnb)(*args)
    if rc != 0:
        raise ValueError("bad arguments")
    return {"ub": int(res.ub), "proven": bool(res.proven), "nodes_bounded": int(res.nodes_bounded),
            "steps": int(res.steps), "improvements": int(res.improvements),
            "max_stack": int(res.max_stack), "incumbent": inc,
            "seconds_total": float(res.seconds_total), "seconds_bound": float(res.seconds_bound),
            "steplog": log[:min(int(res.steps), steplog_cap)] if steplog_cap else None}
