"""Thin ctypes binding of libfspbb.so (include/fspbb.h).

Argument marshalling only: every step of the bound runs in the library's HIP
kernels.  Device buffers are torch tensors (torch is used for device memory
and streams); each function has the name of the C entry point it calls,
without the ``fsp_`` prefix.  Importing this module does not need a GPU;
calling into the library does, and the calls raise if the library has not
been built (``python -m paper_1208_3933_amd.build``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfspbb.so")

OK = 0
E_INVAL = -1
E_RANGE = -2
E_NOMEM = -3
E_DEVICE = -4
E_BADNODE = -5
E_NODEVICE = -6
BUDGET = 1
PENDING = 2
LB_INVALID = -1

INSTANCE_HEADS = 1
INSTANCE_PAIR_SUBSET = 2

UB_NEH = -1
UB_NONE = 0x7FFFFFFF

VARIANT_AUTO = 0
VARIANT_LANE32 = 1
VARIANT_PACKED16 = 2
VARIANT_WAVEPAIR = 3
VARIANT_WIDE = 4

_i32p = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p


class FspError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} {last_error_string()}".strip())


class InstanceInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("pairs", ctypes.c_int32),
                ("max_value", ctypes.c_int32), ("packed16", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("table_bytes", ctypes.c_int64)]


class StepResult(ctypes.Structure):
    _fields_ = [("n_children", ctypes.c_int64), ("n_survivors", ctypes.c_int64), ("ub_out", ctypes.c_int32),
                ("improved", ctypes.c_int32), ("fingerprint", ctypes.c_int64)]


class SolveResult(ctypes.Structure):
    _fields_ = [("opt", ctypes.c_int32), ("proven", ctypes.c_int32), ("nodes_bounded", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("ub0", ctypes.c_int32), ("improvements", ctypes.c_int32),
                ("max_stack", ctypes.c_int64)]


class ExploreResult(ctypes.Structure):
    _fields_ = [("opt", ctypes.c_int32), ("proven", ctypes.c_int32), ("nodes_bounded", ctypes.c_int64),
                ("pools", ctypes.c_int64), ("threads", ctypes.c_int32), ("ub0", ctypes.c_int32),
                ("seconds", ctypes.c_double)]


class PoolDesc(ctypes.Structure):
    _fields_ = [("inst", ctypes.c_void_p), ("prefixes", ctypes.c_void_p), ("depths", ctypes.c_void_p),
                ("N", ctypes.c_int64), ("out_lb", ctypes.c_void_p)]


BATCH_GRAPH = 1

FORM_PERSISTENT = 0
FORM_GRID = 1


class TuneResult(ctypes.Structure):
    _fields_ = [("waves_per_group", ctypes.c_int32), ("candidates", ctypes.c_int32), ("best_us", ctypes.c_double),
                ("default_us", ctypes.c_double), ("cand_wpg", ctypes.c_int32 * 8), ("cand_us", ctypes.c_double * 8),
                ("form", ctypes.c_int32), ("reserved", ctypes.c_int32), ("grid_us", ctypes.c_double),
                ("persistent_us", ctypes.c_double)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_int64), ("max_active", ctypes.c_int32),
                ("tick_children", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("active", ctypes.c_int32), ("pending", ctypes.c_int32), ("mem_used", ctypes.c_int64),
                ("ticks", ctypes.c_int64), ("nodes_bounded", ctypes.c_int64), ("last_children", ctypes.c_int64),
                ("last_searches", ctypes.c_int32), ("swap_outs", ctypes.c_int64), ("swap_ins", ctypes.c_int64)]


_lib = None
_SIGNATURES = {
    "fsp_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "fsp_last_error_string": (ctypes.c_char_p, []),
    "fsp_create_instance": (ctypes.c_int32, [_i32p, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_vp)]),
    "fsp_create_instance_ex": (ctypes.c_int32, [_i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.POINTER(_vp)]),
    "fsp_create_instance_pairs": (ctypes.c_int32, [_i32p, ctypes.c_int32, ctypes.c_int32, _i32p, ctypes.c_int32,
                                                   ctypes.c_int32, ctypes.POINTER(_vp)]),
    "fsp_destroy_instance": (ctypes.c_int32, [_vp]),
    "fsp_get_instance_info": (ctypes.c_int32, [_vp, ctypes.POINTER(InstanceInfo)]),
    "fsp_bound_pool": (ctypes.c_int32, [_vp, _vp, _vp, ctypes.c_int64, _vp, _vp]),
    "fsp_bound_pool_variant": (ctypes.c_int32, [_vp, _vp, _vp, ctypes.c_int64, _vp, ctypes.c_int32, _vp]),
    "fsp_bound_pool_noalloc": (ctypes.c_int32, [_vp, _vp, _vp, ctypes.c_int64, _vp, _vp]),
    "fsp_noalloc_max_nodes": (ctypes.c_int64, [_vp]),
    "fsp_pool_status": (ctypes.c_int32, [_vp, _vp, ctypes.POINTER(ctypes.c_int64)]),
    "fsp_neh": (ctypes.c_int32, [_vp, _i32p, ctypes.POINTER(ctypes.c_int32)]),
    "fsp_branch_and_prune": (ctypes.c_int32, [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp, _vp,
                                              ctypes.c_int64, _vp, ctypes.POINTER(StepResult), _vp]),
    "fsp_solve": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(SolveResult),
                                   _i32p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, _vp]),
    "fsp_solve_ex": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.POINTER(SolveResult), _i32p, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.c_int64, _vp]),
    "fsp_explore": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.POINTER(ExploreResult), _i32p, _vp]),
    "fsp_batch_create": (ctypes.c_int32, [ctypes.POINTER(PoolDesc), ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(_vp)]),
    "fsp_batch_run": (ctypes.c_int32, [_vp, _vp]),
    "fsp_batch_destroy": (ctypes.c_int32, [_vp]),
    "fsp_batch_info": (ctypes.c_int32, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "fsp_bound_pools_batched": (ctypes.c_int32, [ctypes.POINTER(PoolDesc), ctypes.c_int32, _vp]),
    "fsp_autotune": (ctypes.c_int32, [_vp, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(TuneResult)]),
    "fsp_tune_get": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32)]),
    "fsp_tune_set": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "fsp_tune_get_form": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "fsp_tune_set_form": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "fsp_tune_save": (ctypes.c_int32, [ctypes.c_char_p]),
    "fsp_tune_load": (ctypes.c_int32, [ctypes.c_char_p]),
    "fsp_server_create": (ctypes.c_int32, [ctypes.POINTER(ServerConfig), _vp, ctypes.POINTER(_vp)]),
    "fsp_server_submit": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.POINTER(ctypes.c_int64)]),
    "fsp_server_step": (ctypes.c_int32, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ServerStats)]),
    "fsp_server_poll": (ctypes.c_int32, [_vp, ctypes.c_int64, ctypes.POINTER(SolveResult), _i32p]),
    "fsp_server_destroy": (ctypes.c_int32, [_vp]),
    "fsp_timing_enable": (ctypes.c_int32, [_vp, ctypes.c_int32]),
    "fsp_timing_read": (ctypes.c_int32, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64)]),
    "fsp_probe_peak": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int64, _vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]),
    "fsp_release_cached": (ctypes.c_int32, []),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1208_3933_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().fsp_status_string(int(status)).decode()


def last_error_string() -> str:
    return lib().fsp_last_error_string().decode()


def _check(status: int, what: str) -> int:
    if status < 0:
        raise FspError(status, what)
    return status


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev_i32(t, name, shape=None):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous int32 CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


class Instance:
    """An instance created by fsp_create_instance (owns the device tables)."""

    def __init__(self, p, heads: bool = False, pairs=None):
        p = np.ascontiguousarray(p, dtype=np.int32)
        if p.ndim != 2:
            raise ValueError("p must be an n x m matrix")
        self.n, self.m = int(p.shape[0]), int(p.shape[1])
        h = _vp()
        if pairs is not None:
            pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
            st = lib().fsp_create_instance_pairs(p.ctypes.data_as(_i32p), self.n, self.m, pr.ctypes.data_as(_i32p),
                                                 int(pr.shape[0]), INSTANCE_HEADS if heads else 0, ctypes.byref(h))
        elif heads:
            st = lib().fsp_create_instance_ex(p.ctypes.data_as(_i32p), self.n, self.m, INSTANCE_HEADS,
                                              ctypes.byref(h))
        else:
            st = lib().fsp_create_instance(p.ctypes.data_as(_i32p), self.n, self.m, ctypes.byref(h))
        _check(st, "fsp_create_instance")
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("instance destroyed")
        return self._h

    def info(self) -> dict:
        return get_instance_info(self)

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().fsp_destroy_instance(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def create_instance(p, heads: bool = False, pairs=None) -> Instance:
    """heads: releases as the earliest starts of unscheduled jobs (FSP_INSTANCE_HEADS);
    pairs: (P, 2) machine pairs (k, l), k < l, the bound takes its maximum over
    (fsp_create_instance_pairs), else every pair."""
    return Instance(p, heads, pairs)


def destroy_instance(inst: Instance) -> None:
    inst.close()


def get_instance_info(inst: Instance) -> dict:
    info = InstanceInfo()
    _check(lib().fsp_get_instance_info(inst.handle, ctypes.byref(info)), "fsp_get_instance_info")
    return {f: getattr(info, f) for f, _ in InstanceInfo._fields_}


def bound_pool(inst: Instance, prefixes, depths, out_lb, stream=None, variant: int = VARIANT_AUTO) -> None:
    """Enqueue the bound of every node of a pool (async on the stream)."""
    N = int(depths.shape[0])
    a = _dev_i32(prefixes, "prefixes", (N, inst.n))
    b = _dev_i32(depths, "depths", (N,))
    c = _dev_i32(out_lb, "out_lb", (N,))
    s = _stream_handle(stream)
    if variant == VARIANT_AUTO:
        st = lib().fsp_bound_pool(inst.handle, a, b, N, c, s)
    else:
        st = lib().fsp_bound_pool_variant(inst.handle, a, b, N, c, int(variant), s)
    _check(st, "fsp_bound_pool")


def bound_pool_noalloc(inst: Instance, prefixes, depths, out_lb, stream=None) -> None:
    """fsp_bound_pool_noalloc: the bound of every node of a pool with no
    allocation (the workspace is the library's fixed per-device array; calls
    that overlap on one device race)."""
    N = int(depths.shape[0])
    a = _dev_i32(prefixes, "prefixes", (N, inst.n))
    b = _dev_i32(depths, "depths", (N,))
    c = _dev_i32(out_lb, "out_lb", (N,))
    _check(lib().fsp_bound_pool_noalloc(inst.handle, a, b, N, c, _stream_handle(stream)), "fsp_bound_pool_noalloc")


def noalloc_max_nodes(inst: Instance) -> int:
    """Largest pool fsp_bound_pool_noalloc accepts for this instance."""
    return int(lib().fsp_noalloc_max_nodes(inst.handle))


def bound_pool_variant(inst: Instance, prefixes, depths, out_lb, variant: int, stream=None) -> None:
    bound_pool(inst, prefixes, depths, out_lb, stream, variant)


def pool_status(inst: Instance, stream=None) -> int:
    """Synchronise the stream; return the number of invalid nodes met since the last call."""
    n_bad = ctypes.c_int64(0)
    st = lib().fsp_pool_status(inst.handle, _stream_handle(stream), ctypes.byref(n_bad))
    if st != E_BADNODE:
        _check(st, "fsp_pool_status")
    return int(n_bad.value)


def timing_enable(inst: Instance, on: bool = True, chained: bool = False) -> None:
    """Event timing of each bound launch; chained: a launch's start is the
    previous launch's end (back-to-back launches on one stream), one event
    record fewer per launch."""
    _check(lib().fsp_timing_enable(inst.handle, (2 if chained else 1) if on else 0), "fsp_timing_enable")


def timing_read(inst: Instance):
    """(decode_ms, scan_ms, launches) summed over the launches since the last read."""
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    _check(lib().fsp_timing_read(inst.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
           "fsp_timing_read")
    return a.value, b.value, int(c.value)


def release_cached() -> None:
    """Returns the device scratch the library keeps for reuse to the driver."""
    _check(lib().fsp_release_cached(), "fsp_release_cached")


PROBE_VALU16, PROBE_VALU32, PROBE_LDS, PROBE_HBM = 0, 1, 2, 3


def probe_peak(kind: int, nbytes: int = 1 << 30, stream=None):
    """(rate, ms) of one peak-probe kernel on the current device: 16-bit or
    32-bit operations/s, or bytes/s for LDS and HBM (a copy of nbytes)."""
    rate, ms = ctypes.c_double(), ctypes.c_double()
    _check(lib().fsp_probe_peak(int(kind), int(nbytes), _stream_handle(stream), ctypes.byref(rate), ctypes.byref(ms)),
           "fsp_probe_peak")
    return rate.value, ms.value


def neh(inst: Instance):
    """(makespan, permutation) of the NEH heuristic."""
    perm = np.empty(inst.n, np.int32)
    ms = ctypes.c_int32()
    _check(lib().fsp_neh(inst.handle, perm.ctypes.data_as(_i32p), ctypes.byref(ms)), "fsp_neh")
    return int(ms.value), perm


def branch_and_prune(inst: Instance, parents, parent_depths, ub_in: int, children, child_depths,
                     child_lb=None, incumbent=None, stream=None) -> dict:
    """One branch-and-bound step (synchronous).  Survivors land in children /
    child_depths (/ child_lb) in child order.  Returns the step result."""
    K = int(parent_depths.shape[0])
    a = _dev_i32(parents, "parents", (K, inst.n))
    b = _dev_i32(parent_depths, "parent_depths", (K,))
    cap = int(child_depths.shape[0])
    c = _dev_i32(children, "children", (cap, inst.n))
    d = _dev_i32(child_depths, "child_depths", (cap,))
    e = _dev_i32(child_lb, "child_lb", (cap,)) if child_lb is not None else None
    f = _dev_i32(incumbent, "incumbent", (inst.n,)) if incumbent is not None else None
    res = StepResult()
    st = lib().fsp_branch_and_prune(inst.handle, a, b, K, int(ub_in), c, d, e, cap, f, ctypes.byref(res),
                                    _stream_handle(stream))
    out = {fn: getattr(res, fn) for fn, _ in StepResult._fields_}
    out["status"] = st
    if st not in (OK, E_RANGE, E_BADNODE):
        _check(st, "fsp_branch_and_prune")
    return out


SOLVE_BEST_FIRST = 1
SOLVE_DEVICE_STEPS = 2


def solve(inst: Instance, ub0: int = UB_NEH, pool_cap: int = 1 << 18, node_budget: int = 1 << 62,
          steplog_cap: int = 0, stream=None, best_first: bool = False, device_steps: bool = False) -> dict:
    """Branch-and-bound with the search state on the device: depth first
    (stack), or best first (frontier ordered by bound and insertion);
    device_steps: depth first with the steps chosen on the device
    (FSP_SOLVE_DEVICE_STEPS)."""
    res = SolveResult()
    perm = np.empty(inst.n, np.int32)
    log = np.zeros((max(steplog_cap, 1), 6), np.int64)
    flags = (SOLVE_BEST_FIRST if best_first else 0) | (SOLVE_DEVICE_STEPS if device_steps else 0)
    st = lib().fsp_solve_ex(inst.handle, int(ub0), int(pool_cap), int(node_budget), flags, ctypes.byref(res),
                            perm.ctypes.data_as(_i32p), log.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            int(steplog_cap), _stream_handle(stream))
    if st not in (OK, BUDGET):
        _check(st, "fsp_solve")
    out = {fn: getattr(res, fn) for fn, _ in SolveResult._fields_}
    out["status"] = st
    out["perm"] = perm
    out["steplog"] = log[:min(res.steps, steplog_cap)] if steplog_cap else None
    return out


def explore(inst: Instance, ub0: int = UB_NEH, threads: int = 8, pool_cap: int = 1 << 14,
            node_budget: int = 1 << 62, stream=None) -> dict:
    """Hybrid search: host explorer threads, shared GPU bounding of their pools."""
    res = ExploreResult()
    perm = np.empty(inst.n, np.int32)
    st = lib().fsp_explore(inst.handle, int(ub0), int(threads), int(pool_cap), int(node_budget),
                           ctypes.byref(res), perm.ctypes.data_as(_i32p), _stream_handle(stream))
    if st not in (OK, BUDGET):
        _check(st, "fsp_explore")
    out = {fn: getattr(res, fn) for fn, _ in ExploreResult._fields_}
    out["status"] = st
    out["perm"] = perm
    return out


def _pool_descs(pools):
    """pools: list of (instance, prefixes, depths, out_lb) with device tensors."""
    arr = (PoolDesc * len(pools))()
    keep = []
    for i, (inst, pre, dep, out) in enumerate(pools):
        N = int(dep.shape[0])
        arr[i].inst = inst.handle.value
        arr[i].prefixes = _dev_i32(pre, "prefixes", (N, inst.n)) if N else None
        arr[i].depths = _dev_i32(dep, "depths", (N,)) if N else None
        arr[i].N = N
        arr[i].out_lb = _dev_i32(out, "out_lb", (N,)) if N else None
        keep.append((inst, pre, dep, out))
    return arr, keep


class Batch:
    """A planned batch (fsp_batch_create); run() enqueues one bounding of every pool."""

    def __init__(self, pools, graph: bool = True):
        self._arr, self._keep = _pool_descs(pools)
        h = _vp()
        _check(lib().fsp_batch_create(self._arr, len(pools), BATCH_GRAPH if graph else 0, ctypes.byref(h)),
               "fsp_batch_create")
        self._h = h

    def run(self, stream=None):
        _check(lib().fsp_batch_run(self._h, _stream_handle(stream)), "fsp_batch_run")

    def info(self):
        t, k, g = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().fsp_batch_info(self._h, ctypes.byref(t), ctypes.byref(k), ctypes.byref(g)), "fsp_batch_info")
        return {"total_nodes": t.value, "items": k.value, "grid": g.value}

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().fsp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def batch_create(pools, graph: bool = True) -> Batch:
    return Batch(pools, graph)


def bound_pools_batched(pools, stream=None) -> None:
    arr, _keep = _pool_descs(pools)
    _check(lib().fsp_bound_pools_batched(arr, len(pools), _stream_handle(stream)), "fsp_bound_pools_batched")


def autotune(inst: Instance, sample_nodes: int = 16384, reps: int = 3) -> dict:
    """Time every scan tile schedule for the instance's shape and keep the fastest."""
    r = TuneResult()
    _check(lib().fsp_autotune(inst.handle, int(sample_nodes), int(reps), ctypes.byref(r)), "fsp_autotune")
    return {"waves_per_group": r.waves_per_group, "best_us": r.best_us, "default_us": r.default_us,
            "candidates": {int(r.cand_wpg[i]): float(r.cand_us[i]) for i in range(r.candidates)},
            "form": r.form, "grid_us": r.grid_us, "persistent_us": r.persistent_us}


def tune_get(n: int, m: int):
    """(waves_per_group, tuned) for a shape."""
    w, t = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().fsp_tune_get(int(n), int(m), ctypes.byref(w), ctypes.byref(t)), "fsp_tune_get")
    return int(w.value), bool(t.value)


def tune_set(n: int, m: int, waves_per_group: int) -> None:
    _check(lib().fsp_tune_set(int(n), int(m), int(waves_per_group)), "fsp_tune_set")


def tune_get_form(n: int, m: int) -> int:
    f = ctypes.c_int32()
    _check(lib().fsp_tune_get_form(int(n), int(m), ctypes.byref(f)), "fsp_tune_get_form")
    return int(f.value)


def tune_set_form(n: int, m: int, form: int) -> None:
    _check(lib().fsp_tune_set_form(int(n), int(m), int(form)), "fsp_tune_set_form")


def tune_save(path: str) -> None:
    _check(lib().fsp_tune_save(path.encode()), "fsp_tune_save")


def tune_load(path: str) -> None:
    _check(lib().fsp_tune_load(path.encode()), "fsp_tune_load")


class Server:
    """A serving loop of concurrent searches (fsp_server_*).  Instances given
    to submit() are kept referenced here until their search is polled."""

    def __init__(self, mem_budget_bytes: int, max_active: int = 64, tick_children: int = 0, stream=None):
        cfg = ServerConfig(int(mem_budget_bytes), int(max_active), int(tick_children))
        h = _vp()
        _check(lib().fsp_server_create(ctypes.byref(cfg), _stream_handle(stream), ctypes.byref(h)),
               "fsp_server_create")
        self._h = h
        self._insts = {}
        self._ids = np.zeros(4096, np.int64)

    def submit(self, inst: Instance, ub0: int = UB_NEH, pool_cap: int = 1 << 14, node_budget: int = 1 << 62) -> int:
        i = ctypes.c_int64()
        _check(lib().fsp_server_submit(self._h, inst.handle, int(ub0), int(pool_cap), int(node_budget),
                                       ctypes.byref(i)), "fsp_server_submit")
        self._insts[int(i.value)] = inst
        return int(i.value)

    def step(self):
        """One step call: (ids finished in it, stats dict)."""
        nd = ctypes.c_int32()
        st = ServerStats()
        rc = lib().fsp_server_step(self._h, self._ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   len(self._ids), ctypes.byref(nd), ctypes.byref(st))
        _check(rc, "fsp_server_step")
        ids = [int(x) for x in self._ids[:min(nd.value, len(self._ids))]]
        return ids, {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def poll(self, id_: int):
        """None while pending, else the result dict of fsp_solve (with status)."""
        res = SolveResult()
        inst = self._insts.get(int(id_))
        perm = np.empty(inst.n if inst is not None else 1, np.int32)
        st = lib().fsp_server_poll(self._h, int(id_), ctypes.byref(res), perm.ctypes.data_as(_i32p))
        if st == PENDING:
            return None
        if st not in (OK, BUDGET):
            _check(st, "fsp_server_poll")
        self._insts.pop(int(id_), None)
        out = {fn: getattr(res, fn) for fn, _ in SolveResult._fields_}
        out["status"] = st
        out["perm"] = perm
        return out

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().fsp_server_destroy(self._h)
            self._h = None
            self._insts = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def server_create(mem_budget_bytes: int, max_active: int = 64, tick_children: int = 0, stream=None) -> Server:
    return Server(mem_budget_bytes, max_active, tick_children, stream)
