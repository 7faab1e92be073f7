"""Shared helpers for the tests: seeded workloads, oracle fan-out, device setup."""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_1208_3933_amd import gen

# The pool workloads (n, m, pool size) of the plain bounding configurations.
CONFIG_SHAPES = {0: (20, 5, 4096), 1: (50, 10, 65536), 2: (200, 20, 262144)}


def workload(config: int, n: int, m: int, count: int, instance: int = 0, dmin=0, dmax=None):
    p = gen.processing_times(n, m, gen.make_seed(config, instance, gen.PURPOSE_TIMES))
    pre, dep = gen.random_pool(n, count, gen.make_seed(config, instance, gen.PURPOSE_POOL), dmin, dmax)
    return p, pre, dep


def host_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def oracle_bounds(p, prefixes, depths, threads: int | None = None) -> np.ndarray:
    """Oracle bounds of a pool, fanned out over host threads (each call is the
    plain single-threaded oracle on a slice)."""
    threads = threads or host_threads()
    N = depths.shape[0]
    if N == 0:
        return np.zeros(0, np.int32)
    chunks = np.array_split(np.arange(N), min(threads * 4, N))
    out = np.empty(N, np.int32)
    with cf.ThreadPoolExecutor(threads) as ex:
        futs = {ex.submit(oracle.bound_pool, p, prefixes[c], depths[c]): c for c in chunks if len(c)}
        for f, c in futs.items():
            out[c] = f.result()
    return out


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1208_3933_amd import fspbb
    fspbb.lib()  # raises if the HIP library is missing
    return torch


def to_dev(torch, *arrays):
    return [torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for a in arrays]


def host_dfs_steps(p, ub0, pool_cap, nsteps):
    """The first nsteps pool steps of the depth-first search of the oracle's
    order rules, built on the host with every child bounded by the oracle
    (fanned out over host threads).  Returns per step the step-log row
    [parents, children, UB, pushed, stack, fingerprint], the parents in pop
    order and the survivors (rows, bounds) in child order."""
    n = p.shape[0]
    ub = int(ub0)
    root = int(oracle.bound(p, []))
    stack_rows = [np.zeros(n, np.int32)] if root < ub else []
    stack_dep = [0] if root < ub else []
    nodes, out = 1, []
    for _ in range(nsteps):
        if not stack_rows:
            break
        par_rows, par_dep, nchild = [], [], 0
        while stack_rows:
            c = n - stack_dep[-1]
            if par_rows and nchild + c > pool_cap:
                break
            nchild += c
            par_rows.append(stack_rows.pop())
            par_dep.append(stack_dep.pop())
        kids, kdep, kjob = [], [], []
        for row, d in zip(par_rows, par_dep):
            sched = np.zeros(n, bool)
            sched[row[:d]] = True
            free = np.nonzero(~sched)[0]
            block = np.zeros((len(free), n), np.int32)
            block[:, :d] = row[:d]
            block[:, d] = free
            kids.append(block)
            kdep.append(np.full(len(free), d + 1, np.int32))
            kjob.append(free.astype(np.int64))
        kids, kdep, kjob = np.concatenate(kids), np.concatenate(kdep), np.concatenate(kjob)
        lbs = oracle_bounds(p, kids, kdep)
        nodes += len(kdep)
        leaf = np.nonzero((kdep == n) & (lbs < ub))[0]
        if len(leaf):
            best = leaf[np.argmin(lbs[leaf])]  # argmin takes the first of equal values
            ub = int(lbs[best])
        keep = np.nonzero((kdep < n) & (lbs < ub))[0]
        S = len(keep)
        fp = int(((S - np.arange(S)) * (kjob[keep] + 1)).sum())
        for i in keep[::-1]:
            stack_rows.append(kids[i])
            stack_dep.append(int(kdep[i]))
        out.append({"log": [len(par_rows), len(kdep), ub, S, len(stack_rows), fp],
                    "parents": (np.array(par_rows), np.array(par_dep, np.int32)),
                    "ub_in": None, "survivors": (kids[keep], kdep[keep], lbs[keep]), "nodes": nodes})
    ubs = [int(ub0)] + [s["log"][2] for s in out]
    for s, u in zip(out, ubs):
        s["ub_in"] = u
    return out


def survivors_digest(rows, depths, lbs) -> str:
    """SHA-256 of a step's survivors in order: each survivor's prefix (up to
    the largest depth), depth and bound as little-endian int32."""
    d = int(depths.max()) if len(depths) else 0
    a = np.concatenate([np.asarray(rows)[:, :d], np.asarray(depths)[:, None], np.asarray(lbs)[:, None]], axis=1)
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()


GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name: str):
    with open(os.path.join(GOLDEN_DIR, name)) as f:
        return json.load(f)
