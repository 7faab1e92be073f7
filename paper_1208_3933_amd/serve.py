"""Serving workload driver over the library's serving loop (fsp_server_*).

A stream of depth-first branch-and-bound solves (each from the NEH upper
bound, with a node budget) over seeded instances of mixed shape arrives as a
Poisson process; the driver submits each request at its arrival time, calls
the server's step while work is pending, and records each request's latency
from arrival to result on the host.  Instances are created once and stay
resident on the device (their tables are reused by every request on them).

Requests are drawn from instances screened beforehand by solving each alone
(fsp_solve, same pool_cap and budget): instances proven optimal within the
budget enter the stream; the others are reported by shape.  The largest
shapes (200 x 20, and 500 x 20 whose tables do not fit LDS) rarely close
within any budget on random U[1,99] instances; they enter the stream as
searches stopped by a smaller node budget of their own, whose results are as
deterministic as a proof, and their latency is reported apart.  The
screened alone results are also the reference each served result must equal.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import fspbb, gen

# Instance shapes of the serving stream and their sampling weights (small
# shapes more frequent).
SHAPES = [(20, 5), (20, 10), (50, 5), (50, 10), (100, 5), (100, 10), (200, 10), (200, 20), (500, 20)]
WEIGHTS = [6, 5, 4, 3, 3, 2, 2, 1, 1]
CONFIG = 4
# Shapes served as budget-stopped searches (node budget of their own).
BUDGETED = {(200, 20), (500, 20)}
RESULT_FIELDS = ("opt", "proven", "nodes_bounded", "steps", "ub0", "improvements", "max_stack", "status")


@dataclass
class Candidate:
    shape: int
    seed: int
    p: np.ndarray
    inst: object = None
    alone: dict = field(default_factory=dict)
    alone_s: float = 0.0
    budgeted: bool = False  # served as a budget-stopped search
    budget: int = 0         # its node budget (0: the stream's)


def candidates(seeds_per_shape: int, shapes=SHAPES, budgeted_budget: int = 0) -> list:
    """Seeded instances per shape.  With budgeted_budget > 0, the shapes of
    BUDGETED are served as searches stopped after that many nodes."""
    out = []
    for si, (n, m) in enumerate(shapes):
        for i in range(seeds_per_shape):
            p = gen.processing_times(n, m, gen.make_seed(CONFIG, si * 1000 + i, gen.PURPOSE_TIMES))
            c = Candidate(si, i, p)
            if budgeted_budget > 0 and (n, m) in BUDGETED:
                c.budgeted, c.budget = True, budgeted_budget
            out.append(c)
    return out


def screen(cands, pool_cap: int, budget: int, stream=None) -> None:
    """Creates each candidate's instance and solves it alone (timed)."""
    import torch
    for c in cands:
        if c.inst is None:
            c.inst = fspbb.create_instance(c.p)
        if not c.budget:
            c.budget = budget
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.alone = fspbb.solve(c.inst, fspbb.UB_NEH, pool_cap, c.budget, 0, stream)
        c.alone_s = time.perf_counter() - t0


def sample_requests(cands, count: int, seed: int) -> list:
    """count candidates drawn with replacement: a shape by WEIGHTS among the
    shapes with servable candidates (proven, or budget-stopped by design),
    then one of its servable candidates uniformly."""
    proven = {}
    for k, c in enumerate(cands):
        if c.alone.get("proven") or c.budgeted:
            proven.setdefault(c.shape, []).append(k)
    shapes = sorted(proven)
    if not shapes:
        return []
    w = np.array([WEIGHTS[s] for s in shapes], np.float64)
    cum = np.cumsum(w / w.sum())
    u = gen.uniform01(seed, 2 * count)
    out = []
    for r in range(count):
        s = shapes[min(int(np.searchsorted(cum, u[2 * r], side="right")), len(shapes) - 1)]
        lst = proven[s]
        out.append(lst[min(int(u[2 * r + 1] * len(lst)), len(lst) - 1)])
    return out


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    u = gen.uniform01(seed, count)
    gaps = -np.log1p(-u) / rate
    return np.cumsum(gaps)


def run(cands, reqs, arrivals, pool_cap: int, budget: int, mem_budget: int, max_active: int,
        tick_children: int = 0, stream=None) -> dict:
    """Serves reqs (candidate indices) arriving at `arrivals` (s from start;
    None = all at once).  Returns latencies, results and loop statistics."""
    n = len(reqs)
    lat = np.zeros(n)
    results = [None] * n
    ids = {}
    ticks = 0
    active_sum = 0
    with fspbb.server_create(mem_budget, max_active, tick_children, stream) as srv:
        t0 = time.perf_counter()
        arr = np.zeros(n) if arrivals is None else np.asarray(arrivals)
        nxt = 0
        done = 0
        nodes0 = 0
        while done < n:
            now = time.perf_counter() - t0
            while nxt < n and arr[nxt] <= now:
                c = cands[reqs[nxt]]
                ids[srv.submit(c.inst, fspbb.UB_NEH, pool_cap, c.budget or budget)] = nxt
                nxt += 1
            if len(ids) == done and nxt < n:
                # idle until the next arrival
                wait = arr[nxt] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
                continue
            fin, st = srv.step()
            tnow = time.perf_counter() - t0
            ticks += 1
            active_sum += st["last_searches"]
            for i in fin:
                r = ids[i]
                results[r] = srv.poll(i)
                lat[r] = tnow - arr[r]
                done += 1
            nodes0 = st["nodes_bounded"]
        wall = time.perf_counter() - t0
    mism = 0
    for k, r in enumerate(reqs):
        a, b = cands[r].alone, results[k]
        if any(a[f] != b[f] for f in RESULT_FIELDS) or not (a["perm"] == b["perm"]).all():
            mism += 1
    return {"latency_s": lat, "results": results, "wall_s": wall, "nodes_bounded": nodes0, "ticks": ticks,
            "mean_searches_per_tick": active_sum / max(ticks, 1), "mismatches": mism}


def percentile(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else math.nan
