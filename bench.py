"""Benchmark: nodes bounded per second on one MI355X, plain and batched, and
the latency of served branch-and-bound solves.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Headline workload (the 200 jobs x 20 machines plain-bounding configuration):
one seeded instance with processing times i.i.d. U[1,99], a pool of 262,144
nodes whose depths are uniform on 0..199 and whose prefixes are seeded random
job sequences; inputs are resident in HBM before timing starts.  A step is one
fsp_bound_pool call over the whole pool (decode + scan kernels).  Prints one
JSON line.  Further legs:
  batched  the same pool as 64 pools of 4,096 in one graph-captured batch vs
           64 plain launches, and 64 seeded instances of mixed shape with
           log-normal pool sizes, batched vs plain;
  peaks    probe kernels for the packed 16-bit and 32-bit VALU, LDS reads and
           an HBM copy: what the chip delivers at its running clock, beside
           the published peaks (the scan's roofline also gives its fraction
           of the 16-bit probe's rate);
  variants the three mappings of the bound (lane per two nodes, lane per
           node, wave per node) on the 50 x 10 and 200 x 20 pools; the heads
           bound variant (earliest-start releases) and best-first selection:
           heads throughput on the same pool, and solves of small instances
           depth first, depth first with heads, and best first;
  bnb      branch-and-bound from NEH on the 200 x 20 instance, depth first and
           best first; the hybrid scheme (host explorer threads, shared GPU
           bounding over PCIe) against the device-resident search;
  serving  a Poisson stream of solves over mixed shapes through the serving
           loop: p50/p99 latency, nodes/s, and identity with each solve alone;
  tables   nodes/s over the shape x pool grid of the paper's Tables II/III,
           device-resident and with the pool's transfers in the timed region;
  cpu_baseline  the plain C oracle on a bounded prefix of the pool on the
           host cores (its bounds are also compared with the GPU's), on
           one core per table shape (the ratio the paper's tables report),
           and the share of a short sequential oracle search spent bounding.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "nodes bounded/s at 200x20 (batched vs plain) + p50/p99 solve latency"
N_JOBS, N_MACH, POOL = 200, 20, 262144
CONFIG = 2
# Peak of the unit the scan kernel is bound by: packed 16-bit integer VALU ops,
# 256 CUs x 4 SIMDs x 16 lanes x 2 halves x 2.4 GHz.
PEAK_U16_OPS = 256 * 4 * 16 * 2 * 2.4e9
# Published or unit-count peaks the probes are set against: 32-bit VALU (one
# op per lane per clock), LDS reads at 256 bytes per clock per CU (the LDS
# probe reaches 1.9x the 128 bytes per clock of the previous generation, so
# the read path is twice as wide), HBM3E 8 TB/s.
PEAK_I32_OPS = 256 * 4 * 16 * 2.4e9
PEAK_LDS_BYTES = 256 * 256 * 2.4e9
PEAK_HBM_BYTES = 8.0e12


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "scan16_200x20_pool262144_hbm_traffic.md")


def measured_traffic():
    """HBM bytes per scan launch from the committed counter passes, or None
    when the kernel sources have changed since they were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.startswith(("traffic_bytes_per_launch: ", "source_sha256: ")))
    files = [line for line in text.splitlines() if line.startswith("(SHA-256 of the concatenated files ")]
    if len(fields) != 2 or not files:
        return None
    names = files[0].split("files ", 1)[1].split(";")[0].split(", ")
    h = hashlib.sha256()
    for name in names:
        h.update(open(os.path.join(ROOT, "paper_1208_3933_amd", "csrc", name.strip()), "rb").read())
    if h.hexdigest() != fields["source_sha256"].strip():
        return None
    return int(fields["traffic_bytes_per_launch"])


def algorithmic_scan_ops(n: int, m: int, depths: np.ndarray) -> float:
    """Integer ops of the pair scans of one pool, counted as in Table I / Fig. 2:
    per node and pair, n membership tests, 4 ops per unscheduled job (two
    adds, a max and an add) and 2 for the tail and the max over pairs."""
    P = m * (m - 1) // 2
    nprime = (n - depths.astype(np.int64)).sum()
    return float(P * (n * len(depths) + 4 * nprime + 2 * len(depths)))


def host_cores() -> dict:
    """Host CPUs this process may use: the count the OS reports, the CPUs of
    its affinity mask, and the cgroup CPU quota (a container's share), with
    the least of them as the cores to run on."""
    visible = os.cpu_count() or 1
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = visible
    quota = None
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = float(q) / float(per)
    except (OSError, ValueError):
        try:
            q = int(open("/sys/fs/cgroup/cpu/cpu.cfs_quota_us").read())
            per = int(open("/sys/fs/cgroup/cpu/cpu.cfs_period_us").read())
            if q > 0:
                quota = q / per
        except (OSError, ValueError):
            pass
    usable = min(visible, affinity, int(quota) if quota else visible)
    return {"os_cpu_count": visible, "affinity": affinity, "cgroup_quota": quota, "usable": max(1, usable)}


def cpu_baseline(p, pre, dep, sample: int, threads: int, gpu_lb: np.ndarray) -> dict:
    import concurrent.futures as cf

    import oracle
    idx = np.arange(min(sample, len(dep)))
    chunks = np.array_split(idx, threads * 4)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda c: oracle.bound_pool(p, pre[c], dep[c]), chunks))
    dt = time.perf_counter() - t0
    want = np.concatenate(parts)
    return {"value": len(idx) / dt, "unit": "nodes/s", "cores": threads, "kind": "oracle",
            "sample": f"first {len(idx)} nodes of the same 200x20 pool, plain C oracle, one thread per usable "
                      f"host core",
            "gpu_bounds_equal": bool((gpu_lb[idx] == want).all())}


def bound_share(p) -> dict:
    """Share of the oracle's sequential depth-first search spent bounding, the
    figure the paper gives for its CPU B&B (Sec. I): 200x20 from the NEH bound,
    steps of up to 4,096 children, stopped after 4,096 nodes, one thread."""
    import oracle
    ms, perm = oracle.neh(p)
    r = oracle.bnb(p, ms, perm, pool_cap=4096, node_budget=4096)
    return {"share": r["seconds_bound"] / r["seconds_total"], "seconds": r["seconds_total"],
            "nodes": r["nodes_bounded"], "steps": r["steps"],
            "search": "200x20 DFS from NEH, pool_cap 4096, node budget 4096, one thread"}


def peaks_leg(stream) -> dict:
    """What the chip delivers at its running clock: each probe kernel's rate
    (best of three) and its fraction of the published or unit-count peak."""
    from paper_1208_3933_amd import fspbb
    out = {}
    for name, kind, peak, unit, scale in [("valu_u16", fspbb.PROBE_VALU16, PEAK_U16_OPS, "TOP/s", 1e12),
                                          ("valu_i32", fspbb.PROBE_VALU32, PEAK_I32_OPS, "TOP/s", 1e12),
                                          ("lds_read", fspbb.PROBE_LDS, PEAK_LDS_BYTES, "TB/s", 1e12),
                                          ("hbm_copy", fspbb.PROBE_HBM, PEAK_HBM_BYTES, "TB/s", 1e12)]:
        rate = max(fspbb.probe_peak(kind, 1 << 30, stream)[0] for _ in range(3))
        out[name] = {"achieved": rate / scale, "peak": peak / scale, "unit": unit, "frac": rate / peak}
    return out


def _time(fn, reps: int) -> float:
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def _time_best(fn, reps: int, rounds: int = 3) -> float:
    """Per-call time of the fastest of `rounds` back-to-back timings of `reps`
    calls (a host hiccup inside one round does not set the figure)."""
    return min(_time(fn, reps) for _ in range(rounds))


def batched_leg(inst, pre_d, dep_d, reps: int, stream) -> dict:
    """Batched (one graph-captured persistent launch) vs plain (one launch per
    pool) on the same pools, outputs compared element by element."""
    import torch

    from paper_1208_3933_amd import fspbb, gen
    out = {}

    def compare(name, pools):
        plain_out = [torch.full_like(o, -7) for _, _, _, o in pools]

        def plain():
            for (i, a, b, _), o in zip(pools, plain_out):
                fspbb.bound_pool(i, a, b, o, stream)
        with fspbb.batch_create(pools, graph=True) as b:
            for _ in range(3):
                plain()
                b.run(stream)
            t_plain = _time(plain, reps)
            t_batch = _time(lambda: b.run(stream), reps)
            info = b.info()
        same = all(bool(torch.equal(o, q)) for (_, _, _, o), q in zip(pools, plain_out))
        nodes = info["total_nodes"]
        out[name] = {"pools": len(pools), "nodes": nodes, "plain_ms": t_plain * 1e3, "batched_ms": t_batch * 1e3,
                     "plain_nodes_per_s": nodes / t_plain, "batched_nodes_per_s": nodes / t_batch,
                     "speedup": t_plain / t_batch, "identical": same, "work_items": info["items"],
                     "scan_workgroups": info["grid"]}

    # the 200 x 20 pool as 64 pools of 4096 nodes
    N = int(dep_d.shape[0])
    k = 64
    step = N // k
    pools = [(inst, pre_d[i * step:(i + 1) * step], dep_d[i * step:(i + 1) * step],
              torch.empty(step, dtype=torch.int32, device=dep_d.device)) for i in range(k)]
    compare("200x20_64x4096", pools)
    # the whole pool as one batch entry
    compare("200x20_whole_pool", [(inst, pre_d, dep_d, torch.empty(N, dtype=torch.int32, device=dep_d.device))])
    # 64 seeded instances of mixed shape with log-normal pool sizes
    shapes = [(20, 5), (20, 10), (20, 20), (50, 10), (100, 20), (200, 20)]
    sizes = gen.lognormal_pool_sizes(64, gen.make_seed(3, 0, gen.PURPOSE_SIZES))
    insts, pools = [], []
    for i in range(64):
        n, m = shapes[i % 6]
        ins = fspbb.create_instance(gen.processing_times(n, m, gen.make_seed(3, i, gen.PURPOSE_TIMES)))
        pr, dp = gen.random_pool(n, int(sizes[i]), gen.make_seed(3, i, gen.PURPOSE_POOL))
        insts.append(ins)
        pools.append((ins, torch.from_numpy(pr).cuda(), torch.from_numpy(dp).cuda(),
                      torch.empty(int(sizes[i]), dtype=torch.int32, device="cuda")))
    compare("mixed_64_instances", pools)
    for ins in insts:
        ins.close()
    # the tuner's timing of both scan launch forms (one workgroup per work item,
    # persistent) for each shape of the mixed batch, on its seeded sample pool;
    # the tuning table is put back afterwards so that later legs run as before
    forms = {}
    for n, m in shapes:
        w0, _ = fspbb.tune_get(n, m)
        f0 = fspbb.tune_get_form(n, m)
        with fspbb.create_instance(gen.processing_times(n, m, gen.make_seed(3, 100 + n, gen.PURPOSE_TIMES))) as ins:
            t = fspbb.autotune(ins, 16384, 3)
        fspbb.tune_set(n, m, w0)
        fspbb.tune_set_form(n, m, f0)
        forms["%dx%d" % (n, m)] = {"waves_per_group": t["waves_per_group"], "grid_us": t["grid_us"],
                                   "persistent_us": t["persistent_us"],
                                   "persistent_vs_grid": t["grid_us"] / t["persistent_us"]}
    out["tuner_forms_16384_nodes"] = forms
    return out


def adjacent_pairs(m: int) -> list:
    """Machine pairs (k, k+1) and (0, m-1): m pairs (m - 1 when m = 2) of the
    m(m-1)/2, including one that ends on the last machine."""
    return sorted({(k, k + 1) for k in range(m - 1)} | {(0, m - 1)})


def variants_leg(p, pre_d, dep_d, steps: int, stream, solve_seeds: int = 6) -> dict:
    """The next rows of the path: the bound variants (heads: releases as the
    earliest starts of unscheduled jobs; a subset of the machine pairs: the
    adjacent ones and (0, m-1)) and best-first selection.  Bound throughput
    of each variant on the same 200x20 pool, and solves from NEH of seeded
    small instances with each strategy (same pool_cap and budget)."""
    import torch

    from paper_1208_3933_amd import fspbb, serve
    out = {}
    m20 = int(p.shape[1])
    for key, kw in (("heads_bound_200x20_nodes_per_s", {"heads": True}),
                    ("adjacent_pairs_bound_200x20_nodes_per_s", {"pairs": adjacent_pairs(m20)})):
        with fspbb.create_instance(p, **kw) as inst:
            o = dep_d.new_empty(dep_d.shape)
            for _ in range(2):
                fspbb.bound_pool(inst, pre_d, dep_d, o, stream)
            t = _time(lambda: fspbb.bound_pool(inst, pre_d, dep_d, o, stream), steps)
            out[key] = int(dep_d.shape[0]) / t
    # the three mappings of the bound on the 50 x 10 and 200 x 20 pools
    from paper_1208_3933_amd import gen
    mappings = {}
    for (n, m, N, cfg) in [(50, 10, 65536, 1), (200, 20, 262144, 2)]:
        if n == 200:
            pp, a, b = p, pre_d, dep_d
        else:
            pp = gen.processing_times(n, m, gen.make_seed(cfg, 0, gen.PURPOSE_TIMES))
            hp, hd = gen.random_pool(n, N, gen.make_seed(cfg, 0, gen.PURPOSE_POOL))
            a, b = torch.from_numpy(hp).cuda(), torch.from_numpy(hd).cuda()
        row = {}
        with fspbb.create_instance(pp) as inst:
            o = b.new_empty(b.shape)
            for name, v in (("lane_per_two_nodes_u16", fspbb.VARIANT_PACKED16),
                            ("lane_per_node_i32_lds_masks", fspbb.VARIANT_WIDE),
                            ("lane_per_node_i32", fspbb.VARIANT_LANE32), ("wave_per_node_i32", fspbb.VARIANT_WAVEPAIR)):
                fspbb.bound_pool(inst, a, b, o, stream, variant=v)
                t = _time(lambda: fspbb.bound_pool(inst, a, b, o, stream, variant=v), max(2, steps // 4))
                row[name] = N / t
        mappings["%dx%d_pool%d" % (n, m, N)] = row
    out["mappings_nodes_per_s"] = mappings
    # an instance past the 16-bit guard: 200 x 20 with times U[1,300] takes the
    # 32-bit kernels; every bound of the default one equals the other's
    pw = gen.processing_times(200, 20, gen.make_seed(18, 200, gen.PURPOSE_TIMES), 1, 300)
    wrow = {}
    with fspbb.create_instance(pw) as inst:
        assert not inst.info()["packed16"]
        o1, o2 = dep_d.new_empty(dep_d.shape), dep_d.new_empty(dep_d.shape)
        for name, v, o in (("default_lane_per_node_i32_lds_masks", fspbb.VARIANT_AUTO, o1),
                           ("lane_per_node_i32", fspbb.VARIANT_LANE32, o2)):
            fspbb.bound_pool(inst, pre_d, dep_d, o, stream, variant=v)
            t = _time(lambda: fspbb.bound_pool(inst, pre_d, dep_d, o, stream, variant=v), max(2, steps // 4))
            wrow[name] = int(dep_d.shape[0]) / t
        torch.cuda.synchronize()
        wrow["same_bounds"] = bool((o1 == o2).all().item())
    out["wide_values_200x20_pool262144_nodes_per_s"] = wrow

    if solve_seeds <= 0:
        return out
    shapes = [(20, 5), (20, 10), (50, 5), (100, 5)]
    cands = serve.candidates(solve_seeds, shapes)
    budget, cap = 2_000_000, 8192
    modes = {"dfs": (False, False, False, False), "dfs_device_steps": (False, False, False, True),
             "dfs_heads": (True, False, False, False), "best_first": (False, True, False, False),
             "dfs_adjacent_pairs": (False, False, True, False)}
    rows = {}
    for c in cands:
        key = "%dx%d" % shapes[c.shape]
        r = rows.setdefault(key, {"instances": 0})
        r["instances"] += 1
        for mode, (heads, bfirst, sub, dev) in modes.items():
            pairs = adjacent_pairs(int(c.p.shape[1])) if sub else None
            with fspbb.create_instance(c.p, heads=heads, pairs=pairs) as inst:
                t0 = time.perf_counter()
                res = fspbb.solve(inst, fspbb.UB_NEH, cap, budget, 0, stream, best_first=bfirst, device_steps=dev)
                dt = time.perf_counter() - t0
            r[mode + "_proven"] = r.get(mode + "_proven", 0) + int(res["proven"])
            r[mode + "_nodes"] = r.get(mode + "_nodes", 0) + int(res["nodes_bounded"])
            r[mode + "_s"] = r.get(mode + "_s", 0.0) + dt
    out["solves"] = rows
    out["pool_cap"], out["node_budget"] = cap, budget
    return out


def hybrid_leg(inst, p200, stream, threads: int) -> dict:
    """The paper's host-driven scheme with several host explorers (fsp_explore:
    host stacks and branching, shared GPU bounding with PCIe copies of every
    pool) against the device-resident depth-first search: time to the proof on
    a seeded 20x5 instance, and nodes/s on the 200x20 instance with a budget."""
    from paper_1208_3933_amd import fspbb, gen
    out = {"threads": threads}
    p = gen.processing_times(20, 5, gen.make_seed(4, 2, gen.PURPOSE_TIMES))  # proven within ~1.5 M nodes
    with fspbb.create_instance(p) as i20:
        fspbb.solve(i20, fspbb.UB_NEH, 8192, 10000, 0, stream)
        t0 = time.perf_counter()
        d = fspbb.solve(i20, fspbb.UB_NEH, 8192, 1 << 40, 0, stream)
        td = time.perf_counter() - t0
        fspbb.explore(i20, fspbb.UB_NEH, threads, 8192, 10000, stream)  # warm-up
        h = fspbb.explore(i20, fspbb.UB_NEH, threads, 8192, 1 << 40, stream)
    out["20x5_proof"] = {"device_dfs_s": td, "device_dfs_nodes": d["nodes_bounded"], "hybrid_s": h["seconds"],
                         "hybrid_nodes": h["nodes_bounded"], "hybrid_launches": h["pools"],
                         "same_optimum": bool(d["proven"] and h["proven"] and d["opt"] == h["opt"])}
    budget = 16 * POOL
    fspbb.explore(inst, fspbb.UB_NEH, threads, POOL // threads, POOL, stream)  # warm-up
    h = fspbb.explore(inst, fspbb.UB_NEH, threads, POOL // threads, budget, stream)
    out["200x20_budget"] = {"hybrid_nodes_per_s": h["nodes_bounded"] / h["seconds"], "nodes": h["nodes_bounded"],
                            "launches": h["pools"], "pool_cap_per_explorer": POOL // threads}
    return out


TABLE_SHAPES = [(200, 20), (100, 20), (50, 20), (20, 20)]
TABLE_POOLS = [4096 << k for k in range(7)]


def tables_leg(stream, reps: int) -> dict:
    """The grid of the paper's Tables II/III (shapes 20..200 x 20, pools 4096 ..
    262144 nodes): nodes/s with the pool resident on the device, and with the
    pool copied from pinned host memory and the bounds copied back in the timed
    region (the paper's timing includes those transfers)."""
    import torch

    from paper_1208_3933_amd import fspbb, gen
    out = {}
    for n, m in TABLE_SHAPES:
        p = gen.processing_times(n, m, gen.make_seed(6, n, gen.PURPOSE_TIMES))
        pre, dep = gen.random_pool(n, TABLE_POOLS[-1], gen.make_seed(6, n, gen.PURPOSE_POOL))
        h_pre = torch.from_numpy(pre).pin_memory()
        h_dep = torch.from_numpy(dep).pin_memory()
        h_out = torch.empty(TABLE_POOLS[-1], dtype=torch.int32).pin_memory()
        d_pre, d_dep = h_pre.cuda(), h_dep.cuda()
        d_out = torch.empty(TABLE_POOLS[-1], dtype=torch.int32, device="cuda")
        row = {}
        with fspbb.create_instance(p) as inst:
            for N in TABLE_POOLS:
                a, b, o = d_pre[:N], d_dep[:N], d_out[:N]

                def device_only():
                    fspbb.bound_pool(inst, a, b, o, stream)

                def with_transfers():
                    a.copy_(h_pre[:N], non_blocking=True)
                    b.copy_(h_dep[:N], non_blocking=True)
                    fspbb.bound_pool(inst, a, b, o, stream)
                    h_out[:N].copy_(o, non_blocking=True)

                for fn in (device_only, with_transfers, device_only, with_transfers):
                    fn()
                # more calls per timing for smaller pools, so that the final
                # synchronisation is a small share of each timing
                r = reps * max(1, TABLE_POOLS[4] // N)
                t_dev = _time_best(device_only, r)
                t_xfer = _time_best(with_transfers, r)
                row[str(N)] = {"device_nodes_per_s": N / t_dev, "with_transfers_nodes_per_s": N / t_xfer}
        out["%dx%d" % (n, m)] = row
    return out


def single_core_rates() -> dict:
    """The plain oracle on one host thread per shape of the table grid, on a
    sample of about half a second each (the paper's reference is one CPU
    core)."""
    import oracle
    from paper_1208_3933_amd import gen
    sample = {200: 256, 100: 512, 50: 1024, 20: 4096}
    out = {}
    for n, m in TABLE_SHAPES:
        p = gen.processing_times(n, m, gen.make_seed(6, n, gen.PURPOSE_TIMES))
        pre, dep = gen.random_pool(n, sample[n], gen.make_seed(6, n, gen.PURPOSE_POOL))
        t0 = time.perf_counter()
        oracle.bound_pool(p, pre, dep)
        out["%dx%d" % (n, m)] = sample[n] / (time.perf_counter() - t0)
    return out


def serving_leg(n_requests: int, seeds_per_shape: int, pool_cap: int, budget: int, large_budget: int,
                stream) -> dict:
    """Poisson stream of solves at 0.7 x the measured saturation rate.  The
    200x20 and 500x20 requests are searches stopped after large_budget nodes;
    the latency of proven solves and of those is reported apart."""
    from paper_1208_3933_amd import gen, serve
    cands = serve.candidates(seeds_per_shape, budgeted_budget=large_budget)
    serve.screen(cands[:4], pool_cap, budget, stream)  # warm-up
    serve.screen(cands, pool_cap, budget, stream)
    unsolved = {}
    for c in cands:
        if not c.alone["proven"] and not c.budgeted:
            key = "%dx%d" % serve.SHAPES[c.shape]
            unsolved[key] = unsolved.get(key, 0) + 1
    mem = 32 << 30
    sat_reqs = serve.sample_requests(cands, max(50, n_requests // 8), gen.make_seed(serve.CONFIG, 1, gen.PURPOSE_ARRIVALS))
    sat = serve.run(cands, sat_reqs, None, pool_cap, budget, mem, 256, 0, stream)
    sat_rate = len(sat_reqs) / sat["wall_s"]
    alone_s = sum(cands[r].alone_s for r in sat_reqs)
    reqs = serve.sample_requests(cands, n_requests, gen.make_seed(serve.CONFIG, 2, gen.PURPOSE_ARRIVALS))
    rate = 0.7 * sat_rate
    arr = serve.poisson_arrivals(n_requests, rate, gen.make_seed(serve.CONFIG, 3, gen.PURPOSE_ARRIVALS))
    r = serve.run(cands, reqs, arr, pool_cap, budget, mem, 256, 0, stream)
    lat_all = r["latency_s"] * 1e3
    proven = np.array([not cands[k].budgeted for k in reqs], bool)
    lat_ms = lat_all[proven]
    stopped = {}
    for key in sorted({"%dx%d" % serve.SHAPES[cands[k].shape] for k in reqs if cands[k].budgeted}):
        sel = np.array(["%dx%d" % serve.SHAPES[cands[k].shape] == key and cands[k].budgeted for k in reqs], bool)
        x = lat_all[sel]
        stopped[key] = {"requests": int(sel.sum()), "node_budget": large_budget,
                        "p50_ms": serve.percentile(x, 50), "p99_ms": serve.percentile(x, 99),
                        "mean_ms": float(x.mean())}
    for c in cands:
        c.inst.close()
    return {"requests": n_requests, "rate_per_s": rate, "proven_requests": int(proven.sum()),
            "p50_ms": serve.percentile(lat_ms, 50),
            "p99_ms": serve.percentile(lat_ms, 99), "mean_ms": float(lat_ms.mean()),
            "budget_stopped_by_shape": stopped,
            "nodes_per_s": r["nodes_bounded"] / r["wall_s"], "solves_per_s": n_requests / r["wall_s"],
            "wall_s": r["wall_s"], "mean_searches_per_step": r["mean_searches_per_tick"],
            "mismatches_vs_alone": r["mismatches"] + sat["mismatches"],
            "saturation": {"requests": len(sat_reqs), "solves_per_s": sat_rate,
                           "nodes_per_s": sat["nodes_bounded"] / sat["wall_s"],
                           "alone_sequential_solves_per_s": len(sat_reqs) / alone_s,
                           "speedup_vs_alone_sequential": alone_s / sat["wall_s"]},
            "pool_cap": pool_cap, "node_budget": budget,
            "screened": len(cands), "proven": sum(1 for c in cands if c.alone["proven"]),
            "unsolved_by_shape": unsolved}


def bnb_leg(inst, steps: int, stream, best_first: bool = False, device_steps: bool = False) -> dict:
    """Branch-and-bound from the NEH upper bound on the same instance, pool
    steps of 262,144 children (the paper's largest pool), search state resident
    on the device: depth first (stack) or best first (frontier by bound).  The
    host NEH heuristic runs once before the timed search (its time is reported
    as neh_ms); the search from that bound is the one fsp_solve runs from
    FSP_UB_NEH, node for node."""
    import torch

    from paper_1208_3933_amd import fspbb
    t0 = time.perf_counter()
    ub0, _ = fspbb.neh(inst)
    neh_ms = (time.perf_counter() - t0) * 1e3
    kw = {"best_first": best_first, "device_steps": device_steps}
    fspbb.solve(inst, ub0, POOL, 1 + steps * POOL, 0, stream, **kw)  # warm-up: the same search
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fspbb.solve(inst, ub0, POOL, 1 + steps * POOL, 0, stream, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"nodes_per_s": r["nodes_bounded"] / dt, "nodes_bounded": r["nodes_bounded"], "steps": r["steps"],
            "ms_per_step": dt * 1e3 / max(r["steps"], 1), "ub": r["opt"], "ub0_neh": ub0, "neh_ms": neh_ms,
            "pool_cap": POOL, "proven": bool(r["proven"]),
            ("max_frontier" if best_first else "max_stack"): r["max_stack"]}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20, help="untimed pools first (the clocks take some tens to settle)")
    ap.add_argument("--cpu-sample", type=int, default=16384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--bnb-steps", type=int, default=8, help="pool steps of the 200x20 DFS leg (0 = skip)")
    ap.add_argument("--batched-reps", type=int, default=20, help="repetitions of the batched leg (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests of the serving leg (0 = skip)")
    ap.add_argument("--serve-seeds", type=int, default=10, help="screened instances per shape")
    ap.add_argument("--serve-pool-cap", type=int, default=8192)
    ap.add_argument("--serve-budget", type=int, default=2000000)
    ap.add_argument("--serve-large-budget", type=int, default=131072,
                    help="node budget of the served 200x20 and 500x20 searches (0 = serve proven instances only)")
    ap.add_argument("--tables-reps", type=int, default=10,
                    help="repetitions per point of the shape x pool grid of the paper's tables (0 = skip)")
    ap.add_argument("--variant-solves", type=int, default=6,
                    help="seeded instances per shape solved with each strategy in the variants leg (0 = skip)")
    ap.add_argument("--no-variants", "--no-heads", dest="heads", action="store_false",
                    help="skip the leg of the bound and selection variants")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="run one plain device copy of this many bytes before timing (a kernel of known "
                         "traffic, to scale HBM counters read under a profiler)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the bound path runs on "
              "one device; a pool would shard across GPUs by node ranges with no exchange, a search by sharing its incumbent)", file=sys.stderr)
        return 2

    import torch

    from paper_1208_3933_amd import fspbb, gen
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    fspbb.lib()

    p = gen.processing_times(N_JOBS, N_MACH, gen.make_seed(CONFIG, 0, gen.PURPOSE_TIMES))
    pre, dep = gen.random_pool(N_JOBS, POOL, gen.make_seed(CONFIG, 0, gen.PURPOSE_POOL))
    print(f"[bench] workload ready: {N_JOBS}x{N_MACH}, pool {POOL}", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    pre_d = torch.from_numpy(pre).to(dev)
    dep_d = torch.from_numpy(dep).to(dev)
    out = torch.empty(POOL, dtype=torch.int32, device=dev)
    inst = fspbb.create_instance(p)
    stream = torch.cuda.current_stream()

    if args.copy_bytes > 0:
        src = torch.ones(args.copy_bytes // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)  # one elementwise kernel: reads and writes copy_bytes each
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        fspbb.bound_pool(inst, pre_d, dep_d, out, stream)
    torch.cuda.synchronize()
    if fspbb.pool_status(inst, stream) != 0:
        raise RuntimeError("invalid nodes in the benchmark pool")

    gpu_lb = out.cpu().numpy()

    # chained event timing: two event records per step (after the decode,
    # after the scan), each step's decode measured from the previous scan's end
    fspbb.timing_enable(inst, True, chained=True)
    fspbb.timing_read(inst)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fspbb.bound_pool(inst, pre_d, dep_d, out, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dec_ms, scan_ms, launches = fspbb.timing_read(inst)
    fspbb.timing_enable(inst, False)
    print(f"[bench] timed {args.steps} steps", file=sys.stderr, flush=True)

    elapsed = t1 - t0
    value = POOL * args.steps / elapsed
    scan_avg_s = scan_ms / 1e3 / max(launches, 1)
    ops = algorithmic_scan_ops(N_JOBS, N_MACH, dep)
    achieved = ops / scan_avg_s / 1e12
    peak = PEAK_U16_OPS / 1e12
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "nodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": "plain bounding, 200 jobs x 20 machines (190 pairs), U[1,99] times, "
                               "pool of 262144 nodes, depths U{0..199}",
                   "n": N_JOBS, "m": N_MACH, "pool": POOL,
                   "kernel": "decode16 + scan16 (%d waves per 128-node group)" % fspbb.tune_get(N_JOBS, N_MACH)[0]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TOP/s",
                     "frac": achieved / peak, "traffic": measured_traffic(), "traffic_unit": "bytes/launch",
                     "kernel": "bound_scan16_kernel", "kernel_avg_ms": scan_avg_s * 1e3,
                     "decode_avg_ms": dec_ms / max(launches, 1)},
        "plain_nodes_per_s": value,
    }
    result["peaks"] = peaks_leg(stream)
    probe = result["peaks"]["valu_u16"]["achieved"]
    result["roofline"]["probe_peak"] = probe
    result["roofline"]["frac_of_probe_peak"] = achieved / probe
    if args.batched_reps > 0:
        result["batched"] = batched_leg(inst, pre_d, dep_d, args.batched_reps, stream)
        print("[bench] batched leg done", file=sys.stderr, flush=True)
    if args.heads:
        result["variants"] = variants_leg(p, pre_d, dep_d, args.steps, stream, args.variant_solves)
        print("[bench] variants leg done", file=sys.stderr, flush=True)
    if args.bnb_steps > 0:
        result["bnb"] = bnb_leg(inst, args.bnb_steps, stream)
        result["bnb_device_steps"] = bnb_leg(inst, args.bnb_steps, stream, device_steps=True)
        result["bnb_best_first"] = bnb_leg(inst, args.bnb_steps, stream, best_first=True)
        result["hybrid"] = hybrid_leg(inst, p, stream, max(1, min(16, os.cpu_count() or 1)))
        print("[bench] bnb leg done", file=sys.stderr, flush=True)
    if args.serve_requests > 0:
        result["serving"] = serving_leg(args.serve_requests, args.serve_seeds, args.serve_pool_cap,
                                        args.serve_budget, args.serve_large_budget, stream)
        s = result["serving"]
        result["p50_ms"], result["p99_ms"] = s["p50_ms"], s["p99_ms"]
        print("[bench] serving leg done", file=sys.stderr, flush=True)
    if args.tables_reps > 0:
        result["tables"] = tables_leg(stream, args.tables_reps)
        print("[bench] tables leg done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        cores = host_cores()
        result["cpu_baseline"] = cpu_baseline(p, pre, dep, args.cpu_sample, cores["usable"], gpu_lb)
        result["cpu_baseline"]["host"] = cores
        one = single_core_rates()
        result["cpu_baseline"]["single_core_nodes_per_s"] = one
        result["cpu_baseline"]["bound_share_of_search"] = bound_share(p)
        if "tables" in result:  # GPU (with transfers) over one oracle core, the form of the paper's tables
            result["tables_ratio_vs_one_core"] = {
                shape: {N: round(v["with_transfers_nodes_per_s"] / one[shape], 1) for N, v in row.items()}
                for shape, row in result["tables"].items()}
    inst.close()
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
