"""Depth-first searches whose steps are chosen and accounted for on the device
(FSP_SOLVE_DEVICE_STEPS: several steps per host synchronisation) against the
oracle's search and against the host-driven fsp_solve: every counter, the
incumbent and the whole step log (parents, children, UB, pushed, stack size,
fingerprint) must be equal."""
import numpy as np
import pytest

import oracle
from helpers import load_golden, require_gpu
from paper_1208_3933_amd import fspbb, gen

pytestmark = pytest.mark.gpu

FIELDS = ("opt", "proven", "nodes_bounded", "steps", "ub0", "improvements", "max_stack", "status")


def times(n, m, seed, lo=1, hi=99):
    return gen.processing_times(n, m, gen.make_seed(8, seed, gen.PURPOSE_TIMES), lo, hi)


def compare(p, ub_mode, pool_cap, budget=1 << 62, steplog_cap=1 << 16, heads=False):
    ub0 = fspbb.UB_NEH if ub_mode == "neh" else fspbb.UB_NONE
    with fspbb.create_instance(p, heads=heads) as inst:
        dev = fspbb.solve(inst, ub0, pool_cap, budget, steplog_cap, device_steps=True)
        host = fspbb.solve(inst, ub0, pool_cap, budget, steplog_cap)
    for f in FIELDS:
        assert dev[f] == host[f], (f, dev[f], host[f])
    assert (dev["perm"] == host["perm"]).all()
    assert dev["steplog"].shape == host["steplog"].shape and (dev["steplog"] == host["steplog"]).all()
    if not heads:
        if ub_mode == "neh":
            ms, perm = oracle.neh(p)
            want = oracle.bnb(p, ms, perm, pool_cap=pool_cap, node_budget=budget, steplog_cap=steplog_cap)
        else:
            want = oracle.bnb(p, fspbb.UB_NONE, None, pool_cap=pool_cap, node_budget=budget, steplog_cap=steplog_cap)
        assert (dev["opt"], bool(dev["proven"]), dev["nodes_bounded"], dev["steps"]) == \
            (want["ub"], want["proven"], want["nodes_bounded"], want["steps"])
        assert (dev["steplog"] == want["steplog"]).all()
        assert (dev["perm"] == want["incumbent"]).all()
    return dev


@pytest.mark.parametrize("n,m,seed", [(6, 3, 11), (8, 4, 12), (9, 5, 13), (10, 3, 14)])
@pytest.mark.parametrize("pool_cap", [1, 3, 16, 1 << 20])
@pytest.mark.parametrize("ub_mode", ["neh", "none"])
def test_device_steps_small(n, m, seed, pool_cap, ub_mode):
    require_gpu()
    got = compare(times(n, m, seed), ub_mode, pool_cap)
    assert got["proven"]


@pytest.mark.parametrize("n,m,seed,pool_cap,budget", [(20, 5, 21, 256, 200000), (15, 8, 22, 64, 50000),
                                                      (20, 10, 23, 4096, 60000), (50, 10, 24, 2048, 20000),
                                                      (30, 20, 25, 100, 30000), (12, 6, 26, 7, 1 << 40)])
def test_device_steps_medium(n, m, seed, pool_cap, budget):
    require_gpu()
    compare(times(n, m, seed), "neh", pool_cap, budget)


def test_device_steps_first_parent_over_pool_cap():
    """pool_cap below a parent's children: every step takes one parent."""
    require_gpu()
    compare(times(40, 5, 27), "none", 5, budget=5000)


def test_device_steps_200x20_benchmarked_pool_cap():
    """The benchmarked search (200 x 20 from NEH, pool_cap 262,144) for three
    steps: the step log equals the oracle-built fixture."""
    require_gpu()
    g = load_golden("bnb_200x20_neh_cap262144.json")
    p = gen.processing_times(g["n"], g["m"], gen.make_seed(*g["seed"]))
    steps = g["steps"]
    with fspbb.create_instance(p) as inst:
        got = fspbb.solve(inst, fspbb.UB_NEH, g["pool_cap"], steps[1]["nodes_after"] + 1, steplog_cap=8,
                          device_steps=True)
    assert got["ub0"] == g["neh"]
    assert got["steps"] == 3 and got["nodes_bounded"] == steps[2]["nodes_after"]
    for k in range(3):
        assert got["steplog"][k].tolist() == steps[k]["log"], k


def test_device_steps_root_pruned_and_tiny_budget():
    require_gpu()
    p = times(10, 5, 31)
    lb0 = oracle.bound(p, [])
    with fspbb.create_instance(p) as inst:
        r = fspbb.solve(inst, lb0, 16, 1 << 40, device_steps=True)
        assert r["proven"] and r["nodes_bounded"] == 1 and r["steps"] == 0 and (r["perm"] == -1).all()
        a = fspbb.solve(inst, fspbb.UB_NONE, 4, 30, 64, device_steps=True)
        b = fspbb.solve(inst, fspbb.UB_NONE, 4, 30, 64)
    assert a["status"] == b["status"] == fspbb.BUDGET
    assert (a["nodes_bounded"], a["steps"]) == (b["nodes_bounded"], b["steps"])
    assert (a["steplog"] == b["steplog"]).all()


def test_device_steps_fall_back_on_32bit_and_heads_instances():
    require_gpu()
    compare(times(9, 4, 32, 1, 100000), "neh", 16)         # the 32-bit path: host-driven steps
    compare(times(9, 4, 33), "neh", 16, heads=True)         # heads: host-driven steps


def test_device_steps_flag_errors():
    require_gpu()
    with fspbb.create_instance(times(6, 3, 34)) as inst:
        with pytest.raises(fspbb.FspError) as ei:
            fspbb.solve(inst, fspbb.UB_NEH, 16, 1 << 20, best_first=True, device_steps=True)
        assert ei.value.status == fspbb.E_INVAL
