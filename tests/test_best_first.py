"""Best-first search on the device (fsp_solve_ex with FSP_SOLVE_BEST_FIRST)
against the oracle's best-first search: every counter, the step log (parents,
children, upper bound, survivors, frontier size, fingerprint) and the
incumbent."""
import numpy as np
import pytest

import oracle
from helpers import require_gpu
from paper_1208_3933_amd import fspbb, gen

pytestmark = pytest.mark.gpu


def times(n, m, seed, lo=1, hi=99):
    return gen.processing_times(n, m, gen.make_seed(15, seed, gen.PURPOSE_TIMES), lo, hi)


def compare(p, ub_mode, cap, budget=1 << 62, heads=False):
    if ub_mode == "neh":
        ms, perm = oracle.neh(p)
        want = oracle.bnb(p, ms, perm, pool_cap=cap, node_budget=budget, steplog_cap=1 << 20, heads=heads,
                          best_first=True)
        ub0 = fspbb.UB_NEH
    else:
        want = oracle.bnb(p, fspbb.UB_NONE, None, pool_cap=cap, node_budget=budget, steplog_cap=1 << 20,
                          heads=heads, best_first=True)
        ub0 = fspbb.UB_NONE
    with fspbb.create_instance(p, heads=heads) as inst:
        got = fspbb.solve(inst, ub0, cap, budget, 1 << 20, best_first=True)
    assert got["opt"] == want["ub"]
    assert bool(got["proven"]) == want["proven"]
    assert got["nodes_bounded"] == want["nodes_bounded"]
    assert got["steps"] == want["steps"]
    assert got["improvements"] == want["improvements"]
    assert got["max_stack"] == want["max_stack"]
    assert (got["perm"] == want["incumbent"]).all()
    assert (got["steplog"] == want["steplog"]).all()
    return got


@pytest.mark.parametrize("n,m,seed", [(6, 3, 1), (8, 4, 2), (9, 5, 3), (10, 3, 4)])
@pytest.mark.parametrize("cap", [1, 3, 16, 1 << 20])
@pytest.mark.parametrize("ub_mode", ["neh", "none"])
def test_best_first_small_matches_oracle(n, m, seed, cap, ub_mode):
    require_gpu()
    p = times(n, m, seed)
    if ub_mode == "none" and n == 10 and cap <= 3:
        # the full search takes tens of thousands of one- to three-parent
        # steps: stopped by a node budget, the first 6,000 nodes still match
        got = compare(p, ub_mode, cap, budget=6000)
        assert got["status"] == fspbb.BUDGET and not got["proven"]
        return
    got = compare(p, ub_mode, cap)
    assert got["proven"]
    if n <= 8:
        assert got["opt"] == oracle.brute(p)


@pytest.mark.parametrize("n,m,seed,cap,budget", [(12, 5, 11, 64, 1 << 62), (15, 8, 12, 512, 40000),
                                                 (20, 5, 13, 256, 60000), (20, 10, 14, 4096, 60000)])
def test_best_first_medium_matches_oracle(n, m, seed, cap, budget):
    require_gpu()
    compare(times(n, m, seed), "neh", cap, budget)


def test_best_first_heads_and_large_values():
    require_gpu()
    compare(times(10, 6, 21), "neh", 32, heads=True)
    compare(times(9, 4, 22, 1, 100000), "neh", 40)  # the 32-bit kernel


def test_best_first_grows_its_slab():
    """A frontier far beyond the initial 4096 slots, against the oracle."""
    require_gpu()
    got = compare(times(14, 6, 31), "none", 50, budget=150000)
    assert got["max_stack"] > 4096


def test_best_first_finds_what_depth_first_finds():
    require_gpu()
    p = times(11, 5, 41)
    with fspbb.create_instance(p) as inst:
        a = fspbb.solve(inst, fspbb.UB_NEH, 128)
        b = fspbb.solve(inst, fspbb.UB_NEH, 128, best_first=True)
    assert a["proven"] and b["proven"] and a["opt"] == b["opt"]
