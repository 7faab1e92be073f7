"""Hybrid search (fsp_explore): host explorer threads with shared GPU bounding.
Node counts depend on thread timing, so the checks are on what is unique --
the optimum and the proof -- and on the validity of the schedule returned."""
import numpy as np
import pytest

import oracle
from helpers import require_gpu
from paper_1208_3933_amd import fspbb, gen

pytestmark = pytest.mark.gpu


def times(n, m, seed, lo=1, hi=99):
    return gen.processing_times(n, m, gen.make_seed(16, seed, gen.PURPOSE_TIMES), lo, hi)


@pytest.mark.parametrize("n,m,seed", [(6, 3, 1), (8, 4, 2), (9, 5, 3)])
@pytest.mark.parametrize("threads,cap", [(1, 16), (4, 3), (8, 64)])
def test_explore_small_finds_the_optimum(n, m, seed, threads, cap):
    require_gpu()
    p = times(n, m, seed)
    opt = oracle.brute(p)
    with fspbb.create_instance(p) as inst:
        for ub0 in (fspbb.UB_NEH, fspbb.UB_NONE):
            r = fspbb.explore(inst, ub0, threads, cap)
            assert r["proven"] and r["opt"] == opt
            assert sorted(r["perm"].tolist()) == list(range(n))
            assert oracle.makespan(p, r["perm"]) == opt
            assert r["nodes_bounded"] >= 1 and r["pools"] >= 1


@pytest.mark.parametrize("n,m,seed,cap", [(12, 5, 11, 256), (11, 6, 12, 64)])
def test_explore_matches_device_search(n, m, seed, cap):
    """Same optimum as the oracle's and the device's depth-first searches."""
    require_gpu()
    p = times(n, m, seed)
    ms, perm = oracle.neh(p)
    want = oracle.bnb(p, ms, perm, pool_cap=cap)
    assert want["proven"]
    with fspbb.create_instance(p) as inst:
        d = fspbb.solve(inst, fspbb.UB_NEH, cap)
        for threads in (1, 8):
            r = fspbb.explore(inst, fspbb.UB_NEH, threads, cap)
            assert r["proven"] and r["opt"] == want["ub"] == d["opt"]
            assert oracle.makespan(p, r["perm"]) == r["opt"]


def test_explore_heads_and_budget():
    require_gpu()
    p = times(10, 6, 21)
    opt = oracle.bnb(p, 1 << 30, None, pool_cap=64)["ub"]
    with fspbb.create_instance(p, heads=True) as inst:
        r = fspbb.explore(inst, fspbb.UB_NEH, 4, 64)
        assert r["proven"] and r["opt"] == opt
    with fspbb.create_instance(times(20, 10, 22)) as inst:
        r = fspbb.explore(inst, fspbb.UB_NEH, 4, 512, node_budget=20000)
        assert not r["proven"] and r["status"] == fspbb.BUDGET and r["nodes_bounded"] >= 20000
        assert sorted(r["perm"].tolist()) == list(range(20))


@pytest.mark.parametrize("n,m,seed", [(10, 6, 41), (12, 20, 42), (25, 3, 43)])
def test_explore_pair_subset_and_wide(n, m, seed):
    """Pair subsets (adjacent pairs plus (0, m - 1)) and instances outside the
    incremental path's limits reach the oracle's optimum."""
    require_gpu()
    p = times(n, m, seed)
    S = [(k, k + 1) for k in range(m - 1)] + ([(0, m - 1)] if m > 2 else [])
    for pairs in (S, None):
        want = oracle.bnb(p, *oracle.neh(p), pool_cap=256, pairs=pairs)
        assert want["proven"]
        with fspbb.create_instance(p, pairs=pairs) as inst:
            r = fspbb.explore(inst, fspbb.UB_NEH, 4, 256)
        assert r["proven"] and r["opt"] == want["ub"]
        assert oracle.makespan(p, r["perm"]) == r["opt"]


def test_explore_rejects_bad_arguments():
    require_gpu()
    with fspbb.create_instance(times(6, 3, 31)) as inst:
        for args in [(0, 16), (300, 16), (2, 0)]:
            with pytest.raises(fspbb.FspError):
                fspbb.explore(inst, fspbb.UB_NEH, *args)
