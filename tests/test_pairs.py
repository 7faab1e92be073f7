"""Bounds over a subset of the machine pairs (fsp_create_instance_pairs) on the
device against the oracle's pair-subset mode: pools in the three kernel
mappings, a batch mixing subset and full instances, whole searches (depth
first and best first, every counter and the step log) and served searches."""
import numpy as np
import pytest

import oracle
from helpers import require_gpu, to_dev
from paper_1208_3933_amd import fspbb, gen

pytestmark = pytest.mark.gpu


def subsets(m, seed):
    """Adjacent pairs, pairs ending on the last machine, and a seeded random
    subset holding one pair that ends on the last machine."""
    every = [(k, l) for k in range(m) for l in range(k + 1, m)]
    rng = np.random.default_rng(seed)
    pick = [pr for pr in every if rng.random() < 0.3 and pr[1] < m - 1] + [(int(rng.integers(0, m - 1)), m - 1)]
    return [[(k, k + 1) for k in range(m - 1)], [(k, m - 1) for k in range(m - 1)], pick]


@pytest.mark.parametrize("variant", [fspbb.VARIANT_LANE32, fspbb.VARIANT_PACKED16, fspbb.VARIANT_WAVEPAIR,
                                     fspbb.VARIANT_WIDE])
@pytest.mark.parametrize("n,m,N", [(20, 5, 4096), (50, 10, 3000), (30, 20, 2000), (9, 32, 700)])
def test_pair_subset_pool_parity(variant, n, m, N):
    torch = require_gpu()
    p = gen.processing_times(n, m, gen.make_seed(15, n * 100 + m, gen.PURPOSE_TIMES))
    pre, dep = gen.random_pool(n, N, gen.make_seed(15, n * 100 + m, gen.PURPOSE_POOL), 0, n)
    pre_d, dep_d = to_dev(torch, pre, dep)
    for S in subsets(m, n + m):
        want = oracle.bound_pool(p, pre, dep, pairs=S)
        with fspbb.create_instance(p, pairs=S) as inst:
            info = inst.info()
            assert info["pairs"] == len(S)
            assert info["flags"] == (fspbb.INSTANCE_PAIR_SUBSET if len(S) < m * (m - 1) // 2 else 0)
            out = torch.full((N,), -7, dtype=torch.int32, device="cuda")
            fspbb.bound_pool(inst, pre_d, dep_d, out, variant=variant)
            got = out.cpu().numpy()
        assert (got == want).all(), (S, np.nonzero(got != want)[0][:10])


def test_pair_subset_200x20_sampled():
    torch = require_gpu()
    n, m, N = 200, 20, 65536
    p = gen.processing_times(n, m, gen.make_seed(2, 0, gen.PURPOSE_TIMES))
    pre, dep = gen.random_pool(n, N, gen.make_seed(2, 0, gen.PURPOSE_POOL))
    pre_d, dep_d = to_dev(torch, pre, dep)
    S = [(k, k + 1) for k in range(m - 1)] + [(0, m - 1)]
    with fspbb.create_instance(p, pairs=S) as inst, fspbb.create_instance(p) as full:
        a = torch.empty(N, dtype=torch.int32, device="cuda")
        b = torch.empty(N, dtype=torch.int32, device="cuda")
        f = torch.empty(N, dtype=torch.int32, device="cuda")
        fspbb.bound_pool(inst, pre_d, dep_d, a, variant=fspbb.VARIANT_PACKED16)
        fspbb.bound_pool(inst, pre_d, dep_d, b, variant=fspbb.VARIANT_LANE32)
        fspbb.bound_pool(full, pre_d, dep_d, f)
        a, b, f = a.cpu().numpy(), b.cpu().numpy(), f.cpu().numpy()
    assert (a == b).all() and (a <= f).all()
    idx = np.arange(0, N, N // 400)
    assert (a[idx] == oracle.bound_pool(p, pre[idx], dep[idx], pairs=S)).all()


def test_pair_subset_and_full_in_one_batch():
    torch = require_gpu()
    pools, want, insts = [], [], []
    for i, (n, m, N, sub) in enumerate([(20, 10, 3000, True), (20, 10, 3000, False), (50, 5, 700, True),
                                        (100, 20, 1500, True), (100, 20, 900, False)]):
        p = gen.processing_times(n, m, gen.make_seed(16, i, gen.PURPOSE_TIMES))
        pre, dep = gen.random_pool(n, N, gen.make_seed(16, i, gen.PURPOSE_POOL))
        S = subsets(m, i)[i % 3] if sub else None
        inst = fspbb.create_instance(p, pairs=S)
        insts.append(inst)
        pre_d, dep_d = to_dev(torch, pre, dep)
        out = torch.full((N,), -7, dtype=torch.int32, device="cuda")
        pools.append((inst, pre_d, dep_d, out))
        idx = np.arange(0, N, 7)
        want.append((idx, oracle.bound_pool(p, pre[idx], dep[idx], pairs=S)))
    with fspbb.batch_create(pools, graph=True) as b:
        b.run()
        torch.cuda.synchronize()
    for (inst, _, _, out), (idx, w) in zip(pools, want):
        assert (out.cpu().numpy()[idx] == w).all()
    for inst in insts:
        inst.close()


@pytest.mark.parametrize("best_first", [False, True])
@pytest.mark.parametrize("n,m,seed,cap", [(8, 4, 1, 16), (9, 5, 2, 1), (10, 6, 3, 64), (12, 5, 4, 256)])
def test_pair_subset_solve_matches_oracle(n, m, seed, cap, best_first):
    require_gpu()
    p = gen.processing_times(n, m, gen.make_seed(17, seed, gen.PURPOSE_TIMES))
    ms, perm = oracle.neh(p)
    S = subsets(m, seed)[seed % 3]
    want = oracle.bnb(p, ms, perm, pool_cap=cap, steplog_cap=1 << 16, best_first=best_first, pairs=S)
    with fspbb.create_instance(p, pairs=S) as inst:
        got = fspbb.solve(inst, fspbb.UB_NEH, cap, 1 << 62, 1 << 16, best_first=best_first)
    assert got["opt"] == want["ub"] and bool(got["proven"]) == want["proven"]
    assert got["nodes_bounded"] == want["nodes_bounded"] and got["steps"] == want["steps"]
    assert got["improvements"] == want["improvements"] and got["max_stack"] == want["max_stack"]
    assert (got["perm"] == want["incumbent"]).all()
    assert (got["steplog"] == want["steplog"]).all()
    if n <= 9:
        assert got["opt"] == oracle.brute(p)


def test_pair_subset_served_same_as_alone():
    require_gpu()
    reqs = []
    for i, (n, m, cap, sub) in enumerate([(10, 6, 64, True), (10, 6, 64, False), (11, 5, 128, True),
                                          (9, 8, 16, True), (12, 4, 300, False)]):
        p = gen.processing_times(n, m, gen.make_seed(18, i, gen.PURPOSE_TIMES))
        reqs.append((fspbb.create_instance(p, pairs=subsets(m, i)[i % 3] if sub else None), cap))
    alone = [fspbb.solve(inst, fspbb.UB_NEH, cap) for inst, cap in reqs]
    got = {}
    with fspbb.server_create(1 << 30, 16) as srv:
        ids = {srv.submit(inst, fspbb.UB_NEH, cap): k for k, (inst, cap) in enumerate(reqs)}
        while len(got) < len(reqs):
            done, _ = srv.step()
            for i in done:
                got[ids[i]] = srv.poll(i)
    for k, a in enumerate(alone):
        g = got[k]
        for f in ("opt", "proven", "nodes_bounded", "steps", "improvements", "max_stack", "status"):
            assert a[f] == g[f], (k, f)
        assert (a["perm"] == g["perm"]).all()
    for inst, _ in reqs:
        inst.close()
