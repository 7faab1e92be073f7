"""The heads variant of the bound (FSP_INSTANCE_HEADS: releases as the earliest
starts of unscheduled jobs) on the device against the oracle's heads mode:
plain pools in both kernel families, batches mixing variants, whole searches
and served searches."""
import numpy as np
import pytest

import oracle
from helpers import require_gpu, to_dev
from paper_1208_3933_amd import fspbb, gen

pytestmark = pytest.mark.gpu


def oracle_heads(p, pre, dep):
    return oracle.bound_pool(p, pre, dep, heads=True)


@pytest.mark.parametrize("variant", [fspbb.VARIANT_LANE32, fspbb.VARIANT_PACKED16, fspbb.VARIANT_WIDE])
@pytest.mark.parametrize("n,m,N", [(20, 5, 4096), (20, 10, 3000), (50, 10, 2000), (7, 32, 700), (1, 4, 5)])
def test_heads_pool_parity(variant, n, m, N):
    torch = require_gpu()
    p = gen.processing_times(n, m, gen.make_seed(11, n * 100 + m, gen.PURPOSE_TIMES))
    pre, dep = gen.random_pool(n, N, gen.make_seed(11, n * 100 + m, gen.PURPOSE_POOL), 0, n)
    want = oracle_heads(p, pre, dep)
    plain = oracle.bound_pool(p, pre, dep)
    assert (want >= plain).all()
    with fspbb.create_instance(p, heads=True) as inst:
        assert inst.info()["flags"] == fspbb.INSTANCE_HEADS
        pre_d, dep_d = to_dev(torch, pre, dep)
        out = torch.full((N,), -7, dtype=torch.int32, device="cuda")
        fspbb.bound_pool(inst, pre_d, dep_d, out, variant=variant)
        got = out.cpu().numpy()
        assert (got == want).all(), np.nonzero(got != want)[0][:10]


def test_heads_200x20_sampled():
    torch = require_gpu()
    n, m, N = 200, 20, 65536
    p = gen.processing_times(n, m, gen.make_seed(2, 0, gen.PURPOSE_TIMES))
    pre, dep = gen.random_pool(n, N, gen.make_seed(2, 0, gen.PURPOSE_POOL))
    with fspbb.create_instance(p, heads=True) as inst:
        pre_d, dep_d = to_dev(torch, pre, dep)
        a = torch.empty(N, dtype=torch.int32, device="cuda")
        b = torch.empty(N, dtype=torch.int32, device="cuda")
        fspbb.bound_pool(inst, pre_d, dep_d, a, variant=fspbb.VARIANT_PACKED16)
        fspbb.bound_pool(inst, pre_d, dep_d, b, variant=fspbb.VARIANT_LANE32)
        a, b = a.cpu().numpy(), b.cpu().numpy()
    assert (a == b).all()
    idx = np.arange(0, N, N // 500)
    assert (a[idx] == oracle_heads(p, pre[idx], dep[idx])).all()


def test_heads_and_plain_in_one_batch():
    torch = require_gpu()
    pools, want = [], []
    insts = []
    for i, (n, m, N, heads) in enumerate([(20, 10, 3000, True), (20, 10, 3000, False), (50, 5, 700, True),
                                          (100, 20, 1500, True), (100, 20, 900, False)]):
        p = gen.processing_times(n, m, gen.make_seed(12, i, gen.PURPOSE_TIMES))
        pre, dep = gen.random_pool(n, N, gen.make_seed(12, i, gen.PURPOSE_POOL))
        inst = fspbb.create_instance(p, heads=heads)
        insts.append(inst)
        pre_d, dep_d = to_dev(torch, pre, dep)
        out = torch.full((N,), -7, dtype=torch.int32, device="cuda")
        pools.append((inst, pre_d, dep_d, out))
        idx = np.arange(0, N, 7)
        want.append((idx, oracle.bound_pool(p, pre[idx], dep[idx], heads=heads)))
    with fspbb.batch_create(pools, graph=True) as b:
        b.run()
        torch.cuda.synchronize()
    for (inst, _, _, out), (idx, w) in zip(pools, want):
        assert (out.cpu().numpy()[idx] == w).all()
    for inst in insts:
        inst.close()


@pytest.mark.parametrize("n,m,seed,cap", [(8, 4, 1, 16), (9, 5, 2, 1), (10, 6, 3, 64), (12, 5, 4, 256)])
def test_heads_solve_matches_oracle(n, m, seed, cap):
    require_gpu()
    p = gen.processing_times(n, m, gen.make_seed(13, seed, gen.PURPOSE_TIMES))
    ms, perm = oracle.neh(p)
    want = oracle.bnb(p, ms, perm, pool_cap=cap, steplog_cap=1 << 16, heads=True)
    with fspbb.create_instance(p, heads=True) as inst:
        got = fspbb.solve(inst, fspbb.UB_NEH, cap, 1 << 62, 1 << 16)
    assert got["opt"] == want["ub"] and bool(got["proven"]) == want["proven"]
    assert got["nodes_bounded"] == want["nodes_bounded"] and got["steps"] == want["steps"]
    assert got["improvements"] == want["improvements"] and got["max_stack"] == want["max_stack"]
    assert (got["perm"] == want["incumbent"]).all()
    assert (got["steplog"] == want["steplog"]).all()
    if n <= 9:
        assert got["opt"] == oracle.brute(p)


def test_heads_served_same_as_alone():
    require_gpu()
    reqs = []
    for i, (n, m, cap, heads) in enumerate([(10, 6, 64, True), (10, 6, 64, False), (11, 5, 128, True),
                                            (9, 8, 16, True), (12, 4, 300, False)]):
        p = gen.processing_times(n, m, gen.make_seed(14, i, gen.PURPOSE_TIMES))
        reqs.append((fspbb.create_instance(p, heads=heads), cap))
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
