"""Batched bounding (many pools, one persistent graph-captured launch) against
the plain per-pool launch and the oracle, element by element."""
import numpy as np
import pytest

import oracle
from helpers import oracle_bounds, require_gpu, to_dev
from paper_1208_3933_amd import fspbb, gen

pytestmark = pytest.mark.gpu

CONFIG3_SHAPES = [(20, 5), (20, 10), (20, 20), (50, 10), (100, 20), (200, 20)]
SHAPES = CONFIG3_SHAPES + [(500, 20)]  # 500 x 20: the mask tile alone fills most of LDS


def make_batch(torch, n_pools, sizes, config=3, invalid_in=None, shapes=SHAPES):
    pools, host = [], []
    insts = {}
    for i in range(n_pools):
        n, m = shapes[i % len(shapes)]
        key = (n, m, i // len(shapes) % 2)  # two instances per shape, pools share them
        if key not in insts:
            p = gen.processing_times(n, m, gen.make_seed(config, len(insts), gen.PURPOSE_TIMES))
            insts[key] = (fspbb.create_instance(p), p)
        inst, p = insts[key]
        N = int(sizes[i])
        pre, dep = gen.random_pool(n, N, gen.make_seed(config, 100 + i, gen.PURPOSE_POOL))
        if invalid_in is not None and i in invalid_in and N > 3:
            dep = dep.copy()
            dep[1] = n + 5
        pre_d, dep_d = to_dev(torch, pre, dep)
        out = torch.full((N,), -7, dtype=torch.int32, device="cuda")
        pools.append((inst, pre_d, dep_d, out))
        host.append((p, pre, dep))
    return pools, host, insts


def plain_bounds(torch, pools):
    res = []
    for inst, pre_d, dep_d, _ in pools:
        N = int(dep_d.shape[0])
        o = torch.full((N,), -9, dtype=torch.int32, device="cuda")
        if N:
            fspbb.bound_pool(inst, pre_d, dep_d, o)
        res.append(o)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in res]


@pytest.mark.parametrize("form", [fspbb.FORM_GRID, fspbb.FORM_PERSISTENT])
@pytest.mark.parametrize("graph", [True, False])
def test_mixed_batch_matches_plain_and_oracle(graph, form):
    torch = require_gpu()
    sizes = [300, 1000, 129, 0, 2048, 700, 128, 4000, 64, 513, 1, 3000]
    # invalid nodes in a pool decoded in depth order (1000 nodes) and in one decoded in pool order (129)
    pools, host, insts = make_batch(torch, len(sizes), sizes, invalid_in=(1, 2))
    want_plain = plain_bounds(torch, pools)
    saved = {(n, m): fspbb.tune_get_form(n, m) for n, m in SHAPES}
    for n, m in SHAPES:
        fspbb.tune_set_form(n, m, form)
    try:
        with fspbb.batch_create(pools, graph=graph) as b:
            info = b.info()
            assert info["total_nodes"] == sum(sizes)
            if form == fspbb.FORM_GRID:
                assert info["grid"] == info["items"]
            b.run()
            torch.cuda.synchronize()
    finally:
        for (n, m), f in saved.items():
            fspbb.tune_set_form(n, m, f)
    for i, (inst, _, _, out) in enumerate(pools):
        got = out.cpu().numpy()
        assert (got == want_plain[i]).all(), i
        p, pre, dep = host[i]
        if len(dep):
            idx = np.arange(0, len(dep), max(1, len(dep) // 300))
            assert (got[idx] == oracle_bounds(p, pre[idx], dep[idx])).all(), i
    for inst, _ in insts.values():
        fspbb.pool_status(inst)
        inst.close()


def test_graph_replays_with_eager_work_between():
    torch = require_gpu()
    sizes = [500, 257, 1200, 64, 900, 300]
    pools, host, insts = make_batch(torch, len(sizes), sizes, config=5)
    with fspbb.batch_create(pools, graph=True) as b:
        for rep in range(4):
            # change the pools' contents in place (same buffers), with eager work between replays
            for i, (inst, pre_d, dep_d, out) in enumerate(pools):
                n = inst.n
                g = torch.Generator(device="cpu").manual_seed(1000 * rep + i)
                dep_d.copy_(torch.randint(0, n + 1, (dep_d.shape[0],), generator=g, dtype=torch.int32))
                out.fill_(-5)
            scratch = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work
            want = plain_bounds(torch, pools)
            b.run()
            torch.cuda.synchronize()
            assert torch.isfinite(scratch)
            for i, (_, _, _, out) in enumerate(pools):
                assert (out.cpu().numpy() == want[i]).all(), (rep, i)
    for inst, _ in insts.values():
        inst.close()


def test_one_shot_batched():
    torch = require_gpu()
    sizes = [100, 2000, 333]
    pools, host, insts = make_batch(torch, len(sizes), sizes, config=6)
    want = plain_bounds(torch, pools)
    fspbb.bound_pools_batched(pools)
    for i, (_, _, _, out) in enumerate(pools):
        assert (out.cpu().numpy() == want[i]).all()
    for inst, _ in insts.values():
        inst.close()


def test_full_batched_configuration():
    """64 seeded instances of mixed shape, log-normal pool sizes 256..131072."""
    torch = require_gpu()
    sizes = gen.lognormal_pool_sizes(64, gen.make_seed(3, 0, gen.PURPOSE_SIZES))
    pools, host, insts = make_batch(torch, 64, sizes, shapes=CONFIG3_SHAPES)
    want = plain_bounds(torch, pools)
    with fspbb.batch_create(pools, graph=True) as b:
        b.run()
        b.run()
        torch.cuda.synchronize()
    for i, (_, _, _, out) in enumerate(pools):
        got = out.cpu().numpy()
        assert (got == want[i]).all(), i
        p, pre, dep = host[i]
        idx = np.arange(0, len(dep), max(1, len(dep) // 24))
        assert (got[idx] == oracle_bounds(p, pre[idx], dep[idx])).all(), i
    for inst, _ in insts.values():
        inst.close()


def test_batch_rejects_bad_descriptors():
    torch = require_gpu()
    p = gen.processing_times(10, 4, gen.make_seed(7, 0, 0), 1, 100000)  # beyond the 16-bit path
    with fspbb.create_instance(p) as inst:
        d = torch.zeros((1,), dtype=torch.int32, device="cuda")
        pre = torch.zeros((1, 10), dtype=torch.int32, device="cuda")
        with pytest.raises(fspbb.FspError):
            fspbb.batch_create([(inst, pre, d, d)])


@pytest.mark.parametrize("n,m", [(20, 5), (50, 10), (200, 20)])
def test_autotune_picks_a_measured_schedule(n, m):
    torch = require_gpu()
    p = gen.processing_times(n, m, gen.make_seed(8, n, 0))
    with fspbb.create_instance(p) as inst:
        r = fspbb.autotune(inst, sample_nodes=4096, reps=2)
        assert r["waves_per_group"] in r["candidates"]
        assert r["grid_us"] == min(r["candidates"].values())
        assert fspbb.tune_get(n, m) == (r["waves_per_group"], True)
        assert r["form"] in (fspbb.FORM_GRID, fspbb.FORM_PERSISTENT) and fspbb.tune_get_form(n, m) == r["form"]
        assert r["best_us"] == min(r["grid_us"], r["persistent_us"])
        # bounds stay identical under the tuned schedule
        pre, dep = gen.random_pool(n, 3000, gen.make_seed(8, n, 1))
        pre_d, dep_d = to_dev(torch, pre, dep)
        out = torch.empty(3000, dtype=torch.int32, device="cuda")
        fspbb.bound_pool(inst, pre_d, dep_d, out)
        idx = np.arange(0, 3000, 10)
        assert (out.cpu().numpy()[idx] == oracle_bounds(p, pre[idx], dep[idx])).all()


# Shapes whose rule-of-thumb tile (16 / wpg groups of (n + 1) x 256 bytes of
# masks) would exceed the 160 KB of LDS: 100 x 5 (8 groups, 206,848 B),
# 500 x 10 (4 groups, 256 KB), 200 x 10 and 200 x 20 over the 19 adjacent
# pairs (4 groups, 205,824 B).  The planner raises the waves per group until
# the tile fits.
BIG_TILE_SHAPES = [(100, 5, None), (500, 10, None), (200, 10, None), (200, 20, "adjacent")]


@pytest.mark.parametrize("graph", [True, False])
def test_batch_shapes_whose_rule_tile_exceeds_lds(graph):
    torch = require_gpu()
    pools, host, insts = [], [], []
    for s, (n, m, sub) in enumerate(BIG_TILE_SHAPES):
        p = gen.processing_times(n, m, gen.make_seed(3, 700 + s, gen.PURPOSE_TIMES))
        pairs = [(k, k + 1) for k in range(m - 1)] if sub else None
        inst = fspbb.create_instance(p, pairs=pairs)
        insts.append(inst)
        wpg, tuned = fspbb.tune_get(n, m)
        if not sub and not tuned:
            assert (16 // wpg) * (n + 1) * 256 <= 160 * 1024, (n, m, wpg)
        for N in (2048, 2047, 900):
            pre, dep = gen.random_pool(n, N, gen.make_seed(3, 710 + 10 * s + N % 7, gen.PURPOSE_POOL))
            pre_d, dep_d = to_dev(torch, pre, dep)
            out = torch.full((N,), -7, dtype=torch.int32, device="cuda")
            pools.append((inst, pre_d, dep_d, out))
            host.append((p, pre, dep, pairs))
    want_plain = plain_bounds(torch, pools)
    with fspbb.batch_create(pools, graph=graph) as b:
        b.run()
        b.run()
        torch.cuda.synchronize()
    for i, (inst, _, _, out) in enumerate(pools):
        got = out.cpu().numpy()
        assert (got == want_plain[i]).all(), i
        p, pre, dep, pairs = host[i]
        idx = np.arange(len(dep)) if p.shape[0] <= 100 else np.arange(0, len(dep), 7)
        want = oracle.bound_pool(p, pre[idx], dep[idx], pairs=pairs)
        assert (got[idx] == want).all(), i
    for inst in insts:
        assert fspbb.pool_status(inst) == 0
        inst.close()
