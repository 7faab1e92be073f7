"""fsp_bound_pool_noalloc (the entry point that allocates nothing) against
fsp_bound_pool through the C ABI, bit-exact, on two calls in a row whose
second input is smaller, so that what the first call left in the shared
per-device workspace cannot leak into the second.  Also: the size limit is
enforced before any launch, invalid nodes are reported as by fsp_bound_pool,
and a 32-bit instance takes the 32-bit path over the same array.
"""
import numpy as np
import pytest

from helpers import CONFIG_SHAPES, oracle_bounds, require_gpu, to_dev, workload
from paper_1208_3933_amd import fspbb, gen

pytestmark = pytest.mark.gpu


def _bounds(torch, inst, pre, dep, noalloc):
    pre_d, dep_d = to_dev(torch, pre, dep)
    out = torch.full((dep.shape[0],), -7, dtype=torch.int32, device="cuda")
    if noalloc:
        fspbb.bound_pool_noalloc(inst, pre_d, dep_d, out)
    else:
        fspbb.bound_pool(inst, pre_d, dep_d, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _check_pair(torch, inst, p, pre, dep, sample=256):
    want = _bounds(torch, inst, pre, dep, noalloc=False)
    got = _bounds(torch, inst, pre, dep, noalloc=True)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} of {dep.shape[0]} differ, first {bad[:5]}: {got[bad[:5]]} vs {want[bad[:5]]}"
    idx = np.unique(gen.splitmix64(gen.make_seed(7, dep.shape[0], 9), sample) % np.uint64(dep.shape[0]))
    idx = idx.astype(np.int64)
    assert (got[idx] == oracle_bounds(p, pre[idx], dep[idx])).all()


def test_noalloc_matches_bound_pool_large_then_small():
    torch = require_gpu()
    n, m, N = CONFIG_SHAPES[2]  # the benchmarked 200 x 20 pool of 262,144 nodes
    p, pre, dep = workload(2, n, m, N)
    with fspbb.create_instance(p) as inst:
        assert inst.info()["packed16"] == 1
        assert fspbb.noalloc_max_nodes(inst) >= N
        _check_pair(torch, inst, p, pre, dep)
        # second call, smaller and ragged (not a multiple of the 128-node group)
        _check_pair(torch, inst, p, pre[:5001], dep[:5001])
        assert fspbb.pool_status(inst) == 0


def test_noalloc_two_instances_in_a_row():
    torch = require_gpu()
    for config, N in [(1, 65536), (0, 1000)]:
        n, m, _ = CONFIG_SHAPES[config]
        p, pre, dep = workload(config, n, m, N)
        with fspbb.create_instance(p) as inst:
            _check_pair(torch, inst, p, pre, dep)


def test_noalloc_invalid_nodes_and_empty_pool():
    torch = require_gpu()
    p, pre, dep = workload(12, 40, 6, 777)
    pre = pre.copy()
    dep = dep.copy()
    dep[3] = 41             # depth out of range
    dep[10] = 5
    pre[10, :5] = [1, 2, 3, 2, 4]   # repeated job
    with fspbb.create_instance(p) as inst:
        got = _bounds(torch, inst, pre, dep, noalloc=True)
        assert fspbb.pool_status(inst) == 2
        want = _bounds(torch, inst, pre, dep, noalloc=False)
        assert fspbb.pool_status(inst) == 2
        assert (got == want).all()
        assert got[3] == fspbb.LB_INVALID and got[10] == fspbb.LB_INVALID
        e = torch.zeros((0, 40), dtype=torch.int32, device="cuda")
        d = torch.zeros((0,), dtype=torch.int32, device="cuda")
        fspbb.bound_pool_noalloc(inst, e, d, torch.zeros((0,), dtype=torch.int32, device="cuda"))


def test_noalloc_rejects_pools_beyond_its_array():
    torch = require_gpu()
    p, _, _ = workload(13, 20, 5, 1)
    with fspbb.create_instance(p) as inst:
        cap = fspbb.noalloc_max_nodes(inst)
        assert 0 < cap < 10_000_000
        pre = torch.zeros((cap + 1, 20), dtype=torch.int32, device="cuda")
        dep = torch.zeros((cap + 1,), dtype=torch.int32, device="cuda")
        out = torch.full((cap + 1,), -7, dtype=torch.int32, device="cuda")
        with pytest.raises(fspbb.FspError) as ei:
            fspbb.bound_pool_noalloc(inst, pre, dep, out)
        assert ei.value.status == fspbb.E_RANGE
        torch.cuda.synchronize()
        assert int((out != -7).sum()) == 0  # nothing was launched


def test_noalloc_32bit_instance_large_then_small():
    torch = require_gpu()
    n, m, N = 200, 20, 150000
    p = gen.processing_times(n, m, gen.make_seed(14, 0, gen.PURPOSE_TIMES), 1, 300)
    pre, dep = gen.random_pool(n, N, gen.make_seed(14, 0, gen.PURPOSE_POOL))
    with fspbb.create_instance(p) as inst:
        assert inst.info()["packed16"] == 0
        assert N <= fspbb.noalloc_max_nodes(inst) < 262144
        _check_pair(torch, inst, p, pre, dep)
        _check_pair(torch, inst, p, pre[:777], dep[:777])
