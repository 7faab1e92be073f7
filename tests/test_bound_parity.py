"""GPU bounds against the oracle, element by element, through the C ABI.

Bounds are integers: the bar is bit-exact equality.  Small configurations are
checked on every node; the 200 x 20 pool of 262,144 nodes (the size and launch
the benchmark times) is checked on a seeded sample against the oracle and on
every node against the second kernel family, plus leaf rows against the
makespan.
"""
import numpy as np
import pytest

import oracle
from helpers import CONFIG_SHAPES, oracle_bounds, require_gpu, to_dev, workload
from paper_1208_3933_amd import fspbb, gen

pytestmark = pytest.mark.gpu

VARIANTS = [fspbb.VARIANT_LANE32, fspbb.VARIANT_PACKED16, fspbb.VARIANT_WAVEPAIR, fspbb.VARIANT_WIDE]


def gpu_bounds(torch, inst, pre, dep, variant=fspbb.VARIANT_AUTO):
    pre_d, dep_d = to_dev(torch, pre, dep)
    out = torch.full((dep.shape[0],), -7, dtype=torch.int32, device="cuda")
    fspbb.bound_pool(inst, pre_d, dep_d, out, variant=variant)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("config", [0, 1])
@pytest.mark.parametrize("variant", VARIANTS)
def test_full_pool_parity(config, variant):
    torch = require_gpu()
    n, m, N = CONFIG_SHAPES[config]
    p, pre, dep = workload(config, n, m, N)
    want = oracle_bounds(p, pre, dep)
    with fspbb.create_instance(p) as inst:
        got = gpu_bounds(torch, inst, pre, dep, variant)
        assert fspbb.pool_status(inst) == 0
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} mismatches, first {bad[:5]}: got {got[bad[:5]]} want {want[bad[:5]]}"


def test_200x20_full_pool_sampled_parity():
    torch = require_gpu()
    n, m, N = CONFIG_SHAPES[2]
    p, pre, dep = workload(2, n, m, N)
    with fspbb.create_instance(p) as inst:
        assert inst.info()["packed16"] == 1
        got = gpu_bounds(torch, inst, pre, dep)                           # the benchmarked launch
        got32 = gpu_bounds(torch, inst, pre, dep, fspbb.VARIANT_LANE32)   # the other kernel families
        gotwp = gpu_bounds(torch, inst, pre, dep, fspbb.VARIANT_WAVEPAIR)
        gotw = gpu_bounds(torch, inst, pre, dep, fspbb.VARIANT_WIDE)
        assert fspbb.pool_status(inst) == 0
    assert (got == got32).all() and (got == gotwp).all() and (got == gotw).all()
    idx = np.unique(gen.splitmix64(gen.make_seed(2, 0, 9), 3000) % np.uint64(N)).astype(np.int64)
    want = oracle_bounds(p, pre[idx], dep[idx])
    assert (got[idx] == want).all()
    leaves = np.nonzero(dep == n - 1)[0][:50]
    for i in leaves:  # one job left: the child leaf's makespan bounds it from above
        full = list(pre[i])
        assert got[i] <= oracle.makespan(p, full)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("N", [1, 63, 127, 129, 257, 1000])
def test_ragged_pool_sizes(variant, N):
    torch = require_gpu()
    p, pre, dep = workload(10, 30, 7, N, instance=N)
    want = oracle_bounds(p, pre, dep)
    with fspbb.create_instance(p) as inst:
        assert (gpu_bounds(torch, inst, pre, dep, variant) == want).all()


def test_empty_pool_is_a_noop():
    torch = require_gpu()
    p, _, _ = workload(11, 10, 4, 1)
    with fspbb.create_instance(p) as inst:
        e = torch.zeros((0, 10), dtype=torch.int32, device="cuda")
        d = torch.zeros((0,), dtype=torch.int32, device="cuda")
        o = torch.zeros((0,), dtype=torch.int32, device="cuda")
        fspbb.bound_pool(inst, e, d, o)
        assert fspbb.pool_status(inst) == 0


@pytest.mark.parametrize("variant", VARIANTS)
def test_root_and_leaves(variant):
    """Depth 0 (the root) and depth n (complete permutations: the makespan)."""
    torch = require_gpu()
    n, m = 40, 9
    p, pre, _ = workload(12, n, m, 300)
    dep = np.where(np.arange(300) % 2 == 0, 0, n).astype(np.int32)
    with fspbb.create_instance(p) as inst:
        got = gpu_bounds(torch, inst, pre, dep, variant)
    root = oracle.bound(p, [])
    for i in range(300):
        want = root if dep[i] == 0 else oracle.makespan(p, pre[i])
        assert got[i] == want


@pytest.mark.parametrize("variant", VARIANTS)
def test_two_machines_is_exact(variant):
    torch = require_gpu()
    n = 7
    p, pre, dep = workload(13, n, 2, 200)
    with fspbb.create_instance(p) as inst:
        got = gpu_bounds(torch, inst, pre, dep, variant)
    for i in range(200):
        assert got[i] == oracle.brute(p, pre[i, :dep[i]])


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("n,m,lo,hi", [(1, 2, 1, 99), (1, 32, 1, 99), (33, 32, 1, 99), (64, 3, 1, 3),
                                       (65, 17, 1, 99), (512, 4, 1, 30), (96, 20, 1, 2), (512, 32, 1, 99)])
def test_shape_and_value_edges(variant, n, m, lo, hi):
    torch = require_gpu()
    p = gen.processing_times(n, m, gen.make_seed(14, n * 100 + m, 0), lo, hi)
    pre, dep = gen.random_pool(n, 400, gen.make_seed(14, n * 100 + m, 1), 0, n)
    want = oracle_bounds(p, pre, dep)
    with fspbb.create_instance(p) as inst:
        assert (gpu_bounds(torch, inst, pre, dep, variant) == want).all()


@pytest.mark.parametrize("variant", [fspbb.VARIANT_AUTO, fspbb.VARIANT_LANE32, fspbb.VARIANT_WAVEPAIR])
def test_largest_shape_on_the_32bit_kernel(variant):
    """512 jobs and 32 machines, the limits of both, with values that need
    32-bit arithmetic (max_value 543 x 100,000)."""
    torch = require_gpu()
    n, m = 512, 32
    p = gen.processing_times(n, m, gen.make_seed(15, 1, 0), 1, 100000)
    pre, dep = gen.random_pool(n, 300, gen.make_seed(15, 1, 1), 0, n)
    want = oracle_bounds(p, pre, dep)
    with fspbb.create_instance(p) as inst:
        assert inst.info()["packed16"] == 0
        assert (gpu_bounds(torch, inst, pre, dep, variant) == want).all()


def test_large_values_use_the_32bit_kernel():
    torch = require_gpu()
    n, m = 50, 10
    p = gen.processing_times(n, m, gen.make_seed(15, 0, 0), 1, 100000)
    pre, dep = gen.random_pool(n, 700, gen.make_seed(15, 0, 1))
    want = oracle_bounds(p, pre, dep)
    with fspbb.create_instance(p) as inst:
        assert inst.info()["packed16"] == 0
        assert (gpu_bounds(torch, inst, pre, dep) == want).all()
        assert (gpu_bounds(torch, inst, pre, dep, fspbb.VARIANT_WAVEPAIR) == want).all()
        assert (gpu_bounds(torch, inst, pre, dep, fspbb.VARIANT_LANE32) == want).all()
        with pytest.raises(fspbb.FspError):
            gpu_bounds(torch, inst, pre, dep, fspbb.VARIANT_PACKED16)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("n", [20, 32])
@pytest.mark.parametrize("one_lane", [False, True])
def test_invalid_nodes(variant, n, one_lane, monkeypatch):
    """Invalid depths, repeated and out-of-range jobs; n = 32 puts an
    out-of-range job's bit past the last mask word.  one_lane forces the
    one-lane decode on the 16-bit path."""
    torch = require_gpu()
    if one_lane:
        monkeypatch.setenv("FSPBB_LANES_BELOW", "1")
    m, N = 5, 500
    p, pre, dep = workload(16, n, m, N)
    pre = pre.copy()
    dep = dep.copy()
    dep[3] = n + 1
    dep[4] = -1
    dep[5] = 5; pre[5, 4] = pre[5, 0]          # repeated job
    dep[6] = 3; pre[6, 1] = n                  # job out of range
    dep[7] = 2; pre[7, 0] = -3                 # negative job
    dep[8] = 2; pre[8, 2] = 999                # junk after the prefix is ignored
    dep[9] = 8; pre[9, 7] = n                  # out of range in a full block of 8 slots
    dep[10] = 16; pre[10, 12] = pre[10, 3]     # repeated within full blocks
    want = oracle_bounds(p, pre, dep)
    assert (want[[3, 4, 5, 6, 7, 9, 10]] == oracle.INVALID).all() and want[8] != oracle.INVALID
    with fspbb.create_instance(p) as inst:
        got = gpu_bounds(torch, inst, pre, dep, variant)
        assert fspbb.pool_status(inst) == 7
        assert fspbb.pool_status(inst) == 0
    assert (got == want).all()


def test_500x20_sampled():
    torch = require_gpu()
    n, m, N = 500, 20, 4096
    p, pre, dep = workload(4, n, m, N)
    with fspbb.create_instance(p) as inst:
        assert inst.info()["packed16"] == 1
        got = gpu_bounds(torch, inst, pre, dep)
        got32 = gpu_bounds(torch, inst, pre, dep, fspbb.VARIANT_LANE32)
        gotwp = gpu_bounds(torch, inst, pre, dep, fspbb.VARIANT_WAVEPAIR)
        gotw = gpu_bounds(torch, inst, pre, dep, fspbb.VARIANT_WIDE)
    assert (got == got32).all() and (got == gotwp).all() and (got == gotw).all()
    idx = np.arange(0, N, 16)
    assert (got[idx] == oracle_bounds(p, pre[idx], dep[idx])).all()


def test_ties_heavy_instance():
    torch = require_gpu()
    n, m = 60, 12
    p = gen.processing_times(n, m, gen.make_seed(17, 0, 0), 1, 3)
    pre, dep = gen.random_pool(n, 2000, gen.make_seed(17, 0, 1))
    want = oracle_bounds(p, pre, dep)
    with fspbb.create_instance(p) as inst:
        for v in VARIANTS:
            assert (gpu_bounds(torch, inst, pre, dep, v) == want).all()


@pytest.mark.parametrize("n,m,N", [(200, 20, 262144), (500, 20, 8192)])
def test_wide_values_full_pool(n, m, N):
    """Processing times U[1,300] put 200 x 20 past the 16-bit guard
    ((n+m-1) * 300 >= 65536), so the pool takes the 32-bit decode + scan with
    masks in LDS: every node against the register-bit-set 32-bit kernel, a
    seeded sample against the oracle (the 200 x 20 pool is the benchmark's
    size and launch for this case)."""
    torch = require_gpu()
    p = gen.processing_times(n, m, gen.make_seed(18, n, gen.PURPOSE_TIMES), 1, 300)
    pre, dep = gen.random_pool(n, N, gen.make_seed(18, n, gen.PURPOSE_POOL))
    with fspbb.create_instance(p) as inst:
        assert inst.info()["packed16"] == 0
        got = gpu_bounds(torch, inst, pre, dep)
        got32 = gpu_bounds(torch, inst, pre, dep, fspbb.VARIANT_LANE32)
        assert fspbb.pool_status(inst) == 0
    assert (got == got32).all()
    idx = np.unique(gen.splitmix64(gen.make_seed(18, n, 9), 1500) % np.uint64(N)).astype(np.int64)
    assert (got[idx] == oracle_bounds(p, pre[idx], dep[idx])).all()


def _tail_edge_instance(last):
    """4 jobs x 8 machines whose largest tail, job 0's after machine 0, is
    30,000 + last; the other tails are at most 7 x 4,000."""
    p = gen.processing_times(4, 8, gen.make_seed(19, 0, 0), 1, 4000)
    p[0, 1:7] = 5000
    p[0, 7] = last
    return p


@pytest.mark.parametrize("p_fn", [lambda: _tail_edge_instance(1742), lambda: _tail_edge_instance(1743),
                                  lambda: gen.processing_times(3, 32, gen.make_seed(19, 1, 0), 1500, 1927),
                                  lambda: gen.processing_times(6, 24, gen.make_seed(19, 2, 0), 1600, 2250)])
@pytest.mark.parametrize("one_lane", [False, True])
def test_tails_near_the_half_precision_range(p_fn, one_lane, monkeypatch):
    """16-bit instances whose largest tail is 0x7bfe (the largest the packed
    half-precision minima take), 0x7bff, or far above it: every bound against
    the oracle, on the small-pool decode and on the one-lane decode."""
    torch = require_gpu()
    p = p_fn()
    n, m = p.shape
    qmax = int(np.cumsum(p[:, ::-1], axis=1)[:, -2].max())
    assert qmax >= 0x7bfe
    if one_lane:
        monkeypatch.setenv("FSPBB_LANES_BELOW", "1")
    pre, dep = gen.random_pool(n, 1000, gen.make_seed(19, n * 100 + m, 1), 0, n)
    want = oracle_bounds(p, pre, dep)
    with fspbb.create_instance(p) as inst:
        assert inst.info()["packed16"] == 1
        for v in (fspbb.VARIANT_AUTO, fspbb.VARIANT_PACKED16):
            assert (gpu_bounds(torch, inst, pre, dep, v) == want).all()
