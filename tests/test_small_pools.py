"""Pools too small to fill the chip (fewer 128-node groups than compute
units) take the four-lanes-per-node decode and a scan whose machine pairs are
split over several workgroups, combined by atomic max.  Bounds are integers:
every one is compared bit-exactly with the oracle, and with the regular
one-lane decode and one-workgroup-per-group scan (FSPBB_SMALL_SPLITS=1) on the
same pool.
"""
import os

import numpy as np
import pytest

import oracle
from helpers import oracle_bounds, require_gpu, to_dev
from paper_1208_3933_amd import fspbb, gen

pytestmark = pytest.mark.gpu


def _bounds(torch, inst, pre, dep, regular=False):
    pre_d, dep_d = to_dev(torch, pre, dep)
    out = torch.full((dep.shape[0],), -7, dtype=torch.int32, device="cuda")
    old = os.environ.get("FSPBB_SMALL_SPLITS")
    if regular:
        os.environ["FSPBB_SMALL_SPLITS"] = "1"
    try:
        fspbb.bound_pool(inst, pre_d, dep_d, out)
        torch.cuda.synchronize()
    finally:
        if regular:
            if old is None:
                del os.environ["FSPBB_SMALL_SPLITS"]
            else:
                os.environ["FSPBB_SMALL_SPLITS"] = old
    return out.cpu().numpy()


@pytest.mark.parametrize("n,m", [(20, 5), (50, 10), (200, 20), (100, 5), (1, 2), (7, 32), (33, 3), (64, 17)])
@pytest.mark.parametrize("N", [1, 63, 64, 129, 1000, 4096])
def test_small_pool_parity(n, m, N):
    torch = require_gpu()
    p = gen.processing_times(n, m, gen.make_seed(19, n * 100 + m, gen.PURPOSE_TIMES))
    pre, dep = gen.random_pool(n, N, gen.make_seed(19, n * 100 + m + N, gen.PURPOSE_POOL), 0, n)
    with fspbb.create_instance(p) as inst:
        assert inst.info()["packed16"] == 1
        got = _bounds(torch, inst, pre, dep)
        reg = _bounds(torch, inst, pre, dep, regular=True)
        assert fspbb.pool_status(inst) == 0
    bad = np.nonzero(got != reg)[0]
    assert bad.size == 0, f"{bad.size} differ from the regular path, first {bad[:5]}: {got[bad[:5]]} vs {reg[bad[:5]]}"
    if n * N <= 200 * 1000:
        want = oracle_bounds(p, pre, dep)
    else:
        idx = np.arange(0, N, 7)
        want, got = oracle_bounds(p, pre[idx], dep[idx]), got[idx]
    assert (got == want).all()


@pytest.mark.parametrize("n,m,N", [(200, 20, 4096), (500, 20, 2048), (512, 32, 700), (200, 20, 32000)])
def test_small_pool_large_shapes_sampled(n, m, N):
    torch = require_gpu()
    p = gen.processing_times(n, m, gen.make_seed(20, n * 100 + m, gen.PURPOSE_TIMES))
    pre, dep = gen.random_pool(n, N, gen.make_seed(20, n * 100 + m, gen.PURPOSE_POOL), 0, n)
    with fspbb.create_instance(p) as inst:
        got = _bounds(torch, inst, pre, dep)
        reg = _bounds(torch, inst, pre, dep, regular=True)
    assert (got == reg).all()
    idx = np.unique(gen.splitmix64(gen.make_seed(20, n, 9), 400) % np.uint64(N)).astype(np.int64)
    assert (got[idx] == oracle_bounds(p, pre[idx], dep[idx])).all()


@pytest.mark.parametrize("lanes", ["4", "8"])
def test_small_pool_invalid_nodes_and_leaves(lanes, monkeypatch):
    monkeypatch.setenv("FSPBB_LANES_PER_NODE", lanes)
    torch = require_gpu()
    n, m, N = 30, 6, 300
    p = gen.processing_times(n, m, gen.make_seed(21, 0, gen.PURPOSE_TIMES))
    pre, dep = gen.random_pool(n, N, gen.make_seed(21, 0, gen.PURPOSE_POOL), 0, n)
    pre, dep = pre.copy(), dep.copy()
    dep[0] = n + 1                          # depth out of range
    dep[1] = -2
    dep[2] = 6; pre[2, 5] = pre[2, 1]        # repeated job
    dep[3] = 4; pre[3, 3] = n                # job out of range
    dep[4] = 3; pre[4, 0] = -1               # negative job
    dep[5] = n                               # complete schedule: the makespan
    dep[6] = 0                               # the root
    want = oracle_bounds(p, pre, dep)
    assert (want[:5] == oracle.INVALID).all()
    with fspbb.create_instance(p) as inst:
        got = _bounds(torch, inst, pre, dep)
        assert fspbb.pool_status(inst) == 5
    assert (got == want).all()
    assert got[5] == oracle.makespan(p, pre[5]) and got[6] == oracle.bound(p, [])


def test_small_pool_heads_instance_takes_the_regular_path():
    torch = require_gpu()
    n, m, N = 20, 10, 1500
    p = gen.processing_times(n, m, gen.make_seed(22, 0, gen.PURPOSE_TIMES))
    pre, dep = gen.random_pool(n, N, gen.make_seed(22, 0, gen.PURPOSE_POOL), 0, n)
    with fspbb.create_instance(p, heads=True) as inst:
        got = _bounds(torch, inst, pre, dep)
    assert (got == oracle.bound_pool(p, pre, dep, heads=True)).all()


@pytest.mark.parametrize("n,m,N", [(200, 20, 1000), (64, 8, 4096)])
def test_small_pool_rows_off_16_byte_boundary(n, m, N):
    """Prefix rows that do not start on a 16-byte boundary are staged word by
    word instead of 16 bytes at a time; the bounds are the same."""
    torch = require_gpu()
    p = gen.processing_times(n, m, gen.make_seed(23, n, gen.PURPOSE_TIMES))
    pre, dep = gen.random_pool(n, N, gen.make_seed(23, n, gen.PURPOSE_POOL), 0, n)
    buf = torch.zeros(N * n + 1, dtype=torch.int32, device="cuda")
    buf[1:] = torch.from_numpy(np.ascontiguousarray(pre).reshape(-1)).to("cuda")
    pre_off = buf[1:].view(N, n)
    assert pre_off.data_ptr() % 16 == 4
    dep_d = torch.from_numpy(dep).to("cuda")
    out = torch.full((N,), -7, dtype=torch.int32, device="cuda")
    with fspbb.create_instance(p) as inst:
        fspbb.bound_pool(inst, pre_off, dep_d, out)
        torch.cuda.synchronize()
        aligned = _bounds(torch, inst, pre, dep)
    got = out.cpu().numpy()
    assert (got == aligned).all()
    idx = np.arange(0, N, 5)
    assert (got[idx] == oracle_bounds(p, pre[idx], dep[idx])).all()


@pytest.mark.parametrize("fill,minp,ppw", [(8, 2, 1), (4, 4, 2), (2, 1, 1)])
def test_small_pool_split_shapes(fill, minp, ppw):
    """Other shapes of the split scan (workgroups per compute unit, least pairs
    per split, pairs per wave) give the same bounds."""
    torch = require_gpu()
    n, m, N = 200, 20, 4096
    p = gen.processing_times(n, m, gen.make_seed(24, 0, gen.PURPOSE_TIMES))
    pre, dep = gen.random_pool(n, N, gen.make_seed(24, 0, gen.PURPOSE_POOL), 0, n)
    keys = {"FSPBB_SPLIT_FILL": fill, "FSPBB_SPLIT_MIN_PAIRS": minp, "FSPBB_SPLIT_PAIRS_PER_WAVE": ppw}
    with fspbb.create_instance(p) as inst:
        want = _bounds(torch, inst, pre, dep, regular=True)
        old = {k: os.environ.get(k) for k in keys}
        try:
            for k, v in keys.items():
                os.environ[k] = str(v)
            got = _bounds(torch, inst, pre, dep)
        finally:
            for k, v in old.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
    assert (got == want).all()


@pytest.mark.parametrize("n,m", [(20, 5), (200, 20), (7, 32), (33, 3), (64, 17), (1, 2), (256, 32)])
@pytest.mark.parametrize("N", [63, 1000, 4096])
@pytest.mark.parametrize("lanes", [4, 8])
def test_small_pool_lanes_per_node(n, m, N, lanes):
    """The small-pool decode with four or eight lanes per node (the machines
    split over the node's lanes) gives the regular path's bounds."""
    torch = require_gpu()
    p = gen.processing_times(n, m, gen.make_seed(25, n * 100 + m, gen.PURPOSE_TIMES))
    pre, dep = gen.random_pool(n, N, gen.make_seed(25, n * 100 + m + N, gen.PURPOSE_POOL), 0, n)
    old = os.environ.get("FSPBB_LANES_PER_NODE")
    with fspbb.create_instance(p) as inst:
        want = _bounds(torch, inst, pre, dep, regular=True)
        try:
            os.environ["FSPBB_LANES_PER_NODE"] = str(lanes)
            got = _bounds(torch, inst, pre, dep)
            assert fspbb.pool_status(inst) == 0
        finally:
            if old is None:
                os.environ.pop("FSPBB_LANES_PER_NODE", None)
            else:
                os.environ["FSPBB_LANES_PER_NODE"] = old
    assert (got == want).all()
    idx = np.arange(0, N, 11)
    assert (got[idx] == oracle_bounds(p, pre[idx], dep[idx])).all()


@pytest.mark.parametrize("n,m,N", [(200, 20, 129), (200, 20, 3000), (100, 10, 1000), (500, 20, 1000), (33, 3, 64)])
def test_one_lane_decode_with_split_scan(n, m, N, monkeypatch):
    """Small pools on the one-lane decode (forced here; the default for more
    than 256 jobs) with the scan's pairs split over several workgroups (also
    forced, for the shapes whose scans are too short to split by default):
    the decode writes 0 to each valid node's bound and the splits take the
    maximum into it.  Invalid nodes and leaves included; every bound against
    the unsplit path, and against the oracle."""
    torch = require_gpu()
    monkeypatch.setenv("FSPBB_LANES_BELOW", "1")
    monkeypatch.setenv("FSPBB_ONE_LANE_FILL", "3")
    p = gen.processing_times(n, m, gen.make_seed(22, n * 100 + m, gen.PURPOSE_TIMES))
    pre, dep = gen.random_pool(n, N, gen.make_seed(22, n * 100 + m + N, gen.PURPOSE_POOL), 0, n)
    dep[1] = n + 2
    dep[2] = -1
    dep[3] = 3
    pre[3, 2] = pre[3, 0]  # repeated job
    with fspbb.create_instance(p) as inst:
        got = _bounds(torch, inst, pre, dep)
        assert fspbb.pool_status(inst) == 3
        reg = _bounds(torch, inst, pre, dep, regular=True)
        assert fspbb.pool_status(inst) == 3
    assert (got[[1, 2, 3]] == oracle.INVALID).all()
    assert (got == reg).all()
    idx = np.arange(N) if n * N <= 200 * 3000 else np.arange(0, N, 5)
    assert (got[idx] == oracle_bounds(p, pre[idx], dep[idx])).all()
