"""Device scratch is kept for reuse per device and stream: bounds on several
streams, searches from several host threads at once, and searches after the
kept memory is released all give the results the same calls give alone."""
import threading

import numpy as np
import pytest

import oracle
from helpers import require_gpu, to_dev
from paper_1208_3933_amd import fspbb, gen

pytestmark = pytest.mark.gpu


def test_pools_on_alternating_streams():
    torch = require_gpu()
    n, m, N = 50, 10, 20000
    p = gen.processing_times(n, m, gen.make_seed(19, 1, gen.PURPOSE_TIMES))
    streams = [torch.cuda.Stream() for _ in range(3)]
    pools = [gen.random_pool(n, N - 1000 * k, gen.make_seed(19, 10 + k, gen.PURPOSE_POOL)) for k in range(3)]
    want = [oracle.bound_pool(p, pre[::97], dep[::97]) for pre, dep in pools]
    with fspbb.create_instance(p) as inst:
        dev = [to_dev(torch, pre, dep) for pre, dep in pools]
        outs = [torch.full((len(dep),), -7, dtype=torch.int32, device="cuda") for _, dep in pools]
        for rnd in range(4):  # each stream reuses its own scratch, and the streams overlap
            for k in range(3):
                fspbb.bound_pool(inst, dev[k][0], dev[k][1], outs[k], streams[(k + rnd) % 3])
        torch.cuda.synchronize()
        got = [o.cpu().numpy() for o in outs]
    for g, w in zip(got, want):
        assert (g[::97] == w).all()


def test_searches_from_several_threads():
    require_gpu()
    shapes = [(12, 5, 1), (11, 6, 2), (14, 4, 3), (10, 8, 4)]
    insts = [fspbb.create_instance(gen.processing_times(n, m, gen.make_seed(20, s, gen.PURPOSE_TIMES)))
             for n, m, s in shapes]
    alone = [fspbb.solve(inst, fspbb.UB_NEH, 64) for inst in insts]
    got = [None] * len(insts)

    def run(k):
        import torch
        with torch.cuda.stream(torch.cuda.Stream()):
            got[k] = [fspbb.solve(insts[k], fspbb.UB_NEH, 64) for _ in range(3)]

    threads = [threading.Thread(target=run, args=(k,)) for k in range(len(insts))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    fspbb.release_cached()
    again = [fspbb.solve(inst, fspbb.UB_NEH, 64) for inst in insts]
    for k, a in enumerate(alone):
        for r in got[k] + [again[k]]:
            for f in ("opt", "nodes_bounded", "steps", "improvements", "max_stack", "status"):
                assert a[f] == r[f], (k, f)
            assert (a["perm"] == r["perm"]).all()
    for inst in insts:
        inst.close()


@pytest.mark.parametrize("chained", [False, True])
def test_kernel_timing_records(chained):
    """Event timing of bound launches, plain (three events per launch) and
    chained (a launch starts at the previous one's end): every launch is
    counted, both parts take time, their sum stays within the wall time of
    the launches, and the bounds are those of an untimed launch."""
    torch = require_gpu()
    n, m, N = 200, 20, 70000
    p = gen.processing_times(n, m, gen.make_seed(23, 0, gen.PURPOSE_TIMES))
    pre, dep = gen.random_pool(n, N, gen.make_seed(23, 0, gen.PURPOSE_POOL))
    with fspbb.create_instance(p) as inst:
        pre_d, dep_d = to_dev(torch, pre, dep)
        ref = torch.empty(N, dtype=torch.int32, device="cuda")
        fspbb.bound_pool(inst, pre_d, dep_d, ref)
        out = torch.empty(N, dtype=torch.int32, device="cuda")
        fspbb.timing_enable(inst, True, chained=chained)
        for rnd in range(2):  # the second round starts a new chain after the read
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                fspbb.bound_pool(inst, pre_d, dep_d, out)
            e1.record()
            torch.cuda.synchronize()
            dec, scan, k = fspbb.timing_read(inst)
            assert k == 5
            assert dec > 0 and scan > 0
            assert dec + scan <= e0.elapsed_time(e1) * 1.01 + 0.01
        fspbb.timing_enable(inst, False)
        assert fspbb.timing_read(inst)[2] == 0
        assert torch.equal(out, ref)
