"""Branch-and-bound on the GPU against the oracle's pool-synchronous DFS.

Node counts, upper-bound trajectories, survivor order fingerprints, the final
makespan and the incumbent permutation are integers and must match exactly.
"""
import numpy as np
import pytest

import oracle
from helpers import load_golden, oracle_bounds, require_gpu, survivors_digest, to_dev
from paper_1208_3933_amd import fspbb, gen

pytestmark = pytest.mark.gpu


def inst_times(n, m, seed, lo=1, hi=99):
    return gen.processing_times(n, m, gen.make_seed(40, seed, 0), lo, hi)


# --- NEH ----------------------------------------------------------------------

@pytest.mark.parametrize("n,m,seed", [(5, 3, 1), (12, 5, 2), (20, 20, 3), (50, 10, 4), (100, 20, 5), (200, 20, 6),
                                      (512, 32, 7)])
def test_neh_matches_oracle(n, m, seed):
    require_gpu()
    p = inst_times(n, m, seed)
    want_ms, want_perm = oracle.neh(p)
    with fspbb.create_instance(p) as inst:
        ms, perm = fspbb.neh(inst)
    assert ms == want_ms
    assert (perm == want_perm).all()


# --- one step -----------------------------------------------------------------

def expected_step(p, parents, depths, ub_in):
    n = p.shape[0]
    kids = []
    for i in range(len(depths)):
        d = int(depths[i])
        if d >= n:
            continue
        pre = [int(x) for x in parents[i, :d]]
        for j in sorted(set(range(n)) - set(pre)):
            kids.append((pre + [j], j))
    rows = np.zeros((max(len(kids), 1), n), np.int32)
    dep = np.zeros(max(len(kids), 1), np.int32)
    for c, (row, _) in enumerate(kids):
        rows[c, :len(row)] = row
        dep[c] = len(row)
    lbs = oracle_bounds(p, rows[:len(kids)], dep[:len(kids)]) if kids else np.zeros(0, np.int32)
    ub, inc = ub_in, None
    for (row, _), lb in zip(kids, lbs):
        if len(row) == n and lb < ub:
            ub, inc = int(lb), row
    surv = [(row, j, int(lb)) for (row, j), lb in zip(kids, lbs) if len(row) < n and lb < ub]
    S = len(surv)
    fp = sum((S - s) * (j + 1) for s, (_, j, _) in enumerate(surv))
    return {"n_children": len(kids), "n_survivors": S, "ub_out": ub, "improved": int(inc is not None),
            "fingerprint": fp, "survivors": surv, "incumbent": inc}


# With no upper bound every non-leaf child survives, so its bound is checked.
# The 16-bit instances bound the children from their parents; the shapes
# cover rows whose length is and is not a multiple of 4, m below, at and
# above 20 (padded machine slots), and up to 32 machines.
@pytest.mark.parametrize("n,m,K,seed,ub_mode", [(8, 4, 9, 1, "none"), (8, 4, 30, 2, "tight"),
                                                (20, 5, 64, 3, "neh"), (50, 10, 40, 4, "neh"),
                                                (12, 6, 50, 5, "deep"), (200, 20, 120, 6, "none"),
                                                (50, 19, 150, 7, "none"), (300, 32, 16, 8, "none"),
                                                (30, 7, 400, 9, "deep"), (512, 32, 4, 10, "none"),
                                                (512, 32, 3, 11, "deep")])
def test_branch_and_prune_step(n, m, K, seed, ub_mode):
    check_step(inst_times(n, m, seed), K, seed, ub_mode)


# Processing times up to 100,000 put the instance on the 32-bit path, whose
# children are bounded from their rows; the largest shape is the limit of
# both jobs and machines.
@pytest.mark.parametrize("n,m,K,seed,ub_mode", [(20, 5, 30, 12, "neh"), (50, 10, 40, 13, "none"),
                                                (512, 32, 3, 14, "none"), (40, 6, 200, 15, "deep")])
def test_branch_and_prune_step_32bit(n, m, K, seed, ub_mode):
    p = inst_times(n, m, seed, 1, 100000)
    check_step(p, K, seed, ub_mode, packed16=0)


def check_step(p, K, seed, ub_mode, packed16=1):
    torch = require_gpu()
    n = p.shape[0]
    if ub_mode == "deep":
        pre, dep = gen.random_pool(n, K, gen.make_seed(41, seed, 1), n - 2, n)
    else:
        pre, dep = gen.random_pool(n, K, gen.make_seed(41, seed, 1))
    neh_ms, _ = oracle.neh(p)
    ub_in = {"none": fspbb.UB_NONE, "neh": neh_ms, "deep": neh_ms + 50,
             "tight": int(np.median(oracle_bounds(p, pre, dep)))}[ub_mode]
    want = expected_step(p, pre, dep, ub_in)
    cap = max(want["n_children"], 1)
    with fspbb.create_instance(p) as inst:
        assert inst.info()["packed16"] == packed16
        pre_d, dep_d = to_dev(torch, pre, dep)
        rows = torch.full((cap, n), -9, dtype=torch.int32, device="cuda")
        cdep = torch.full((cap,), -9, dtype=torch.int32, device="cuda")
        clb = torch.full((cap,), -9, dtype=torch.int32, device="cuda")
        inc = torch.full((n,), -9, dtype=torch.int32, device="cuda")
        res = fspbb.branch_and_prune(inst, pre_d, dep_d, ub_in, rows, cdep, clb, inc)
    assert res["status"] == fspbb.OK
    for key in ["n_children", "n_survivors", "ub_out", "improved", "fingerprint"]:
        assert res[key] == want[key], key
    rows, cdep, clb = rows.cpu().numpy(), cdep.cpu().numpy(), clb.cpu().numpy()
    for s, (row, _, lb) in enumerate(want["survivors"]):
        assert cdep[s] == len(row) and clb[s] == lb
        assert list(rows[s, :len(row)]) == row
    if want["incumbent"] is not None:
        assert list(inc.cpu().numpy()) == want["incumbent"]


def test_branch_and_prune_full_pool_sampled():
    """A full 200 x 20 step (1,324 parents of depth 2: 262,152 children, the
    DFS leg's pool) with no upper bound: every child survives in child order.
    Every row is checked, every bound against the row-based plain bound of
    the same rows, and a sample of bounds against the oracle."""
    torch = require_gpu()
    n, m, K = 200, 20, 1324
    p = gen.processing_times(n, m, gen.make_seed(2, 0, gen.PURPOSE_TIMES))
    pre, dep = gen.random_pool(n, K, gen.make_seed(41, 77, 1), 2, 2)
    nch = K * (n - 2)
    with fspbb.create_instance(p) as inst:
        pre_d, dep_d = to_dev(torch, pre, dep)
        rows = torch.full((nch, n), -9, dtype=torch.int32, device="cuda")
        cdep = torch.full((nch,), -9, dtype=torch.int32, device="cuda")
        clb = torch.full((nch,), -9, dtype=torch.int32, device="cuda")
        res = fspbb.branch_and_prune(inst, pre_d, dep_d, fspbb.UB_NONE, rows, cdep, clb)
        assert res["status"] == fspbb.OK and res["n_children"] == nch and res["n_survivors"] == nch
        plain = torch.full((nch,), -7, dtype=torch.int32, device="cuda")
        fspbb.bound_pool(inst, rows, cdep, plain)
        torch.cuda.synchronize()
        rows3, cdep, clb, plain = rows[:, :3].cpu().numpy(), cdep.cpu().numpy(), clb.cpu().numpy(), plain.cpu().numpy()
    assert (cdep == 3).all() and (clb == plain).all()
    # child c: parent c // 198, its (c % 198)-th unscheduled job in increasing id
    par = np.arange(nch) // (n - 2)
    assert (rows3[:, :2] == pre[par, :2]).all()
    free = np.sort(pre[:, 2:], axis=1)
    assert (rows3[:, 2] == free[par, np.arange(nch) % (n - 2)]).all()
    idx = np.arange(0, nch, nch // 300)
    want = oracle.bound_pool(p, np.ascontiguousarray(np.concatenate([pre[par[idx], :2], rows3[idx, 2:3],
                                                                     np.zeros((len(idx), n - 3), np.int32)], axis=1)),
                             np.full(len(idx), 3, np.int32))
    assert (clb[idx] == want).all()


def test_branch_and_prune_errors():
    torch = require_gpu()
    n, m = 6, 3
    p = inst_times(n, m, 9)
    with fspbb.create_instance(p) as inst:
        pre = torch.tensor([[0, 1, 2, 3, 4, 5], [0, 0, 1, 2, 3, 4]], dtype=torch.int32, device="cuda")
        dep = torch.tensor([2, 3], dtype=torch.int32, device="cuda")  # second parent repeats job 0
        rows = torch.zeros((1, n), dtype=torch.int32, device="cuda")
        cdep = torch.zeros((1,), dtype=torch.int32, device="cuda")
        res = fspbb.branch_and_prune(inst, pre, dep, fspbb.UB_NONE, rows, cdep)
        assert res["status"] == fspbb.E_BADNODE
        dep = torch.tensor([2, 2], dtype=torch.int32, device="cuda")
        pre[1, 1] = 5
        res = fspbb.branch_and_prune(inst, pre, dep, fspbb.UB_NONE, rows, cdep)
        assert res["status"] == fspbb.E_RANGE and res["n_survivors"] == 8 and res["n_children"] == 8


# --- whole searches -----------------------------------------------------------

def compare_solve(p, ub_mode, pool_cap, budget=1 << 62, steplog_cap=1 << 16):
    n = p.shape[0]
    if ub_mode == "neh":
        ms, perm = oracle.neh(p)
        want = oracle.bnb(p, ms, perm, pool_cap=pool_cap, node_budget=budget, steplog_cap=steplog_cap)
        ub0 = fspbb.UB_NEH
    else:
        want = oracle.bnb(p, fspbb.UB_NONE, None, pool_cap=pool_cap, node_budget=budget, steplog_cap=steplog_cap)
        ub0 = fspbb.UB_NONE
    with fspbb.create_instance(p) as inst:
        got = fspbb.solve(inst, ub0, pool_cap, budget, steplog_cap)
    assert got["opt"] == want["ub"]
    assert bool(got["proven"]) == want["proven"]
    assert got["nodes_bounded"] == want["nodes_bounded"]
    assert got["steps"] == want["steps"]
    assert got["improvements"] == want["improvements"]
    assert got["max_stack"] == want["max_stack"]
    assert (got["perm"] == want["incumbent"]).all()
    assert (got["steplog"] == want["steplog"]).all()
    return got


@pytest.mark.parametrize("n,m,seed", [(6, 3, 11), (8, 4, 12), (9, 5, 13), (10, 3, 14)])
@pytest.mark.parametrize("pool_cap", [1, 3, 16, 1 << 20])
@pytest.mark.parametrize("ub_mode", ["neh", "none"])
def test_solve_small_matches_oracle(n, m, seed, pool_cap, ub_mode):
    require_gpu()
    p = inst_times(n, m, seed)
    got = compare_solve(p, ub_mode, pool_cap)
    assert got["proven"]
    if n <= 8:
        assert got["opt"] == oracle.brute(p)


@pytest.mark.parametrize("n,m,seed,pool_cap,budget", [(20, 5, 21, 256, 200000), (15, 8, 22, 64, 50000),
                                                      (20, 10, 23, 4096, 60000), (50, 10, 24, 2048, 20000)])
def test_solve_medium_matches_oracle(n, m, seed, pool_cap, budget):
    require_gpu()
    p = inst_times(n, m, seed)
    compare_solve(p, "neh", pool_cap, budget)


def test_solve_200x20_first_steps_match_oracle():
    """The 200 x 20 configuration from NEH, four pool steps of 1024 children."""
    require_gpu()
    p = gen.processing_times(200, 20, gen.make_seed(2, 0, gen.PURPOSE_TIMES))
    compare_solve(p, "neh", 1024, budget=1 + 3 * 1024)


def test_solve_root_pruned_and_budget():
    require_gpu()
    p = inst_times(10, 5, 31)
    lb0 = oracle.bound(p, [])
    with fspbb.create_instance(p) as inst:
        r = fspbb.solve(inst, lb0, 16, 1 << 40)
        assert r["proven"] and r["nodes_bounded"] == 1 and r["steps"] == 0 and r["opt"] == lb0
        assert (r["perm"] == -1).all()
        r = fspbb.solve(inst, fspbb.UB_NONE, 4, 30)
        assert r["status"] == fspbb.BUDGET and not r["proven"] and r["nodes_bounded"] >= 30


def test_release_cached_returns_memory_and_keeps_results():
    """Scratch kept for reuse goes back to the driver, and searches after it
    give the same results."""
    torch = require_gpu()
    p = gen.processing_times(200, 20, gen.make_seed(2, 0, gen.PURPOSE_TIMES))
    with fspbb.create_instance(p) as inst:
        a = fspbb.solve(inst, fspbb.UB_NEH, 262144, 1 + 2 * 262144)  # keeps a 1.6 GB stack among others
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        fspbb.release_cached()
        free1, _ = torch.cuda.mem_get_info()
        b = fspbb.solve(inst, fspbb.UB_NEH, 262144, 1 + 2 * 262144)
        fspbb.release_cached()
    assert free1 >= free0 + (1 << 30)
    for f in ("opt", "nodes_bounded", "steps", "improvements", "max_stack", "status"):
        assert a[f] == b[f], f


# --- the benchmarked search: 200 x 20 from NEH with 262,144-child pools --------

def test_solve_200x20_neh_benchmarked_pool_cap():
    """The benchmarked search (the 200 x 20 instance of the bound pool, NEH
    upper bound, pool_cap 262,144) for three steps (1 + 200 + 39,800 +
    261,954 nodes).  tests/golden/make_bnb_200x20.py built these steps on the
    host with every child bounded by the oracle.  Every step-log entry
    (parents, children, UB, pushed, stack, fingerprint) must equal it.  The
    third step is then run alone through fsp_branch_and_prune on the same
    parents and upper bound: the survivors in order (rows, depths, bounds)
    must hash to the oracle's, and a sample of them is compared one by one."""
    torch = require_gpu()
    g = load_golden("bnb_200x20_neh_cap262144.json")
    n, cap = g["n"], g["pool_cap"]
    p = gen.processing_times(n, g["m"], gen.make_seed(*g["seed"]))
    steps = g["steps"]
    with fspbb.create_instance(p) as inst:
        budget = steps[1]["nodes_after"] + 1  # the search stops after its third step
        got = fspbb.solve(inst, fspbb.UB_NEH, cap, budget, steplog_cap=8)
        assert got["ub0"] == g["neh"]
        assert got["steps"] == 3 and got["nodes_bounded"] == steps[2]["nodes_after"]
        for k in range(3):
            assert got["steplog"][k].tolist() == steps[k]["log"], k
        last = steps[2]
        pre = np.zeros((len(last["parents"]), n), np.int32)
        pre[:, :last["parents_depth"]] = np.array(last["parents"], np.int32)
        dep = np.full(len(pre), last["parents_depth"], np.int32)
        pre_d, dep_d = to_dev(torch, pre, dep)
        nch = last["log"][1]
        rows = torch.full((nch, n), -9, dtype=torch.int32, device="cuda")
        cdep = torch.full((nch,), -9, dtype=torch.int32, device="cuda")
        clb = torch.full((nch,), -9, dtype=torch.int32, device="cuda")
        res = fspbb.branch_and_prune(inst, pre_d, dep_d, last["ub_in"], rows, cdep, clb)
        torch.cuda.synchronize()
    assert res["status"] == fspbb.OK
    S = last["log"][3]
    assert (res["n_children"], res["n_survivors"], res["ub_out"], res["fingerprint"]) == \
        (nch, S, last["log"][2], last["log"][5])
    d = last["parents_depth"] + 1
    rows, cdep, clb = rows[:S, :d].cpu().numpy(), cdep[:S].cpu().numpy(), clb[:S].cpu().numpy()
    for row in last["survivor_sample"]:
        i = row[0]
        assert rows[i].tolist() == row[1:1 + d] and cdep[i] == d and clb[i] == row[-1], i
    assert survivors_digest(rows, cdep, clb) == last["survivors_sha256"]
