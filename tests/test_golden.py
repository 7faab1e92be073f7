"""The oracle still reproduces its committed regression fixture
(tests/golden/oracle_regression.json, written by tests/golden/make_golden.py
from the oracle alone)."""
import json
import os

import oracle
from paper_1208_3933_amd import gen

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_oracle_regression_fixture():
    with open(os.path.join(HERE, "oracle_regression.json")) as f:
        g = json.load(f)
    for case in g["bounds"]:
        n, m, i = case["n"], case["m"], case["instance"]
        p = gen.processing_times(n, m, gen.make_seed(80, i, 0))
        pre, dep = gen.random_pool(n, case["count"], gen.make_seed(80, i, 1))
        assert [int(x) for x in oracle.bound_pool(p, pre, dep)] == case["lb"]
    for case in g["bnb"]:
        n, m, i = case["n"], case["m"], case["instance"]
        p = gen.processing_times(n, m, gen.make_seed(80, i, 0))
        ms, perm = oracle.neh(p)
        assert ms == case["neh"]
        r = oracle.bnb(p, ms, perm, pool_cap=case["pool_cap"])
        assert (r["ub"], r["nodes_bounded"], r["steps"], r["proven"]) == \
            (case["ub"], case["nodes_bounded"], case["steps"], case["proven"])
        assert [int(x) for x in r["incumbent"]] == case["incumbent"]
