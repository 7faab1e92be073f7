"""Writes oracle_regression.json: bounds and B&B results of the oracle on small
seeded cases.  Calls only the oracle and the seeded generator; rerun it only
when the oracle's arithmetic is changed on purpose (and say why in the commit).

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1208_3933_amd import gen  # noqa: E402

CASES = [(20, 5, 0), (20, 10, 1), (50, 10, 2), (20, 20, 3)]


def main():
    out = {"bounds": [], "bnb": []}
    for n, m, i in CASES:
        p = gen.processing_times(n, m, gen.make_seed(80, i, 0))
        pre, dep = gen.random_pool(n, 16, gen.make_seed(80, i, 1))
        lb = oracle.bound_pool(p, pre, dep)
        out["bounds"].append({"n": n, "m": m, "instance": i, "count": 16,
                              "lb": [int(x) for x in lb]})
    for n, m, i in [(10, 5, 10), (12, 4, 11)]:
        p = gen.processing_times(n, m, gen.make_seed(80, i, 0))
        ms, perm = oracle.neh(p)
        r = oracle.bnb(p, ms, perm, pool_cap=64)
        out["bnb"].append({"n": n, "m": m, "instance": i, "pool_cap": 64, "neh": ms,
                           "ub": r["ub"], "nodes_bounded": r["nodes_bounded"],
                           "steps": r["steps"], "proven": r["proven"],
                           "incumbent": [int(x) for x in r["incumbent"]]})
    with open(os.path.join(HERE, "oracle_regression.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
