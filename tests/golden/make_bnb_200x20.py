"""Writes bnb_200x20_neh_cap262144.json: the first three pool steps of the
depth-first search on the 200 x 20 bound-pool instance from its NEH upper
bound with pools of 262,144 children, every child bounded by the oracle.
Calls only the oracle and the seeded generator (through tests/helpers.py);
it takes a few minutes on 8 host threads.  Rerun it only when the oracle's
arithmetic or order rules are changed on purpose (and say why in the commit).

    python tests/golden/make_bnb_200x20.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from helpers import host_dfs_steps, survivors_digest  # noqa: E402
from paper_1208_3933_amd import gen  # noqa: E402

N_JOBS, N_MACHINES, POOL_CAP, STEPS = 200, 20, 262144, 3


def main():
    p = gen.processing_times(N_JOBS, N_MACHINES, gen.make_seed(2, 0, gen.PURPOSE_TIMES))
    ms, perm = oracle.neh(p)
    steps = host_dfs_steps(p, ms, POOL_CAP, STEPS)
    out = {"n": N_JOBS, "m": N_MACHINES, "seed": [2, 0, gen.PURPOSE_TIMES], "pool_cap": POOL_CAP,
           "neh": int(ms), "steps": []}
    for s in steps:
        pre, dep = s["parents"]
        rows, sdep, lbs = s["survivors"]
        d = int(dep.max())
        sample = list(range(0, len(sdep), max(1, len(sdep) // 64)))
        out["steps"].append({
            "log": [int(x) for x in s["log"]], "nodes_after": int(s["nodes"]), "ub_in": int(s["ub_in"]),
            "parents_depth": d, "parents": [[int(x) for x in r[:d]] for r in pre] if d <= 2 else None,
            "survivors_sha256": survivors_digest(rows, sdep, lbs),
            "survivor_sample": [[i] + [int(x) for x in rows[i, :int(sdep[i])]] + [int(lbs[i])] for i in sample]})
    with open(os.path.join(HERE, "bnb_200x20_neh_cap262144.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))
        f.write("\n")


if __name__ == "__main__":
    main()
