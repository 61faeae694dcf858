"""Writes the stored expected values under tests/golden/ by calling only the
FP64 oracle (oracle/) on seeded generator inputs (gen/).

maxcut_er2000_solve.json: ALM-BM solve of the MaxCut SDP (Sec. 6.1 form, C = -L/4,
X_ii = 1) on the Erdos-Renyi graph n = 2000, M = 10000 (average degree 10),
unit weights, seed 1; starting factor rank 8 (gen.init_factor seed 1), y0 = 0,
sigma = 1, exact line search, p = 1 rank adaptation, stop at relative KKT 1e-6
(Sec. 6 measure).  Run: python tests/golden/make_golden.py
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gen  # noqa: E402
import oracle  # noqa: E402


def maxcut_er2000():
    g = gen.er_graph(2000, 10000, 1, "unit")
    p = oracle.maxcut_sdp(g)
    R0 = gen.init_factor(2000, 8, 1)
    out = oracle.solve(p, R0, opts=oracle.SolveOptions(eps_kkt=1e-6, sigma=1.0, r_max=64))
    k = out["kkt"]
    return {
        "workload": "MaxCut SDP, ER n=2000 M=10000 unit weights seed 1, r0=8, sigma=1, eps=1e-6",
        "status": out["status"], "outer": len(out["history"]), "rank": int(out["R"].shape[1]),
        "pobj": k["pobj"], "dobj": k["dobj"], "pinf": k["pinf"], "dinf": k["dinf"], "gap": k["gap"],
        "kkt": k["kkt"], "sdp_value": -k["pobj"],
    }


if __name__ == "__main__":
    res = maxcut_er2000()
    with open(os.path.join(HERE, "maxcut_er2000_solve.json"), "w") as fh:
        json.dump(res, fh, indent=1)
    print(res)
