"""Writes tests/golden/workloads.json: the accepted seeds and the exact
counts of the synthetic workloads, all computed by the CPU oracle.

  python -m oracle.calibrate

Single ~200-vertex CFG: the first 8 seeds in [0, 2000) whose graph lies in
the shape window (V 180..220, cyclomatic 36..44) and has between 1e5 and 1e6
prime paths.  The stress CFG and the 20-vertex CFG are fixed layouts; their
counts are recorded too.
"""
from __future__ import annotations

import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle  # noqa: E402
from paper_2210_16998_amd import cfggen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "tests", "golden", "workloads.json")


def _counts(g, cap=0):
    st, lv, cy = oracle.count(g, ext_cap=cap)
    if st is None:
        return None
    last = max([L for L in range(len(lv)) if lv[L] or cy[L]] or [0])
    return {"n": g.n, "edges": g.n_edges, "cyclomatic": g.cyclomatic,
            "n_pp": st["n_pp"], "n_extensions": st["n_extensions"],
            "n_cycles": st["n_cycles"], "levels": [int(x) for x in lv[1:last + 1]],
            "cycles_by_len": [int(x) for x in cy[1:last + 1]]}


def main() -> None:
    res = {"generator": "paper_2210_16998_amd.cfggen", "c2": [], "c1": None, "c5": None}
    res["c1"] = _counts(cfggen.c1_cfg(0))
    for s in range(2000):
        g = cfggen.c2_cfg(s)
        if not cfggen.c2_shape_ok(g):
            continue
        c = _counts(g, cap=int(2e8))
        if c is None or not (1e5 <= c["n_pp"] <= 1e6):
            continue
        c["seed"] = s
        res["c2"].append(c)
        print("c2 accept", s, c["n"], c["cyclomatic"], c["n_pp"], c["n_extensions"], flush=True)
        if len(res["c2"]) == 8:
            break
    c5 = cfggen.c5_cfg()
    res["c5"] = _counts(c5)
    res["c5"]["layout"] = {"per_arm": 3, "chain": [1, 1, 1], "tail": 9, "pad_to": 400}
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
