"""Writes tests/golden/stress_sets.json: whole-set figures of the 400-vertex
stress CFG, all computed by the CPU oracle (orc_set_digests):

* the number of prime paths of every first vertex;
* the prime-path set digest (sum mod 2^64 and xor of the per-path FNV-1a 64
  hashes);
* the number of test paths after exact deduplication, the number spliced
  before it, and the test-path set digest.

The sets themselves (2.3e7 prime paths, 8.8e8 entries) are too large to keep
as fixtures; the GPU tests compare their own digests and counts with these.

  python -m oracle.stress_digests [--buckets 4]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle  # noqa: E402
from paper_2210_16998_amd import cfggen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "tests", "golden", "stress_sets.json")


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--buckets", type=int, default=4)
    args = ap.parse_args()
    g = cfggen.c5_cfg()
    t0 = time.time()
    d = oracle.set_digests(g, n_buckets=args.buckets)
    out = {"graph": "stress CFG (cfggen.c5_cfg)", "n": g.n, "edges": g.n_edges,
           "n_pp": d["n_pp"], "pp_digest": [str(x) for x in d["pp_digest"]],
           "pp_per_start": [int(x) for x in d["pp_per_start"]],
           "n_tp": d["n_tp"], "n_spliced": d["n_spliced"],
           "tp_digest": [str(x) for x in d["tp_digest"]],
           "seconds": round(time.time() - t0, 1), "buckets": args.buckets}
    with open(OUT, "w") as f:  # one key per line, lists inline
        f.write("{\n" + ",\n".join(f" {json.dumps(k)}: {json.dumps(v)}" for k, v in out.items())
                + "\n}\n")
    print("wrote", OUT, out["n_pp"], out["n_tp"], out["seconds"], "s")


if __name__ == "__main__":
    main()
