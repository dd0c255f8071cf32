"""Autotuner cache: the extension kernel's launch shape per visited-set
width, measured by tpg_autotune on a representative batch and stored as
JSON keyed by the GPU architecture.

    python -m paper_2210_16998_amd.tuning --out <file>   (tunes on the batched workload)
"""
from __future__ import annotations

import argparse
import json
import os
from typing import Dict, Optional

from . import cfggen, tpg

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "models", "tuning.json")


def arch_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return f"{getattr(p, 'gcnArchName', p.name)}:{p.multi_processor_count}cu"


def load(ws: tpg.Workspace, path: str = DEFAULT_CACHE) -> Optional[Dict]:
    """Applies the cached shape for this GPU to `ws`, if there is one."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        cache = json.load(f)
    t = cache.get(arch_key())
    if t:
        tpg.set_tuning(ws, t)
    return t


def tune_and_save(ws: tpg.Workspace, graphs, path: str = DEFAULT_CACHE) -> Dict:
    t = tpg.autotune(graphs, ws)
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    cache[arch_key()] = t
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(cache, f, indent=1)
    return t


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--graphs", type=int, default=4096)
    a = ap.parse_args()
    graphs = [tpg.load_cfg(g) for g in cfggen.c3_batch(a.graphs)]
    graphs += [tpg.load_cfg(cfggen.c2_cfg(9))]
    ws = tpg.Workspace()
    print(json.dumps(tune_and_save(ws, graphs, a.out)), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
