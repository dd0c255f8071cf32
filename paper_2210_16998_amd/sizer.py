"""Learned sizing for the batched form: data set, training and prediction.

Labels come from exact runs of the batched engine itself: per graph, the
number of simple paths with L entries (L = 1..64, deeper levels pooled into
64) and the prime-path count, as log1p.  Features are the library's 32
structural features.  The network is trained on the GPU by the library's
own forward / backward / Adam kernels.

    python -m paper_2210_16998_amd.sizer --train 100000 --out <file>
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import time
from typing import List, Optional, Tuple

import numpy as np

from . import cfggen, tpg

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = os.path.join(HERE, "models", "sizer.tpgmlp")


def _gen(seeds: List[int]):
    return [cfggen.batch_member_cfg(s) for s in seeds]


def generate(seeds: List[int], workers: int = 16) -> List[cfggen.CFG]:
    """CFGs of the batched workload's distribution, generated in parallel."""
    if workers <= 1 or len(seeds) < 2000:
        return _gen(seeds)
    chunks = [seeds[i:i + 2000] for i in range(0, len(seeds), 2000)]
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        out = []
        for part in ex.map(_gen, chunks):
            out.extend(part)
    return out


def labels(graphs: List[tpg.Graph], ws: tpg.Workspace, chunk: int = 4096) -> np.ndarray:
    """[n, 65] log1p targets from exact batched runs."""
    T = np.zeros((len(graphs), 65), np.float32)
    for a in range(0, len(graphs), chunk):
        part = graphs[a:a + chunk]
        lv = np.zeros((len(part), 64), np.int64)
        res, _ = tpg.batch_test_paths(part, ws=ws, level_counts=lv,
                                      flags=tpg.TPG_NO_TIMING)
        T[a:a + len(part), :64] = np.log1p(lv)
        T[a:a + len(part), 64] = np.log1p(np.diff(res.pp_first))
    return T


def train(X: np.ndarray, T: np.ndarray, epochs: int = 40, lr: float = 2e-3, batch: int = 1024,
          seed: int = 0, log=None) -> tpg.MLP:
    m = tpg.MLP(seed=seed)
    mean = X.mean(0).astype(np.float32)
    std = (X.std(0) + 1e-6).astype(np.float32)
    m.set_normalizer(mean, std)
    rng = np.random.default_rng(seed)
    n = len(X)
    steps = 0
    for ep in range(epochs):
        perm = rng.permutation(n)
        lr_ep = lr * (0.5 * (1 + np.cos(np.pi * ep / epochs)))
        tot = 0.0
        for b in range(0, n - batch + 1, batch):
            idx = perm[b:b + batch]
            tot += m.train_step(X[idx], T[idx], lr_ep)
            steps += 1
        if log:
            log(f"epoch {ep} loss {tot / max(1, n // batch):.4f}")
    return m


def predict(m: tpg.MLP, graphs: List[tpg.Graph]) -> np.ndarray:
    return m.forward(tpg.features(graphs))


def allocation_ratios(pred: np.ndarray, T: np.ndarray) -> dict:
    """Over-allocation = predicted / actual paths (with the engine's 25%
    margin), under-allocation = share of graphs whose prediction with margin
    falls short of their actual paths."""
    p = np.expm1(np.clip(pred[:, :64], 0, 40)).sum(1) * 1.25
    a = np.expm1(T[:, :64]).sum(1)
    return {"over_allocation": float(p.sum() / a.sum()),
            "under_allocated_graphs": float(np.mean(p < a)),
            "rmse_log": float(np.sqrt(np.mean((pred - T) ** 2)))}


def main(argv: Optional[List[str]] = None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=100_000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--out", default=DEFAULT_MODEL)
    ap.add_argument("--report", default=None)
    args = ap.parse_args(argv)
    t0 = time.time()
    seeds = [cfggen.C4_SEED_BASE + i for i in range(args.train)]
    cfgs = generate(seeds)
    print(f"generated {len(cfgs)} CFGs in {time.time() - t0:.1f}s", flush=True)
    graphs = [tpg.load_cfg(g) for g in cfgs]
    ws = tpg.Workspace()
    t1 = time.time()
    X = tpg.features(graphs)
    T = labels(graphs, ws)
    print(f"features + exact labels in {time.time() - t1:.1f}s", flush=True)
    n_tr = int(0.9 * len(X))
    t2 = time.time()
    m = train(X[:n_tr], T[:n_tr], epochs=args.epochs, log=lambda s: print(s, flush=True))
    print(f"trained in {time.time() - t2:.1f}s", flush=True)
    val = allocation_ratios(m.forward(X[n_tr:]), T[n_tr:])
    c3 = [tpg.load_cfg(g) for g in cfggen.c3_batch(4096)]
    c3_T = labels(c3, ws)
    c3_r = allocation_ratios(predict(m, c3), c3_T)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    m.save(args.out)
    rep = {"train_graphs": n_tr, "val_graphs": len(X) - n_tr, "val": val, "batch_4096": c3_r,
           "epochs": args.epochs}
    print(json.dumps(rep), flush=True)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
