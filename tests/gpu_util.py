"""Helpers of the GPU parity tests: run the HIP path, run the oracle,
compare element by element."""
import sys

import numpy as np

import oracle
from paper_2210_16998_amd import tpg

_WS = None


def ws():
    global _WS
    if _WS is None:
        _WS = tpg.Workspace()
    return _WS


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same(gpu, ref) -> bool:
    return (np.array_equal(np.asarray(gpu.offsets), np.asarray(ref.offsets))
            and np.array_equal(np.asarray(gpu.vertices), np.asarray(ref.vertices)))


def first_diff(gpu, ref) -> str:
    a, b = gpu.tolist(), ref.tolist()
    if len(a) != len(b):
        sa, sb = set(map(tuple, a)), set(map(tuple, b))
        return (f"count {len(a)} vs {len(b)}; missing {sorted(sb - sa)[:3]} "
                f"extra {sorted(sa - sb)[:3]}")
    for i, (x, y) in enumerate(zip(a, b)):
        if x != y:
            return f"index {i}: gpu {x} oracle {y}"
    return "equal"


_REF = {}


def ref_pp(g, local=False):
    """Oracle prime paths (prune pass; or the local-rule DFS for the large
    workloads, where the prune pass's sort of every candidate takes minutes -
    the two are pinned equal by the CPU tests)."""
    key = ("pp", g.name, g.n, g.n_edges, g.col_idx.tobytes())
    if key not in _REF:
        if local:
            pl, st = oracle.prime_paths_local(g, 0, g.n)
            st = dict(st)
            _REF[key] = (pl, st, None, None)
        else:
            _REF[key] = oracle.prime_paths(g)
    return _REF[key]


def ref_tp(g):
    key = ("tp", g.name, g.n, g.n_edges, g.col_idx.tobytes())
    if key not in _REF:
        _REF[key] = oracle.test_paths(g, ref_pp(g)[0])
    return _REF[key]


def check_pp(g, flags=0, load_flags=0, w=None, local=False):
    h = tpg.load_cfg(g, load_flags)
    pp, st = tpg.prime_paths(h, ws=w or ws(), flags=flags)
    ref, rst, lv, cy = ref_pp(g, local)
    assert same(pp, ref), f"{g.name}: {first_diff(pp, ref)}"
    assert st["n_pp"] == rst["n_pp"]
    assert st["n_extensions"] == rst["n_extensions"], (g.name, st["n_extensions"], rst["n_extensions"])
    assert st["n_cycles"] == rst["n_cycles"]
    return pp, st, ref


def check_tp(g, flags=0, w=None, local=False):
    h = tpg.load_cfg(g)
    pp, tp, st = tpg.test_paths(h, ws=w or ws(), flags=flags)
    rpp, rst = ref_pp(g, local)[:2]
    assert st["n_extensions"] == rst["n_extensions"] and st["n_cycles"] == rst["n_cycles"]
    rtp, nb = ref_tp(g)
    assert same(pp, rpp), f"{g.name} PP: {first_diff(pp, rpp)}"
    assert same(tp, rtp), f"{g.name} TP: {first_diff(tp, rtp)}"
    assert st["n_tp_spliced"] == nb and st["n_tp"] == len(rtp)
    return pp, tp, st
