"""Test paths by longest-first covering on the GPU (TPG_TP_GREEDY) against
the CPU oracle's plain greedy: exact on graphs where the oracle finishes in
seconds, properties on the ~200-vertex CFGs."""
import numpy as np
import pytest

import oracle
from paper_2210_16998_amd import cfggen, tpg
from tests.goldens import workloads
from tests.gpu_util import ref_pp, say, same

pytestmark = pytest.mark.gpu


def _check(g, w):
    h = tpg.load_cfg(g)
    pp, tp, st = tpg.test_paths(h, ws=w, flags=tpg.TPG_TP_GREEDY)
    rp = oracle.prime_paths(g)[0]
    assert same(pp, rp), g.name
    rt = oracle.test_paths_greedy(g, rp)
    assert same(tp, rt), g.name
    assert st["n_tp"] == len(rt) and st["n_tp_spliced"] == len(rp)


def test_greedy_small_graphs():
    w = tpg.Workspace()
    gs = [cfggen.fig1_cfg(), cfggen.from_edges(1, [], 0, 0)] + [cfggen.c1_cfg(s) for s in range(4)]
    gs += [cfggen.random_small_cfg(50_000 + s, 2 + s % 30, extra=1 + s % 9) for s in range(120)]
    gs += [cfggen.batch_member_cfg(cfggen.C3_SEED_BASE + s) for s in range(150)]
    for k, g in enumerate(gs):
        if k % 50 == 0:
            say("case greedy small", k, g.name)
        _check(g, w)
    w.close()


@pytest.mark.parametrize("seed", [216, 357, 84])
def test_greedy_mid_size_batch_members(seed):
    w = tpg.Workspace()
    g = cfggen.batch_member_cfg(cfggen.C3_SEED_BASE + seed)
    say("case greedy mid", seed, g.n)
    _check(g, w)
    w.close()


def test_greedy_c2_properties():
    rec = workloads()["c2"][0]
    g = cfggen.c2_cfg(rec["seed"])
    h = tpg.load_cfg(g)
    w = tpg.Workspace()
    say("case greedy c2", rec["seed"])
    _, full, _ = tpg.test_paths(h, ws=w)
    pp, tp, st = tpg.test_paths(h, ws=w, flags=tpg.TPG_TP_GREEDY)
    assert same(pp, ref_pp(g, local=True)[0])
    rows = tp.tolist()
    full_rows = set(map(tuple, full.tolist()))
    # canonical, unique, a subset of the spliced test paths, no more of them
    assert rows == sorted(rows) and len(set(map(tuple, rows))) == len(rows)
    assert set(map(tuple, rows)) <= full_rows and len(rows) <= len(full_rows)
    # the same bytes again (the rounds and atomics do not change the result)
    _, tp2, _ = tpg.test_paths(h, ws=w, flags=tpg.TPG_TP_GREEDY)
    assert np.array_equal(tp2.vertices, tp.vertices) and np.array_equal(tp2.offsets, tp.offsets)
    w.close()
