"""The paper's input and output form on the GPU, against the CPU oracle:
switch vertices binarized at load (out-degree <= 2), and prime paths grouped
by their last vertex."""
import numpy as np
import pytest

import oracle
from paper_2210_16998_amd import cfggen, tpg
from tests.goldens import workloads
from tests.gpu_util import say, same

pytestmark = pytest.mark.gpu


def _graphs():
    gs = [cfggen.fig1_cfg(), cfggen.c1_cfg(0)]
    gs += [cfggen.random_small_cfg(60_000 + s, 6 + s % 30, extra=2 + s % 6) for s in range(30)]
    return gs


def test_binarized_prime_and_test_paths():
    w = tpg.Workspace()
    for g in _graphs() + [cfggen.c2_cfg(workloads()["c2"][k]["seed"]) for k in (0, 1)]:
        b = oracle.binarize(g)
        say("case binarized", g.name, g.n, "->", b.n)
        h = tpg.load_cfg(g, tpg.TPG_LOAD_BINARIZE)
        pp, tp, st = tpg.test_paths(h, ws=w)
        if b.n > 100:
            rp = oracle.prime_paths_local(b, 0, b.n)[0]
        else:
            rp = oracle.prime_paths(b)[0]
        rt = oracle.test_paths(b, rp)[0]
        assert same(pp, rp), g.name
        assert same(tp, rt), g.name
    w.close()


def test_prime_paths_grouped_by_last_vertex():
    w = tpg.Workspace()
    for g in _graphs() + [cfggen.c2_cfg(workloads()["c2"][2]["seed"])]:
        say("case by last", g.name)
        h = tpg.load_cfg(g)
        rp = oracle.prime_paths_local(g, 0, g.n)[0] if g.n > 100 else oracle.prime_paths(g)[0]
        ref = oracle.group_by_last(rp)
        got, _ = tpg.prime_paths(h, ws=w, flags=tpg.TPG_ORDER_BY_LAST | tpg.TPG_DIGEST)
        assert same(got, ref), g.name
        assert got.digest == oracle.digest(rp)
        pp, tp, _ = tpg.test_paths(h, ws=w, flags=tpg.TPG_ORDER_BY_LAST)
        assert same(pp, ref)
        assert same(tp, oracle.test_paths(g, rp)[0])
    # not streamable by first vertex
    with pytest.raises(tpg.TpgError):
        tpg.prime_paths_stream(tpg.load_cfg(cfggen.c1_cfg(0)), lambda c, f, e: None, ws=w,
                               flags=tpg.TPG_ORDER_BY_LAST)
    w.close()


def test_binarized_and_grouped_together():
    w = tpg.Workspace()
    g = cfggen.c2_cfg(workloads()["c2"][3]["seed"])
    b = oracle.binarize(g)
    say("case binarized + by last", b.n)
    h = tpg.load_cfg(g, tpg.TPG_LOAD_BINARIZE)
    got, _ = tpg.prime_paths(h, ws=w, flags=tpg.TPG_ORDER_BY_LAST)
    assert same(got, oracle.group_by_last(oracle.prime_paths_local(b, 0, b.n)[0]))
    w.close()
