"""The paper's per-vertex schedule (comparison variant): its prime paths per
end vertex equal the oracle's, its per-round path counts equal the oracle's
per-level counts, and inside a group the paths come by length."""
import numpy as np
import pytest

import oracle
from paper_2210_16998_amd import cfggen, tpg
from tests.gpu_util import say, ws

pytestmark = pytest.mark.gpu


def _groups(pl):
    out = {}
    for p in pl.tolist():
        out.setdefault(p[-1], []).append(p)
    return out


def _check(g, load_flags=0):
    h = tpg.load_cfg(g, load_flags)
    got, st = tpg.prime_paths_vertex_lists(h, ws=ws())
    ref, _, _, _ = oracle.prime_paths(g)
    lasts = [p[-1] for p in got.tolist()]
    assert lasts == sorted(lasts)  # grouped by last vertex, ascending
    gg, rg = _groups(got), _groups(ref)
    assert sorted(gg) == sorted(rg)
    for v, paths in gg.items():
        lens = [len(p) for p in paths]
        assert lens == sorted(lens), v
        assert sorted(paths) == sorted(rg[v]), v
    _, rl, rc = oracle.count(g)
    assert st["n_extensions"] == sum(rl[L] + rc[L] for L in range(2, len(rl)))
    assert st["n_pp"] == len(ref)
    return st


def test_fig1():
    say("case vertex lists fig1")
    st = _check(cfggen.fig1_cfg())
    assert st["n_pp"] == 19


@pytest.mark.parametrize("seed", range(3))
def test_c1(seed):
    say("case vertex lists c1", seed)
    _check(cfggen.c1_cfg(seed))


def test_random_cfgs():
    for s in range(80):
        n = 2 + s % 30
        g = cfggen.random_small_cfg(64_000 + s, n, extra=1 + s % 9)
        if s % 20 == 0:
            say("case vertex lists random cfg", s, n)
        _check(g)


def test_random_digraphs():
    """Self-loops, isolated vertices (a one-entry prime path), dense graphs."""
    for s in range(120):
        n = 1 + s % 11
        g = cfggen.random_digraph(65_000 + s, n, 0.1 + 0.08 * (s % 7))
        if s % 30 == 0:
            say("case vertex lists random digraph", s, n)
        _check(g, tpg.TPG_LOAD_ANY_DIGRAPH)


def test_streaming_is_rejected():
    h = tpg.load_cfg(cfggen.fig1_cfg())
    with pytest.raises(tpg.TpgError) as ei:
        tpg.prime_paths_vertex_lists(h, ws=ws(), flags=tpg.TPG_TP_GREEDY)
    assert ei.value.name == "TPG_ERR_INVALID_ARG"


@pytest.mark.parametrize("k", [5, 9])
def test_loop_diamond_chain_closed_form_and_path_tree(k):
    """A while loop around k diamonds: (3k + 4) 2^k + 1 prime paths (closed
    form derived for the oracle's pins), per end vertex the same as the
    path-tree engine's grouped output."""
    g = cfggen.loop_diamond_chain(k)
    say("case vertex lists loop-diamond", k)
    h = tpg.load_cfg(g)
    got, st = tpg.prime_paths_vertex_lists(h, ws=ws())
    tree, st2 = tpg.prime_paths(h, ws=ws(), flags=tpg.TPG_ORDER_BY_LAST)
    assert st["n_pp"] == st2["n_pp"] == (3 * k + 4) * 2 ** k + 1
    assert st["n_extensions"] == st2["n_extensions"]
    go, gv = np.asarray(got.offsets), np.asarray(got.vertices)
    to, tv = np.asarray(tree.offsets), np.asarray(tree.vertices)
    assert np.array_equal(gv[go[1:] - 1], tv[to[1:] - 1])  # same group sizes, in order
    assert sorted(got.tolist()) == sorted(tree.tolist())
