"""GPU parity of the strongly connected components (Sec. 2, Defs. 3-5) and
of the prime-path types (Defs. 2, 9, 10, 11): labels, flags and types are
integers, compared exactly with the oracle."""
import numpy as np
import pytest

import oracle
from paper_2210_16998_amd import cfggen, tpg
from tests.gpu_util import say, ws
from tests.goldens import workloads

pytestmark = pytest.mark.gpu


def _check_scc(g, load_flags=0):
    h = tpg.load_cfg(g, load_flags)
    comp, fl, nc = tpg.scc(h, ws=ws())
    want = oracle.scc(g)
    assert np.array_equal(comp, want)
    assert np.array_equal(fl, oracle.scc_flags(g, want))
    assert nc == len(set(want.tolist()))
    return h


def _check_types(g, load_flags=0):
    h = _check_scc(g, load_flags)
    pp, _ = tpg.prime_paths(h, ws=ws())
    ref, _, _, _ = oracle.prime_paths(g)
    types, counts = tpg.prime_path_types(h, pp, ws=ws())
    want_t, want_c = oracle.pp_types(g, ref)
    assert np.array_equal(types, want_t)
    assert np.array_equal(counts, want_c)
    return types, counts


def test_fig1_components_and_types_match_the_paper():
    say("case fig1 scc + types")
    g = cfggen.fig1_cfg()
    comp, fl, nc = tpg.scc(tpg.load_cfg(g), ws=ws())
    assert sorted(np.nonzero(comp == 2)[0].tolist()) == [2, 3, 4, 5, 6, 8] and nc == 6
    _, counts = _check_types(g)
    assert counts.tolist() == [0, 2, 11, 4, 2, 0]  # Sec. 2.1: 2 complete, 11 + 4 + 2


@pytest.mark.parametrize("seed", range(4))
def test_c1_layouts(seed):
    say("case c1 scc + types", seed)
    _check_types(cfggen.c1_cfg(seed))


def test_random_cfgs():
    for s in range(120):
        n = 2 + s % 40
        g = cfggen.random_small_cfg(61_000 + s, n, extra=1 + s % 9)
        if s % 20 == 0:
            say("case random cfg scc + types", s, n)
        _check_types(g)


def test_random_digraphs_components():
    """Arbitrary digraphs: self-loops, several components with cycles, arcs
    between them, isolated vertices."""
    for s in range(150):
        n = 1 + s % 17
        g = cfggen.random_digraph(62_000 + s, n, 0.05 + 0.04 * (s % 6))
        if s % 30 == 0:
            say("case random digraph scc", s, n)
        _check_types(g, tpg.TPG_LOAD_ANY_DIGRAPH)


def test_wide_graphs_components():
    for n in (300, 1500, 4096):
        say("case wide scc", n)
        _check_scc(cfggen.random_small_cfg(63_000 + n, n, extra=6))


def test_device_and_host_sets_agree():
    say("case types of a device-resident set")
    g = cfggen.c1_cfg(1)
    h = tpg.load_cfg(g)
    hp, _ = tpg.prime_paths(h, ws=ws())
    t_host, c_host = tpg.prime_path_types(h, hp, ws=ws())
    dp, _ = tpg.prime_paths(h, ws=ws(), flags=tpg.TPG_OUT_DEVICE)
    t_dev, c_dev = tpg.prime_path_types(h, dp, ws=ws())
    assert np.array_equal(t_host, t_dev) and np.array_equal(c_host, c_dev)


def test_malformed_host_sets_are_rejected():
    g = cfggen.fig1_cfg()
    h = tpg.load_cfg(g)

    class P:
        pass
    bad = P()
    bad.offsets = np.array([0, 2, 2], np.int64)  # an empty path
    bad.vertices = np.array([0, 1], np.int32)
    with pytest.raises(tpg.TpgError) as ei:
        tpg.prime_path_types(h, bad, ws=ws())
    assert ei.value.name == "TPG_ERR_INVALID_ARG"
    bad.offsets = np.array([0, 2], np.int64)
    bad.vertices = np.array([0, 99], np.int32)  # outside the graph
    with pytest.raises(tpg.TpgError):
        tpg.prime_path_types(h, bad, ws=ws())


def _scc_subgraph_internal(g, h, comp, fl):
    """Internal prime paths from the extension run on each component with a
    cycle taken alone (Sec. 2.1), filtered by Def. 9: the per-SCC route."""
    out = []
    for c in sorted(set(comp.tolist())):
        vs = [int(v) for v in np.nonzero(comp == c)[0]]
        if not fl[vs[0]] & tpg.TPG_SCC_CYCLIC:
            continue
        loc = {v: i for i, v in enumerate(vs)}
        sub = cfggen.from_edges(len(vs), [(loc[a], loc[int(b)]) for a in vs for b in g.succ(a)
                                          if int(b) in loc], 0, len(vs) - 1)
        spp, _ = tpg.prime_paths(tpg.load_cfg(sub, tpg.TPG_LOAD_ANY_DIGRAPH), ws=ws())
        for p in spp.tolist():
            q = [vs[i] for i in p]
            cyclic = len(q) > 1 and q[0] == q[-1]
            if cyclic or not (fl[q[0]] & tpg.TPG_SCC_ENTRY_VERTEX
                              or fl[q[-1]] & tpg.TPG_SCC_EXIT_VERTEX):
                out.append(q)
    return sorted(out)


@pytest.mark.parametrize("k", [0])
def test_c2_internal_pps_match_the_per_scc_route(k):
    """At the ~200-vertex CFGs' size (beyond the oracle): the types count
    every prime path once, and the internal ones equal what the extension
    finds on each component alone."""
    rec = workloads()["c2"][k]
    g = cfggen.c2_cfg(rec["seed"])
    say("case c2 types", rec["seed"])
    h = tpg.load_cfg(g)
    comp, fl, _ = tpg.scc(h, ws=ws())
    assert np.array_equal(comp, oracle.scc(g))
    pp, _ = tpg.prime_paths(h, ws=ws())
    types, counts = tpg.prime_path_types(h, pp, ws=ws())
    assert counts[0] == 0 and counts.sum() == rec["n_pp"] == len(pp)
    assert np.array_equal(np.bincount(types, minlength=6), counts)
    got = sorted(p for p, t in zip(pp.tolist(), types) if t == tpg.TPG_PP_SCC_INTERNAL)
    assert got == _scc_subgraph_internal(g, h, comp, fl)
