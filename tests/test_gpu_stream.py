"""Digest-only results and streamed delivery on the GPU, against the CPU
oracle: set digests, first-vertex chunks that concatenate to the canonical
prime-path set, test-path chunks, and a callback that stops the call."""
import numpy as np
import pytest

import oracle
from oracle import PathList
from paper_2210_16998_amd import cfggen, tpg
from tests.goldens import workloads
from tests.gpu_util import ref_pp, ref_tp, say

pytestmark = pytest.mark.gpu


def _graphs():
    gs = [cfggen.fig1_cfg(), cfggen.c1_cfg(0), cfggen.from_edges(1, [], 0, 0)]
    gs += [cfggen.random_small_cfg(50_000 + s, 3 + s % 40, extra=1 + s % 7) for s in range(12)]
    return gs


def _concat(chunks):
    offs, vtx, base = [np.zeros(1, np.int64)], [], 0
    for c in chunks:
        offs.append(c.offsets[1:] + base)
        vtx.append(c.vertices)
        base += len(c.vertices)
    return PathList(np.concatenate(offs), np.concatenate(vtx) if vtx else np.zeros(0, np.int32))


def test_digest_only_and_digest_flag():
    w = tpg.Workspace()
    for g in _graphs() + [cfggen.c2_cfg(workloads()["c2"][0]["seed"])]:
        say("case digest", g.name, g.n)
        h = tpg.load_cfg(g)
        rp = ref_pp(g, local=g.n > 100)[0]
        rt = ref_tp(g)[0]
        d, _ = tpg.prime_paths(h, ws=w, flags=tpg.TPG_DIGEST_ONLY)
        assert isinstance(d, tpg.SetDigest)
        assert (d.n_paths, d.n_vertices) == (len(rp), len(rp.vertices))
        assert d.digest == oracle.digest(rp)
        pd, td, _ = tpg.test_paths(h, ws=w, flags=tpg.TPG_DIGEST_ONLY)
        assert pd.digest == oracle.digest(rp) and td.digest == oracle.digest(rt)
        assert (td.n_paths, td.n_vertices) == (len(rt), len(rt.vertices))
        pp, tp, _ = tpg.test_paths(h, ws=w, flags=tpg.TPG_DIGEST)
        assert np.array_equal(pp.vertices, rp.vertices) and np.array_equal(tp.vertices, rt.vertices)
        assert pp.digest == oracle.digest(rp) and tp.digest == oracle.digest(rt)
    w.close()


@pytest.mark.parametrize("chunk", [1, 7, 64, 0])
def test_prime_paths_stream_concatenates(chunk):
    w = tpg.Workspace()
    gs = _graphs() + [cfggen.random_digraph(70_000 + s, 2 + s % 9, 0.3) for s in range(6)]
    for g in gs:
        h = tpg.load_cfg(g, tpg.TPG_LOAD_ANY_DIGRAPH)
        rp = oracle.prime_paths(g)[0]
        got = []

        def on_chunk(c, first, end):
            got.append((c, first, end))
        tot, st = tpg.prime_paths_stream(h, on_chunk, ws=w, chunk_vertices=chunk)
        ranges = [(f, e) for _, f, e in got]
        step = chunk if chunk > 0 else 32
        assert ranges == [(lo, min(lo + step, g.n)) for lo in range(0, g.n, step)]
        for c, f, e in got:
            firsts = c.vertices[c.offsets[:-1]] if len(c) else np.zeros(0)
            assert np.all((firsts >= f) & (firsts < e))
            assert c.digest == oracle.digest(c)
        cat = _concat([c for c, _, _ in got])
        assert np.array_equal(cat.offsets, rp.offsets) and np.array_equal(cat.vertices, rp.vertices), g.name
        assert (tot.n_paths, tot.n_vertices, tot.digest) == (len(rp), len(rp.vertices), oracle.digest(rp))
        assert st["n_pp"] == len(rp)
    say("case stream chunk", chunk, len(gs))
    w.close()


def test_prime_paths_stream_bounds_device_memory():
    """On K_9 every first vertex roots a tree of the same size: streaming one
    first vertex at a time needs a fraction of the whole run's pool."""
    g = cfggen.complete_digraph(9)
    h = tpg.load_cfg(g, tpg.TPG_LOAD_ANY_DIGRAPH)
    rp = oracle.prime_paths(g)[0]
    w_full = tpg.Workspace()
    _, st_full = tpg.prime_paths(h, ws=w_full)
    w_full.close()
    w = tpg.Workspace()
    parts = []
    say("case stream memory K9")
    tot, st = tpg.prime_paths_stream(h, lambda c, f, e: parts.append(c), ws=w, chunk_vertices=1)
    cat = _concat(parts)
    assert np.array_equal(cat.vertices, rp.vertices) and tot.digest == oracle.digest(rp)
    assert st["device_bytes"] < st_full["device_bytes"] // 2, (st["device_bytes"], st_full["device_bytes"])
    w.close()


def test_prime_paths_stream_c2_device_chunks():
    rec = workloads()["c2"][0]
    g = cfggen.c2_cfg(rec["seed"])
    h = tpg.load_cfg(g)
    rp = ref_pp(g, local=True)[0]
    w = tpg.Workspace()
    parts = []

    def on_chunk(c, first, end):
        off, vtx = c.torch_views()
        parts.append(PathList(off.cpu().numpy(), vtx.cpu().numpy()))
    say("case stream c2 device", rec["seed"])
    tot, st = tpg.prime_paths_stream(h, on_chunk, ws=w, flags=tpg.TPG_OUT_DEVICE, chunk_vertices=16)
    cat = _concat(parts)
    assert np.array_equal(cat.offsets, rp.offsets) and np.array_equal(cat.vertices, rp.vertices)
    assert tot.digest == oracle.digest(rp)
    assert st["n_extensions"] == rec["n_extensions"]
    w.close()


@pytest.mark.parametrize("chunk", [1, 1000, 0])
def test_test_paths_stream_chunks(chunk):
    w = tpg.Workspace()
    for g in _graphs()[:6] + [cfggen.c2_cfg(workloads()["c2"][1]["seed"])]:
        h = tpg.load_cfg(g)
        if chunk == 1 and g.n > 100:
            continue
        rp = ref_pp(g, local=g.n > 100)[0]
        rt = ref_tp(g)[0]
        got = []
        pd, td, _ = tpg.test_paths_stream(h, lambda c, f, e: got.append((c, f, e)), ws=w,
                                          chunk_paths=chunk)
        step = chunk if chunk > 0 else 1 << 20
        assert [(f, e) for _, f, e in got] == [(k, min(k + step, len(rt))) for k in range(0, len(rt), step)]
        cat = _concat([c for c, _, _ in got])
        assert np.array_equal(cat.offsets, rt.offsets) and np.array_equal(cat.vertices, rt.vertices)
        assert td.digest == oracle.digest(rt) and pd.digest == oracle.digest(rp)
    say("case tp stream", chunk)
    w.close()


def test_stream_callback_stops_the_call():
    w = tpg.Workspace()
    g = cfggen.c1_cfg(0)
    h = tpg.load_cfg(g)
    say("case stream stop")
    with pytest.raises(tpg.TpgError) as ei:
        tpg.prime_paths_stream(h, lambda c, f, e: True, ws=w, chunk_vertices=5)
    assert ei.value.name == "TPG_ERR_CALLBACK"
    # the workspace stays usable
    pp, _ = tpg.prime_paths(h, ws=w)
    assert np.array_equal(pp.vertices, oracle.prime_paths(g)[0].vertices)
    w.close()
