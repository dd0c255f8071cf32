"""GPU parity of the batched form: every graph of a batch against the CPU
oracle, element by element; sizing modes must not change a single byte."""
import numpy as np
import pytest

import oracle
from paper_2210_16998_amd import cfggen, tpg
from tests.goldens import workloads
from tests.gpu_util import ref_pp, ref_tp, say, ws

pytestmark = pytest.mark.gpu


def _check_batch(cfgs, res):
    for i, g in enumerate(cfgs):
        (po, pv), (to, tv) = res.graph(i)
        rp = ref_pp(g)[0]
        rt, _ = ref_tp(g)
        assert np.array_equal(po, rp.offsets) and np.array_equal(pv, rp.vertices), (i, g.name, "PP")
        assert np.array_equal(to, rt.offsets) and np.array_equal(tv, rt.vertices), (i, g.name, "TP")


def _same_result(a, b):
    return (np.array_equal(a.pp_first, b.pp_first) and np.array_equal(a.tp_first, b.tp_first)
            and np.array_equal(a.pp.offsets, b.pp.offsets)
            and np.array_equal(a.pp.vertices, b.pp.vertices)
            and np.array_equal(a.tp.offsets, b.tp.offsets)
            and np.array_equal(a.tp.vertices, b.tp.vertices))


def _mixed():
    cfgs = [cfggen.fig1_cfg(), cfggen.from_edges(1, [], 0, 0)]
    cfgs += [cfggen.c1_cfg(s) for s in range(4)]
    cfgs += [cfggen.random_small_cfg(7000 + s, 2 + (s * 7) % 150, extra=1 + s % 6) for s in range(40)]
    cfgs += [cfggen.batch_member_cfg(cfggen.C3_SEED_BASE + s) for s in range(40)]
    cfgs += [cfggen.loop_diamond_chain(k) for k in (1, 5, 9)]
    return cfgs


@pytest.mark.parametrize("flags", [0, tpg.TPG_FORCE_TWO_PASS])
def test_batch_mixed(flags):
    cfgs = _mixed()
    say("case batch mixed", len(cfgs), flags)
    hs = [tpg.load_cfg(g) for g in cfgs]
    res, st = tpg.batch_test_paths(hs, ws=ws(), flags=flags)
    assert st["n_unions"] >= 2  # several visited-set widths
    _check_batch(cfgs, res)


def test_batch_level_counts_are_exact():
    cfgs = _mixed()
    hs = [tpg.load_cfg(g) for g in cfgs]
    lv = np.zeros((len(cfgs), 64), np.int64)
    say("case batch level counts")
    tpg.batch_test_paths(hs, ws=ws(), level_counts=lv)
    for i, g in enumerate(cfgs):
        _, rl, rc = oracle.count(g)
        want = np.zeros(64, np.int64)
        for L in range(1, len(rl)):
            want[min(L, 64) - 1] += rl[L] + rc[L]
        assert np.array_equal(lv[i], want), (i, g.name)


def test_batch_c3_full_against_oracle_and_modes():
    cfgs = cfggen.c3_batch(4096)
    hs = [tpg.load_cfg(g) for g in cfgs]
    say("case c3 batch one-pass")
    res, st = tpg.batch_test_paths(hs, ws=ws())
    say("  unions", st["n_unions"], "pp", st["n_pp"], "ext", st["n_extensions"])
    _check_batch(cfgs, res)
    # the same bytes from the plain two-pass sizing and from (exact) predictions
    lv = np.zeros((len(cfgs), 64), np.int64)
    say("case c3 batch two-pass")
    res2, _ = tpg.batch_test_paths(hs, ws=ws(), flags=tpg.TPG_FORCE_TWO_PASS, level_counts=lv)
    pred = np.zeros((len(cfgs), 65), np.float32)
    pred[:, :64] = np.log1p(lv)
    pred[:, 64] = np.log1p(np.diff(res.pp_first))
    say("case c3 batch predicted")
    w = tpg.Workspace()
    res3, st3 = tpg.batch_test_paths(hs, ws=w, predicted=pred)
    assert st3["n_overflows"] == 0
    for r in (res2, res3):
        assert np.array_equal(r.pp_first, res.pp_first) and np.array_equal(r.tp_first, res.tp_first)
        assert np.array_equal(r.pp.offsets, res.pp.offsets)
        assert np.array_equal(r.pp.vertices, res.pp.vertices)
        assert np.array_equal(r.tp.offsets, res.tp.offsets)
        assert np.array_equal(r.tp.vertices, res.tp.vertices)
    w.close()


def test_batch_underpredicted_sizes_fall_back_exactly():
    cfgs = [cfggen.batch_member_cfg(cfggen.C3_SEED_BASE + s) for s in range(200)]
    hs = [tpg.load_cfg(g) for g in cfgs]
    pred = np.zeros((len(cfgs), 65), np.float32)  # predicts (almost) nothing
    w = tpg.Workspace()
    say("case batch under-prediction")
    res, st = tpg.batch_test_paths(hs, ws=w, predicted=pred)
    assert st["n_overflows"] > 0
    _check_batch(cfgs, res)
    w.close()


def test_batch_overpredicted_and_nonfinite_sizes_fall_back_exactly():
    """Predictions far above anything real (every level at log1p 40), and
    infinite or not-a-number entries, under a pool cap: the capacities are
    clamped, unions that cannot be allocated are sized exactly instead, and
    every byte equals the two-pass result, on a fresh workspace and again on
    the warm one."""
    cfgs = [cfggen.batch_member_cfg(cfggen.C3_SEED_BASE + s) for s in range(120)]
    hs = [tpg.load_cfg(g) for g in cfgs]
    say("case batch over-prediction")
    ref, _ = tpg.batch_test_paths(hs, ws=ws(), flags=tpg.TPG_FORCE_TWO_PASS)
    pred = np.full((len(cfgs), 65), 40.0, np.float32)
    pred[3, :] = np.inf
    pred[7, 5] = np.nan
    pred[11, 63] = -np.inf
    w = tpg.Workspace()
    cap = 8 << 30
    res, st = tpg.batch_test_paths(hs, ws=w, predicted=pred, pool_cap=cap)
    assert _same_result(res, ref)
    assert w.bytes <= cap
    res2, _ = tpg.batch_test_paths(hs, ws=w, predicted=pred, pool_cap=cap)
    assert _same_result(res2, ref)
    say("  unions", st["n_unions"], "overflows", st["n_overflows"], "bytes", w.bytes)
    w.close()


def test_batch_device_output():
    cfgs = [cfggen.c1_cfg(s) for s in range(3)] + [cfggen.fig1_cfg()]
    hs = [tpg.load_cfg(g) for g in cfgs]
    say("case batch device output")
    res, _ = tpg.batch_test_paths(hs, ws=ws(), flags=tpg.TPG_OUT_DEVICE)
    off, vtx = res.tp.torch_views()
    off, vtx = off.cpu().numpy(), vtx.cpu().numpy()
    for i, g in enumerate(cfgs):
        a, b = int(res.tp_first[i]), int(res.tp_first[i + 1])
        rt, _ = ref_tp(g)
        o = off[a:b + 1]
        assert np.array_equal(o - o[0], rt.offsets)
        assert np.array_equal(vtx[o[0]:o[-1]], rt.vertices)


def test_tile_shapes_do_not_change_a_byte():
    """Every launch shape of the extension kernel gives identical results."""
    g = cfggen.c2_cfg(2)
    h = tpg.load_cfg(g)
    w = tpg.Workspace()
    outs = []
    for variant in (0, 1, 2):
        for items in (1, 2, 4, 8):
            for wgs in (1, 2):
                tpg.set_tuning(w, {"items": [items] * 7, "wgs_per_cu": [wgs] * 7,
                                   "variant": [variant] * 7})
                say("case tile shape", variant, items, wgs)
                pp, tp, _ = tpg.test_paths(h, ws=w)
                outs.append((pp.offsets.tobytes(), pp.vertices.tobytes(), tp.vertices.tobytes()))
    assert all(o == outs[0] for o in outs)
    rp = ref_pp(g, local=True)[0]
    assert np.array_equal(np.frombuffer(outs[0][1], np.int32), rp.vertices)
    w.close()


def test_autotune_then_batch_is_exact():
    cfgs = [cfggen.batch_member_cfg(cfggen.C3_SEED_BASE + s) for s in range(300)]
    hs = [tpg.load_cfg(g) for g in cfgs]
    w = tpg.Workspace()
    say("case autotune")
    t = tpg.autotune(hs, w)
    assert t["best_ms"][0] > 0 and t["items"][0] in (1, 2, 4, 8) and t["variant"][0] in (0, 1, 2)
    res, _ = tpg.batch_test_paths(hs, ws=w)
    _check_batch(cfgs, res)
    w.close()


@pytest.mark.parametrize("learned", [False, True])
def test_repeated_batch_call_runs_as_one_graph(learned):
    """A batched call that repeats the previous one is captured into one HIP
    graph and then replayed (one launch, one wait): every replay gives the
    bytes of the ordinary call, graph by graph equal to the oracle; a call
    in between that changes the workspace only sends the next one back to
    the ordinary path."""
    cfgs = _mixed()
    hs = [tpg.load_cfg(g) for g in cfgs]
    pred = None
    if learned:
        from paper_2210_16998_amd import sizer
        pred = sizer.predict(tpg.MLP.load(sizer.DEFAULT_MODEL), hs)
    w = tpg.Workspace()
    say("case batch call graph", learned)
    first, st = tpg.batch_test_paths(hs, ws=w, flags=tpg.TPG_NO_TIMING, predicted=pred)
    _check_batch(cfgs, first)
    states, allocs = [st["call_graph"]], [st["n_allocs"]]
    for _ in range(4):
        r, st = tpg.batch_test_paths(hs, ws=w, flags=tpg.TPG_NO_TIMING, predicted=pred)
        states.append(st["call_graph"])
        allocs.append(st["n_allocs"])
        assert _same_result(r, first)
        assert st["n_pp"] == len(first.pp)
    say("  states", states, "allocations", allocs)
    if 3 in states:
        say("  ", tpg.lib().tpg_last_error().decode())
    assert states[0] == 0 and 1 in states and states[-1] == 2
    # another call on the workspace (larger buffers): the batch stays exact
    tpg.test_paths(tpg.load_cfg(cfggen.c2_cfg(workloads()["c2"][0]["seed"])), ws=w)
    for _ in range(3):
        r, st = tpg.batch_test_paths(hs, ws=w, flags=tpg.TPG_NO_TIMING, predicted=pred)
        assert _same_result(r, first)
    # device output through the graph
    for _ in range(3):
        r, st = tpg.batch_test_paths(hs, ws=w, flags=tpg.TPG_NO_TIMING | tpg.TPG_OUT_DEVICE,
                                     predicted=pred)
    off, vtx = r.tp.torch_views()
    assert np.array_equal(off.cpu().numpy(), first.tp.offsets)
    assert np.array_equal(vtx.cpu().numpy(), first.tp.vertices)
    assert st["call_graph"] == 2
    w.close()
