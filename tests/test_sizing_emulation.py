"""The library's one-pass sizing loop (csrc/sizing.h: batches of levels,
growth to the exact size after an overflow, replay) run on the CPU against
the exact level sizes the oracle counts, with a simulated device that applies
the extension kernels' fit test.  It ends, reproduces every level size, and
overflows each level at most once, from a fresh workspace (the smallest
buffers), from a warm one and under predicted sizes; a device that reports
too few children is caught instead of replayed forever."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2210_16998_amd import cfggen
from tests.goldens import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OK, REPEATED = 0, 4


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sizing") / "sizing_sim")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I",
                           os.path.join(ROOT, "paper_2210_16998_amd", "csrc"),
                           os.path.join(ROOT, "tests", "sizing_sim.cpp"), "-o", exe])

    def run(sizes, first_batch=4, held=(0, 0), pred=(0, 0), growth=1.0, stale=0):
        inp = " ".join(map(str, [first_batch, held[0], held[1], pred[0], pred[1], growth, stale,
                                 len(sizes)] + [int(x) for x in sizes]))
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        st, novf, lmax, res, rec, msk, eq = out.split()
        return {"status": int(st), "n_overflows": int(novf), "Lmax": int(lmax),
                "reserves": int(res), "rec": int(rec), "msk": int(msk), "equal": eq == "1"}
    return run


def _sizes(g):
    """Paths per level (entries), closed cycles included: the path tree's
    level sizes."""
    _, lv, cy = oracle.count(g)
    s = (lv + cy)[1:]
    return s[:np.max(np.nonzero(s)) + 1]


def _graphs():
    w = workloads()
    gs = [("c1", cfggen.c1_cfg(0)), ("fig1", cfggen.fig1_cfg()), ("stress", cfggen.c5_cfg())]
    gs += [(f"c2 seed {r['seed']}", cfggen.c2_cfg(r["seed"])) for r in w["c2"]]
    return gs


@pytest.mark.parametrize("growth", [1.0, 1.5])
def test_fresh_workspace_sizing_ends_exact(sim, growth):
    for name, g in _graphs():
        s = _sizes(g)
        r = sim(s, growth=growth)
        assert r["status"] == OK and r["equal"], (name, r)
        assert r["Lmax"] == len(s)
        # each level overflows at most once, and not every level does
        assert r["n_overflows"] <= len(s), (name, r)


def test_largest_c2_cfg_fresh_then_warm(sim):
    """The ~200-vertex CFG whose fresh-workspace run stays off the GPU: on
    the CPU its sizing loop ends, exact, after a bounded number of replays."""
    g = cfggen.c2_cfg(workloads()["c2"][3]["seed"])
    s = _sizes(g)
    fresh = sim(s, growth=1.5)
    assert fresh["status"] == OK and fresh["equal"] and 0 < fresh["n_overflows"] <= len(s)
    # the next call on the same workspace: buffers held, one batch of all levels
    warm = sim(s, first_batch=fresh["Lmax"] + 1, held=(fresh["rec"], fresh["msk"]))
    assert warm["status"] == OK and warm["equal"] and warm["n_overflows"] == 0


def test_predicted_sizes_avoid_replays(sim):
    for name, g in _graphs():
        s = _sizes(g)
        exact = sim(s, pred=(int(1.25 * s.sum()) + g.n + 1024, int(1.25 * s.max()) + 1024))
        assert exact["status"] == OK and exact["equal"] and exact["n_overflows"] == 0, name
        under = sim(s, pred=(1, 1))
        assert under["status"] == OK and under["equal"], name


def test_a_device_reporting_too_few_children_is_an_error(sim):
    """Planted on the simulated device: the size the host reads back for an
    overflowing level's children is short of what the level claimed, so
    growing to it does not suffice.  The loop stops at the second overflow of
    that level instead of replaying it without end."""
    s = _sizes(cfggen.c2_cfg(workloads()["c2"][3]["seed"]))
    r = sim(s, stale=10**9)
    assert r["status"] == REPEATED


def test_held_capacity_beyond_the_node_limit_is_not_asked_for(sim):
    """A workspace whose buffers grew past the 2^31-node index range (a
    union sized from a large prediction before): the next run asks for at
    most the index range, never for more nodes than a tree may hold, and
    ends exact; growth near the limit stops at it as well."""
    lim = 2**31 - 3
    s = _sizes(cfggen.fig1_cfg())
    r = sim(s, held=(3 * 2**30, 0))
    assert r["status"] == OK and r["equal"] and r["rec"] == lim
    r = sim(s, pred=(3 * 2**30, 0))
    assert r["status"] == OK and r["equal"] and r["rec"] == lim
    big = np.array([1, 1_500_000_000, 500_000_000], np.int64)
    r = sim(big, held=(1_000_000_000, 2_000_000_000))
    assert r["status"] == OK and r["equal"] and r["n_overflows"] == 2 and r["rec"] == lim

