"""The allocation-free form of prime-path typing (tpg_prime_path_types_noalloc,
scratch in a fixed device array) against the allocating entry point
(tpg_prime_path_types) on the same device-resident prime-path sets: every
path's type and the per-type counts identical, over calls in a row whose
inputs shrink (the fixed scratch keeps the previous call's contents)."""
import numpy as np
import pytest

from paper_2210_16998_amd import cfggen, tpg
from tests.goldens import workloads
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _cases():
    big = cfggen.c2_cfg(workloads()["c2"][3]["seed"])
    return [("cfg209", big), ("c1", cfggen.c1_cfg(0)), ("fig1", cfggen.fig1_cfg()),
            ("cfg209 again", big)]


def test_noalloc_types_equal_the_allocating_entry_point():
    import torch
    w = tpg.Workspace()
    for name, g in _cases():
        h = tpg.load_cfg(g)
        say("case noalloc types", name, g.n)
        pp, _ = tpg.prime_paths(h, ws=w, flags=tpg.TPG_OUT_DEVICE)
        n = pp.n_paths
        ref_types, ref_counts = tpg.prime_path_types(h, pp, ws=w)
        types = torch.full((max(n, 1),), 255, dtype=torch.uint8, device="cuda")
        counts = tpg.prime_path_types_noalloc(h, pp, types)
        torch.cuda.synchronize()
        assert np.array_equal(counts, ref_counts), (name, counts, ref_counts)
        assert np.array_equal(types[:n].cpu().numpy(), ref_types), name
        assert int(counts.sum()) == n
        # counts only, no per-path output
        assert np.array_equal(tpg.prime_path_types_noalloc(h, pp, None), ref_counts)
    w.close()


def test_noalloc_types_on_a_torch_stream():
    import torch
    g = cfggen.c1_cfg(3)
    h = tpg.load_cfg(g)
    w = tpg.Workspace()
    s = torch.cuda.Stream()
    say("case noalloc types on a stream")
    pp, _ = tpg.prime_paths(h, ws=w, flags=tpg.TPG_OUT_DEVICE, stream=s)
    ref_types, ref_counts = tpg.prime_path_types(h, pp, ws=w, stream=s)
    types = torch.zeros(pp.n_paths, dtype=torch.uint8, device="cuda")
    counts = tpg.prime_path_types_noalloc(h, pp, types, stream=s)
    torch.cuda.synchronize()
    assert np.array_equal(counts, ref_counts)
    assert np.array_equal(types.cpu().numpy(), ref_types)
    w.close()
