"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and validates inputs (no device needed)."""
import re
import os

import numpy as np
import pytest

from paper_2210_16998_amd import cfggen, tpg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tpg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tpg_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported_and_bound():
    L = tpg.lib()
    decl = _declared()
    assert len(decl) >= 14
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(tpg.declared_symbols()) == decl


def test_version_and_status_strings():
    assert "tpg" in tpg.version()
    for s in tpg.STATUS:
        assert tpg.lib().tpg_status_str(s)


def _err(fn):
    with pytest.raises(tpg.TpgError) as ei:
        fn()
    return ei.value.name


def test_load_errors():
    assert _err(lambda: tpg.load_cfg_csr(0, [0], [], 0, 0)) == "TPG_ERR_INVALID_ARG"
    assert _err(lambda: tpg.load_cfg_csr(2, [1, 1, 1], [], 0, 1)) == "TPG_ERR_BAD_CSR"
    assert _err(lambda: tpg.load_cfg_csr(2, [0, 2, 1], [1, 1], 0, 1)) == "TPG_ERR_BAD_CSR"
    assert _err(lambda: tpg.load_cfg_csr(2, [0, 1, 1], [5], 0, 1)) == "TPG_ERR_BAD_CSR"
    assert _err(lambda: tpg.load_cfg_csr(2, [0, 1, 1], [1], 0, 7)) == "TPG_ERR_BAD_ENTRY_EXIT"
    # entry with a predecessor / exit with a successor (Sec. 3 assumptions)
    assert _err(lambda: tpg.load_cfg_csr(3, [0, 1, 2, 3], [1, 0, 0], 0, 2)) == "TPG_ERR_BAD_ENTRY_EXIT"
    # vertex 2 unreachable
    assert _err(lambda: tpg.load_cfg_csr(3, [0, 1, 1, 2], [1, 1], 0, 1)) == "TPG_ERR_UNREACHABLE"
    # duplicate arcs: merged by default, rejected when strict
    g = tpg.load_cfg_csr(2, [0, 2, 2], [1, 1], 0, 1)
    assert g.info() == (2, 1, 0, 1)
    assert _err(lambda: tpg.load_cfg_csr(2, [0, 2, 2], [1, 1], 0, 1, tpg.TPG_LOAD_STRICT)) \
        == "TPG_ERR_BAD_CSR"
    big = 4097
    assert _err(lambda: tpg.load_cfg_csr(big, np.zeros(big + 1, np.int64), [], 0, 1)) \
        == "TPG_ERR_UNSUPPORTED"


def test_load_canonicalizes_rows():
    rp = np.array([0, 3, 4, 4], np.int64)
    ci = np.array([2, 1, 2, 2], np.int32)
    g = tpg.load_cfg_csr(3, rp, ci, 0, 2)
    r2, c2 = g.csr()
    assert r2.tolist() == [0, 2, 3, 3] and c2.tolist() == [1, 2, 2]


def test_any_digraph_flag_skips_cfg_checks():
    k = cfggen.complete_digraph(4)
    with pytest.raises(tpg.TpgError):
        tpg.load_cfg(k)
    g = tpg.load_cfg(k, tpg.TPG_LOAD_ANY_DIGRAPH)
    assert g.info()[0] == 4


def test_generated_workloads_load():
    for g in [cfggen.fig1_cfg(), cfggen.c1_cfg(0), cfggen.c2_cfg(9), cfggen.c5_cfg(),
              cfggen.batch_member_cfg(cfggen.C3_SEED_BASE)]:
        h = tpg.load_cfg(g)
        assert h.info()[0] == g.n


@pytest.mark.skipif(tpg.device_count() > 0, reason="checks the no-device error path")
def test_no_device_is_an_error_not_a_fallback():
    g = tpg.load_cfg(cfggen.fig1_cfg())
    assert _err(lambda: tpg.prime_paths(g)) == "TPG_ERR_DEVICE"


def test_path_type_inputs_are_checked_on_the_host():
    """Malformed host path sets are rejected before any device work; a valid
    one reaches the device, which this machine lacks (an error, not a
    fallback)."""
    g = tpg.load_cfg(cfggen.fig1_cfg())

    class P:
        def __init__(self, off, vtx):
            self.offsets = np.array(off, np.int64)
            self.vertices = np.array(vtx, np.int32)
    assert _err(lambda: tpg.prime_path_types(g, P([0, 2, 2], [0, 1]))) == "TPG_ERR_INVALID_ARG"
    assert _err(lambda: tpg.prime_path_types(g, P([1, 2], [0, 1]))) == "TPG_ERR_INVALID_ARG"
    assert _err(lambda: tpg.prime_path_types(g, P([0, 2], [0, 11]))) == "TPG_ERR_INVALID_ARG"
    assert _err(lambda: tpg.prime_path_types(g, P([0, 2], [0, 1]))) == "TPG_ERR_DEVICE"
    assert _err(lambda: tpg.scc(g)) == "TPG_ERR_DEVICE"
    assert _err(lambda: tpg.prime_paths_vertex_lists(g)) == "TPG_ERR_DEVICE"


def test_noalloc_types_reject_a_graph_beyond_the_fixed_scratch():
    """The allocation-free typing holds its scratch in a fixed 1 MiB device
    array; a graph that needs more is refused before any device work (so no
    device is needed here)."""
    n, deg = 4096, 64
    rows = [sorted({(v + k) % n for k in range(1, deg + 1)}) for v in range(n)]
    row_ptr = np.zeros(n + 1, np.int64)
    row_ptr[1:] = np.cumsum([len(r) for r in rows])
    col = np.concatenate([np.asarray(r, np.int32) for r in rows])
    g = tpg.load_cfg_csr(n, row_ptr, col, 0, n - 1, tpg.TPG_LOAD_ANY_DIGRAPH)
    rc = tpg.lib().tpg_prime_path_types_noalloc(g.handle, None, None, 0, None, None, None)
    assert tpg.STATUS[rc] == "TPG_ERR_CAPACITY"
    assert b"scratch" in tpg.lib().tpg_last_error()
    rc = tpg.lib().tpg_prime_path_types_noalloc(g.handle, None, None, -1, None, None, None)
    assert tpg.STATUS[rc] == "TPG_ERR_INVALID_ARG"
