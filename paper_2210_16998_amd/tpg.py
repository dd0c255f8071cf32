"""Thin ctypes binding of libtpg.so (include/tpg.h): argument marshalling only.

Every step of the path computation runs in the library's HIP kernels; this
module only moves arguments and results.  It fails loudly when the library
has not been built (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtpg.so")

TPG_OK = 0
TPG_LOAD_STRICT = 0x1
TPG_LOAD_ANY_DIGRAPH = 0x2
TPG_LOAD_BINARIZE = 0x4
TPG_OUT_DEVICE = 0x1
TPG_FORCE_TWO_PASS = 0x2
TPG_NO_TIMING = 0x4
TPG_DIGEST = 0x8
TPG_DIGEST_ONLY = 0x10
TPG_STREAM = 0x20
TPG_ORDER_BY_LAST = 0x40
TPG_TP_GREEDY = 0x80
TPG_NO_CALL_GRAPH = 0x100
# strongly connected components and prime-path types (Sec. 2, Defs. 2-10)
TPG_SCC_CYCLIC, TPG_SCC_ENTRY_VERTEX, TPG_SCC_EXIT_VERTEX = 0x1, 0x2, 0x4
TPG_PP_COMPLETE, TPG_PP_SCC_INTERNAL, TPG_PP_SCC_EXIT, TPG_PP_SCC_ENTRY, TPG_PP_OTHER = 1, 2, 3, 4, 5

STATUS = {0: "TPG_OK", -1: "TPG_ERR_INVALID_ARG", -2: "TPG_ERR_BAD_CSR",
          -3: "TPG_ERR_BAD_ENTRY_EXIT", -4: "TPG_ERR_UNREACHABLE",
          -5: "TPG_ERR_OOM_HOST", -6: "TPG_ERR_OOM_DEVICE", -7: "TPG_ERR_CAPACITY",
          -8: "TPG_ERR_DEVICE", -9: "TPG_ERR_UNSUPPORTED", -10: "TPG_ERR_CALLBACK"}


class TpgError(RuntimeError):
    def __init__(self, status: int, message: str) -> None:
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class _Paths(ctypes.Structure):
    _fields_ = [("n_paths", ctypes.c_int64), ("n_vertices", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("vertices", ctypes.c_void_p),
                ("on_device", ctypes.c_int32), ("reserved_", ctypes.c_int32),
                ("digest", ctypes.c_uint64 * 2)]


# int32 (*)(void* ctx, const tpg_paths* chunk, int64 first, int64 end)
_CHUNK_FN = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(_Paths),
                             ctypes.c_int64, ctypes.c_int64)


class _Stats(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("n_extensions", ctypes.c_int64), ("n_cycles", ctypes.c_int64),
                ("n_pp", ctypes.c_int64), ("n_pp_vertices", ctypes.c_int64),
                ("n_tp_spliced", ctypes.c_int64), ("n_tp", ctypes.c_int64),
                ("n_tp_vertices", ctypes.c_int64), ("n_overflows", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("ms_extend", ctypes.c_double),
                ("ms_rank", ctypes.c_double), ("ms_tp", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("ms_extend_kernel", ctypes.c_double),
                ("n_extend_launches", ctypes.c_int64), ("peak_level_nodes", ctypes.c_int64),
                ("n_unions", ctypes.c_int64), ("pred_nodes", ctypes.c_int64),
                ("pred_peak_level_nodes", ctypes.c_int64), ("call_graph", ctypes.c_int64),
                ("n_allocs", ctypes.c_int64)]


class _Opts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("stream", ctypes.c_void_p), ("ws", ctypes.c_void_p),
                ("pool_cap_bytes", ctypes.c_uint64), ("stats", ctypes.POINTER(_Stats)),
                ("level_counts", ctypes.POINTER(ctypes.c_int64)),
                ("level_counts_len", ctypes.c_int32), ("reserved_", ctypes.c_int32),
                ("on_chunk", _CHUNK_FN), ("chunk_ctx", ctypes.c_void_p),
                ("chunk_vertices", ctypes.c_int32), ("reserved2_", ctypes.c_int32),
                ("chunk_paths", ctypes.c_int64)]


class _BatchResult(ctypes.Structure):
    _fields_ = [("pp", _Paths), ("tp", _Paths), ("pp_first", ctypes.POINTER(ctypes.c_int64)),
                ("tp_first", ctypes.POINTER(ctypes.c_int64)), ("n_graphs", ctypes.c_int32),
                ("reserved_", ctypes.c_int32)]


class _Tuning(ctypes.Structure):
    _fields_ = [("items", ctypes.c_int32 * 7), ("wgs_per_cu", ctypes.c_int32 * 7),
                ("variant", ctypes.c_int32 * 7),
                ("best_ms", ctypes.c_double * 7)]


# every symbol include/tpg.h declares, with its signature
_SIGS = {
    "tpg_load_cfg_csr": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "tpg_graph_free": (None, [ctypes.c_void_p]),
    "tpg_graph_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32)]),
    "tpg_graph_csr": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "tpg_workspace_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "tpg_workspace_free": (None, [ctypes.c_void_p]),
    "tpg_workspace_bytes": (ctypes.c_int64, [ctypes.c_void_p]),
    "tpg_prime_paths": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Opts),
                                       ctypes.POINTER(_Paths)]),
    "tpg_test_paths": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Opts),
                                      ctypes.POINTER(_Paths), ctypes.POINTER(_Paths)]),
    "tpg_paths_free": (None, [ctypes.POINTER(_Paths)]),
    "tpg_batch_test_paths": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                            ctypes.POINTER(_Opts), ctypes.c_void_p,
                                            ctypes.POINTER(_BatchResult)]),
    "tpg_batch_result_free": (None, [ctypes.POINTER(_BatchResult)]),
    "tpg_autotune": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                    ctypes.POINTER(_Opts), ctypes.POINTER(_Tuning)]),
    "tpg_workspace_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Tuning)]),
    "tpg_workspace_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Tuning)]),
    "tpg_features": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                    ctypes.c_void_p]),
    "tpg_mlp_num_params": (ctypes.c_int32, []),
    "tpg_mlp_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_uint64,
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "tpg_mlp_free": (None, [ctypes.c_void_p]),
    "tpg_mlp_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "tpg_mlp_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "tpg_mlp_set_normalizer": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p]),
    "tpg_mlp_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_void_p]),
    "tpg_mlp_gradients": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_float)]),
    "tpg_mlp_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int32, ctypes.c_float,
                                          ctypes.POINTER(ctypes.c_float)]),
    "tpg_mlp_save": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "tpg_mlp_load": (ctypes.c_int, [ctypes.c_int32, ctypes.c_char_p,
                                    ctypes.POINTER(ctypes.c_void_p)]),
    "tpg_prime_paths_vertex_lists": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                    ctypes.POINTER(_Paths)]),
    "tpg_scc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "tpg_prime_path_types": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Paths),
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "tpg_ccfg": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Opts), ctypes.c_void_p,
                                ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "tpg_scc_paths": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Opts),
                                     ctypes.POINTER(_Paths), ctypes.POINTER(_Paths),
                                     ctypes.POINTER(_Paths)]),
    "tpg_scc_internal_pps": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Opts),
                                            ctypes.POINTER(_Paths)]),
    "tpg_merged_pps": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Opts),
                                      ctypes.POINTER(_Paths), ctypes.POINTER(_Paths),
                                      ctypes.POINTER(_Paths)]),
    "tpg_prime_path_types_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                    ctypes.c_void_p, ctypes.c_int64,
                                                    ctypes.c_void_p, ctypes.c_void_p,
                                                    ctypes.c_void_p]),
    "tpg_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "tpg_last_error": (ctypes.c_char_p, []),
    "tpg_version": (ctypes.c_char_p, []),
    "tpg_device_count": (ctypes.c_int32, []),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        # Bind libtpg to the HIP runtime torch carries (same soname): one
        # runtime per process, so torch streams and tensors interoperate.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2210_16998_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def declared_symbols():
    return list(_SIGS)


def _check(rc: int) -> None:
    if rc != TPG_OK:
        msg = lib().tpg_last_error()
        raise TpgError(rc, msg.decode() if msg else "")


class Graph:
    """A loaded CFG (library handle, host memory)."""

    def __init__(self, handle: int) -> None:
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def info(self) -> Tuple[int, int, int, int]:
        n, m, e, x = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().tpg_graph_info(self._h, ctypes.byref(n), ctypes.byref(m),
                                    ctypes.byref(e), ctypes.byref(x)))
        return n.value, m.value, e.value, x.value

    def csr(self) -> Tuple[np.ndarray, np.ndarray]:
        n, m, _, _ = self.info()
        rp = np.zeros(n + 1, np.int64)
        ci = np.zeros(max(m, 1), np.int32)
        _check(lib().tpg_graph_csr(self._h, rp.ctypes.data, ci.ctypes.data))
        return rp, ci[:m]

    def close(self) -> None:
        if self._h:
            lib().tpg_graph_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def load_cfg_csr(n: int, row_ptr: np.ndarray, col_idx: np.ndarray, entry: int, exit: int,
                 flags: int = 0) -> Graph:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, np.int32)
    h = ctypes.c_void_p()
    _check(lib().tpg_load_cfg_csr(int(n), rp.ctypes.data, ci.ctypes.data, int(entry),
                                  int(exit), int(flags), ctypes.byref(h)))
    return Graph(h.value)


def load_cfg(cfg, flags: int = 0) -> Graph:
    """Loads a paper_2210_16998_amd.cfggen.CFG."""
    return load_cfg_csr(cfg.n, cfg.row_ptr, cfg.col_idx, cfg.entry, cfg.exit, flags)


class Workspace:
    """Device arena + stream reused across calls (grows on demand)."""

    def __init__(self, device: int = -1) -> None:
        h = ctypes.c_void_p()
        _check(lib().tpg_workspace_create(int(device), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    @property
    def bytes(self) -> int:
        return int(lib().tpg_workspace_bytes(self._h))

    def close(self) -> None:
        if self._h:
            lib().tpg_workspace_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SetDigest:
    """Counts and digest of a set returned without arrays (TPG_DIGEST_ONLY,
    TPG_STREAM)."""

    def __init__(self, p: _Paths) -> None:
        self.n_paths = int(p.n_paths)
        self.n_vertices = int(p.n_vertices)
        self.digest = (int(p.digest[0]), int(p.digest[1]))

    def __len__(self) -> int:
        return self.n_paths


class HostPaths:
    """Host result: offsets int64 [n+1], vertices int32 (copied out of the
    library-owned arrays, which are then released unless `owned` is False,
    as for a streamed chunk the library releases itself)."""

    def __init__(self, p: _Paths, owned: bool = True) -> None:
        n, nv = p.n_paths, p.n_vertices
        self.offsets = np.ctypeslib.as_array(
            ctypes.cast(p.offsets, ctypes.POINTER(ctypes.c_int64)), shape=(n + 1,)).copy()
        self.vertices = (np.ctypeslib.as_array(
            ctypes.cast(p.vertices, ctypes.POINTER(ctypes.c_int32)), shape=(nv,)).copy()
            if nv else np.zeros(0, np.int32))
        self.digest = (int(p.digest[0]), int(p.digest[1]))
        if owned:
            lib().tpg_paths_free(ctypes.byref(p))

    def __len__(self) -> int:
        return len(self.offsets) - 1

    def __getitem__(self, i: int):
        return self.vertices[self.offsets[i]:self.offsets[i + 1]].tolist()

    def tolist(self):
        return [self[i] for i in range(len(self))]


class _CudaArray:
    def __init__(self, ptr: int, n: int, typestr: str) -> None:
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr,
                                         "data": (int(ptr), False), "version": 3}


class DevicePaths:
    """Device result view (TPG_OUT_DEVICE): pointers into the workspace,
    valid until the next call on that workspace."""

    def __init__(self, p: _Paths) -> None:
        self.n_paths = int(p.n_paths)
        self.n_vertices = int(p.n_vertices)
        self.offsets_ptr = int(p.offsets or 0)
        self.vertices_ptr = int(p.vertices or 0)
        self.digest = (int(p.digest[0]), int(p.digest[1]))

    def __len__(self) -> int:
        return self.n_paths

    def torch_views(self):
        """(offsets, vertices) as zero-copy torch tensors on the GPU."""
        import torch
        off = torch.as_tensor(_CudaArray(self.offsets_ptr, self.n_paths + 1, "<i8"),
                              device="cuda")
        vtx = torch.as_tensor(_CudaArray(self.vertices_ptr, max(self.n_vertices, 1), "<i4"),
                              device="cuda")
        return off, vtx[:self.n_vertices]


def _wrap(p: _Paths):
    if not p.offsets:
        return SetDigest(p)
    return DevicePaths(p) if p.on_device else HostPaths(p)


def _opts(ws: Optional[Workspace], flags: int, stream, stats: Optional[_Stats],
          pool_cap: int = 0, level_buf: Optional[np.ndarray] = None) -> _Opts:
    o = _Opts()
    o.struct_size = ctypes.sizeof(_Opts)
    o.flags = int(flags)
    if stream is not None:
        o.stream = ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    o.ws = ws.handle if ws is not None else None
    o.pool_cap_bytes = int(pool_cap)
    o.stats = ctypes.pointer(stats) if stats is not None else None
    if level_buf is not None:
        o.level_counts = level_buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        o.level_counts_len = len(level_buf)
    return o


def _stats_dict(s: _Stats) -> Dict[str, float]:
    return {k: getattr(s, k) for k, _ in _Stats._fields_}


def prime_paths(g: Graph, ws: Optional[Workspace] = None, flags: int = 0, stream=None,
                pool_cap: int = 0, level_counts: Optional[np.ndarray] = None):
    """(paths, stats).  paths is HostPaths, or DevicePaths with TPG_OUT_DEVICE."""
    st = _Stats()
    o = _opts(ws, flags, stream, st, pool_cap, level_counts)
    out = _Paths()
    _check(lib().tpg_prime_paths(g.handle, ctypes.byref(o), ctypes.byref(out)))
    return _wrap(out), _stats_dict(st)


def test_paths(g: Graph, ws: Optional[Workspace] = None, flags: int = 0, stream=None,
               pool_cap: int = 0, want_pp: bool = True):
    """(prime paths or None, test paths, stats)."""
    st = _Stats()
    o = _opts(ws, flags, stream, st, pool_cap)
    pp, tp = _Paths(), _Paths()
    _check(lib().tpg_test_paths(g.handle, ctypes.byref(o),
                                ctypes.byref(pp) if want_pp else None, ctypes.byref(tp)))
    return (_wrap(pp) if want_pp else None), _wrap(tp), _stats_dict(st)


def _stream_call(fn, on_chunk, o: _Opts, *args):
    """Runs fn with a ctypes trampoline for on_chunk(chunk, first, end); the
    chunk is HostPaths (copied) or DevicePaths (valid during the call only).
    A truthy return, or an exception, stops the call."""
    err = []

    def tramp(_ctx, p, first, end):
        try:
            c = p.contents
            chunk = DevicePaths(c) if c.on_device else HostPaths(c, owned=False)
            return 1 if on_chunk(chunk, int(first), int(end)) else 0
        except BaseException as e:  # surfaced after the call returns
            err.append(e)
            return 1
    cb = _CHUNK_FN(tramp)
    o.on_chunk = cb
    rc = fn(*args)
    if err:
        raise err[0]
    _check(rc)


def prime_paths_vertex_lists(g: Graph, ws: Optional[Workspace] = None, flags: int = 0,
                             stream=None, pool_cap: int = 0):
    """(paths, stats) by the paper's per-vertex schedule: prime paths grouped
    by last vertex, by length inside a group."""
    st = _Stats()
    o = _opts(ws, flags, stream, st, pool_cap)
    out = _Paths()
    _check(lib().tpg_prime_paths_vertex_lists(g.handle, ctypes.byref(o), ctypes.byref(out)))
    return _wrap(out), _stats_dict(st)


def scc(g: Graph, ws: Optional[Workspace] = None, stream=None):
    """(comp int32 [n], flags uint8 [n], n_comp): the smallest vertex of each
    vertex's strongly connected component and its TPG_SCC_* flags."""
    n = g.info()[0]
    comp = np.zeros(max(n, 1), np.int32)
    fl = np.zeros(max(n, 1), np.uint8)
    nc = ctypes.c_int32(0)
    o = _opts(ws, 0, stream, None, 0)
    _check(lib().tpg_scc(g.handle, ctypes.byref(o), comp.ctypes.data, fl.ctypes.data,
                         ctypes.byref(nc)))
    return comp[:n], fl[:n], int(nc.value)


def prime_path_types(g: Graph, pps, ws: Optional[Workspace] = None, stream=None,
                     want_types: bool = True):
    """(types uint8 [n] or None, counts int64 [6]) of a prime-path set of g:
    HostPaths / anything with offsets and vertices arrays (host), or
    DevicePaths (read in place on the device)."""
    p = _Paths()
    if isinstance(pps, DevicePaths):
        p.n_paths, p.n_vertices = pps.n_paths, pps.n_vertices
        p.offsets, p.vertices, p.on_device = pps.offsets_ptr, pps.vertices_ptr, 1
        keep = None
    else:
        off = np.ascontiguousarray(pps.offsets, dtype=np.int64)
        vtx = np.ascontiguousarray(pps.vertices, dtype=np.int32)
        keep = (off, vtx)
        p.n_paths, p.n_vertices = len(off) - 1, len(vtx)
        p.offsets, p.vertices, p.on_device = off.ctypes.data, vtx.ctypes.data, 0
    n = int(p.n_paths)
    types = np.zeros(max(n, 1), np.uint8) if want_types else None
    counts = np.zeros(6, np.int64)
    o = _opts(ws, 0, stream, None, 0)
    _check(lib().tpg_prime_path_types(g.handle, ctypes.byref(p), ctypes.byref(o),
                                      types.ctypes.data if want_types else None,
                                      counts.ctypes.data))
    del keep
    return (types[:n] if want_types else None), counts


def ccfg(g: Graph, ws: Optional[Workspace] = None, stream=None):
    """(comp int32 [n], n_comp, arcs int32 [k, 2]): component labels and the
    component graph's arcs (arcs of g between components, CSR order)."""
    n, m = g.info()[0], g.info()[1]
    comp = np.zeros(max(n, 1), np.int32)
    nc = ctypes.c_int32(0)
    na = ctypes.c_int64(0)
    src = np.zeros(max(m, 1), np.int32)
    dst = np.zeros(max(m, 1), np.int32)
    o = _opts(ws, 0, stream, None, 0)
    _check(lib().tpg_ccfg(g.handle, ctypes.byref(o), comp.ctypes.data, ctypes.byref(nc),
                          ctypes.byref(na), src.ctypes.data, dst.ctypes.data, len(src)))
    k = int(na.value)
    return comp[:n], int(nc.value), np.stack([src[:k], dst[:k]], axis=1)


def scc_paths(g: Graph, ws: Optional[Workspace] = None, flags: int = 0, stream=None):
    """(entry_exit, exit_paths, entry_paths) of the components with a cycle
    (Defs. 6-8): HostPaths, or DevicePaths with TPG_OUT_DEVICE."""
    outs = [_Paths(), _Paths(), _Paths()]
    o = _opts(ws, flags, stream, None, 0)
    _check(lib().tpg_scc_paths(g.handle, ctypes.byref(o), *[ctypes.byref(x) for x in outs]))
    return tuple(_wrap(x) for x in outs)


def scc_internal_pps(g: Graph, ws: Optional[Workspace] = None, flags: int = 0, stream=None):
    """SccInternalPPs from the extension on each component with a cycle
    alone (Def. 9), grouped by component."""
    out = _Paths()
    o = _opts(ws, flags, stream, None, 0)
    _check(lib().tpg_scc_internal_pps(g.handle, ctypes.byref(o), ctypes.byref(out)))
    return _wrap(out)


def merged_pps(g: Graph, ws: Optional[Workspace] = None, flags: int = 0, stream=None):
    """(complete, scc_exit, scc_entry) prime paths merged as in Sec. 2.1."""
    outs = [_Paths(), _Paths(), _Paths()]
    o = _opts(ws, flags, stream, None, 0)
    _check(lib().tpg_merged_pps(g.handle, ctypes.byref(o), *[ctypes.byref(x) for x in outs]))
    return tuple(_wrap(x) for x in outs)


def prime_path_types_noalloc(g: Graph, pps, types=None, stream=None) -> np.ndarray:
    """counts int64 [6] of a device prime-path set of g (DevicePaths), and
    each path's type into `types` (a uint8 device tensor of >= n_paths
    elements, or None), without any device allocation by the library."""
    if not isinstance(pps, DevicePaths):
        raise TypeError("prime_path_types_noalloc takes a device path set (DevicePaths)")
    n = int(pps.n_paths)
    if types is not None:
        assert types.dtype.itemsize == 1 and types.numel() >= n and types.is_contiguous()
    counts = np.zeros(6, np.int64)
    st = int(getattr(stream, "cuda_stream", stream or 0))
    _check(lib().tpg_prime_path_types_noalloc(
        g.handle, pps.offsets_ptr, pps.vertices_ptr, n, st or None,
        types.data_ptr() if types is not None else None, counts.ctypes.data))
    return counts


def prime_paths_stream(g: Graph, on_chunk, ws: Optional[Workspace] = None, flags: int = 0,
                       stream=None, chunk_vertices: int = 0, pool_cap: int = 0):
    """Prime paths delivered first-vertex range by range (TPG_STREAM):
    on_chunk(chunk, first, end) gets the prime paths whose first vertex lies
    in [first, end), in canonical order.  Returns (SetDigest of the whole
    set, stats)."""
    st = _Stats()
    o = _opts(ws, flags | TPG_STREAM, stream, st, pool_cap)
    o.chunk_vertices = int(chunk_vertices)
    out = _Paths()
    _stream_call(lib().tpg_prime_paths, on_chunk, o, g.handle, ctypes.byref(o), ctypes.byref(out))
    return SetDigest(out), _stats_dict(st)


def test_paths_stream(g: Graph, on_chunk, ws: Optional[Workspace] = None, flags: int = 0,
                      stream=None, chunk_paths: int = 0, pool_cap: int = 0):
    """Test paths delivered in chunks of chunk_paths (TPG_STREAM):
    on_chunk(chunk, first, end) gets canonical test paths [first, end).
    Returns (SetDigest of the prime paths, SetDigest of the test paths,
    stats)."""
    st = _Stats()
    o = _opts(ws, flags | TPG_STREAM, stream, st, pool_cap)
    o.chunk_paths = int(chunk_paths)
    pp, tp = _Paths(), _Paths()
    _stream_call(lib().tpg_test_paths, on_chunk, o, g.handle, ctypes.byref(o), ctypes.byref(pp),
                 ctypes.byref(tp))
    return SetDigest(pp), SetDigest(tp), _stats_dict(st)


def version() -> str:
    return lib().tpg_version().decode()


def device_count() -> int:
    return int(lib().tpg_device_count())


class BatchResult:
    """Packed results of a batched call: prime and test paths of graph i are
    pp[pp_first[i]:pp_first[i+1]] and tp[tp_first[i]:tp_first[i+1]]."""

    def __init__(self, r: _BatchResult) -> None:
        n = r.n_graphs
        self.n_graphs = n
        self.pp_first = np.ctypeslib.as_array(r.pp_first, shape=(n + 1,)).copy()
        self.tp_first = np.ctypeslib.as_array(r.tp_first, shape=(n + 1,)).copy()
        self.on_device = bool(r.pp.on_device)
        if self.on_device:
            self.pp = DevicePaths(r.pp)
            self.tp = DevicePaths(r.tp)
            # the paths are views into the workspace; release the index arrays only
            r.pp = _Paths()
            r.tp = _Paths()
            lib().tpg_batch_result_free(ctypes.byref(r))
        else:
            pp, tp = _Paths(), _Paths()
            ctypes.memmove(ctypes.byref(pp), ctypes.byref(r.pp), ctypes.sizeof(_Paths))
            ctypes.memmove(ctypes.byref(tp), ctypes.byref(r.tp), ctypes.sizeof(_Paths))
            r.pp = _Paths()
            r.tp = _Paths()
            lib().tpg_batch_result_free(ctypes.byref(r))
            self.pp = HostPaths(pp)
            self.tp = HostPaths(tp)

    def graph(self, i: int):
        """(prime paths, test paths) of graph i as host (offsets, vertices)."""
        def cut(pl, first):
            a, b = int(first[i]), int(first[i + 1])
            off = pl.offsets[a:b + 1]
            return off - off[0], pl.vertices[off[0]:off[-1]]
        return cut(self.pp, self.pp_first), cut(self.tp, self.tp_first)


def batch_test_paths(graphs, ws: Optional[Workspace] = None, flags: int = 0, stream=None,
                     pool_cap: int = 0, predicted: Optional[np.ndarray] = None,
                     level_counts: Optional[np.ndarray] = None):
    """(BatchResult, stats) for a list of Graph.  predicted: float32
    [n, 65] log1p sizes; level_counts: int64 [n, 64] receives the per-graph
    path counts of levels 1..64."""
    n = len(graphs)
    arr = (ctypes.c_void_p * n)(*[g.handle.value for g in graphs])
    st = _Stats()
    lv = None
    if level_counts is not None:
        assert level_counts.dtype == np.int64 and level_counts.size >= 64 * n
        lv = level_counts.reshape(-1)
    o = _opts(ws, flags, stream, st, pool_cap, lv)
    pred_ptr = None
    if predicted is not None:
        predicted = np.ascontiguousarray(predicted, dtype=np.float32)
        assert predicted.shape == (n, 65)
        pred_ptr = predicted.ctypes.data
    r = _BatchResult()
    _check(lib().tpg_batch_test_paths(arr, n, ctypes.byref(o), pred_ptr, ctypes.byref(r)))
    return BatchResult(r), _stats_dict(st)


MLP_IN, MLP_OUT = 32, 65


def features(graphs) -> np.ndarray:
    """[n, 32] float32 structural features (computed by the library)."""
    n = len(graphs)
    arr = (ctypes.c_void_p * n)(*[g.handle.value for g in graphs])
    out = np.zeros((n, MLP_IN), np.float32)
    _check(lib().tpg_features(arr, n, out.ctypes.data))
    return out


def _f32(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float32)
    assert a.shape == shape, (a.shape, shape)
    return a


class MLP:
    """Size predictor on the GPU (see tpg_mlp_* in include/tpg.h)."""

    def __init__(self, device: int = -1, seed: int = 0, _handle=None) -> None:
        if _handle is None:
            h = ctypes.c_void_p()
            _check(lib().tpg_mlp_create(int(device), int(seed), ctypes.byref(h)))
            _handle = h
        self._h = _handle

    @staticmethod
    def num_params() -> int:
        return int(lib().tpg_mlp_num_params())

    @classmethod
    def load(cls, path: str, device: int = -1) -> "MLP":
        h = ctypes.c_void_p()
        _check(lib().tpg_mlp_load(int(device), path.encode(), ctypes.byref(h)))
        return cls(_handle=h)

    def save(self, path: str) -> None:
        _check(lib().tpg_mlp_save(self._h, path.encode()))

    def params(self) -> np.ndarray:
        p = np.zeros(self.num_params(), np.float32)
        _check(lib().tpg_mlp_get_params(self._h, p.ctypes.data))
        return p

    def set_params(self, p: np.ndarray) -> None:
        p = _f32(p, (self.num_params(),))
        _check(lib().tpg_mlp_set_params(self._h, p.ctypes.data))

    def set_normalizer(self, mean: np.ndarray, std: np.ndarray) -> None:
        mean, std = _f32(mean, (MLP_IN,)), _f32(std, (MLP_IN,))
        _check(lib().tpg_mlp_set_normalizer(self._h, mean.ctypes.data, std.ctypes.data))

    def forward(self, x: np.ndarray) -> np.ndarray:
        x = _f32(x, (len(x), MLP_IN))
        y = np.zeros((len(x), MLP_OUT), np.float32)
        _check(lib().tpg_mlp_forward(self._h, x.ctypes.data, len(x), y.ctypes.data))
        return y

    def gradients(self, x: np.ndarray, t: np.ndarray):
        x = _f32(x, (len(x), MLP_IN))
        t = _f32(t, (len(x), MLP_OUT))
        g = np.zeros(self.num_params(), np.float32)
        loss = ctypes.c_float()
        _check(lib().tpg_mlp_gradients(self._h, x.ctypes.data, t.ctypes.data, len(x),
                                       g.ctypes.data, ctypes.byref(loss)))
        return g, float(loss.value)

    def train_step(self, x: np.ndarray, t: np.ndarray, lr: float) -> float:
        x = _f32(x, (len(x), MLP_IN))
        t = _f32(t, (len(x), MLP_OUT))
        loss = ctypes.c_float()
        _check(lib().tpg_mlp_train_step(self._h, x.ctypes.data, t.ctypes.data, len(x),
                                        float(lr), ctypes.byref(loss)))
        return float(loss.value)

    def close(self) -> None:
        if self._h:
            lib().tpg_mlp_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _tuning_dict(tu: _Tuning) -> Dict[str, list]:
    return {"items": list(tu.items), "wgs_per_cu": list(tu.wgs_per_cu),
            "variant": list(tu.variant), "best_ms": list(tu.best_ms)}


def autotune(graphs, ws: Workspace, stream=None) -> Dict[str, list]:
    """Times the extension kernel's launch shapes on these graphs and keeps
    the fastest per visited-set width in `ws`."""
    n = len(graphs)
    arr = (ctypes.c_void_p * n)(*[g.handle.value for g in graphs])
    o = _opts(ws, 0, stream, None)
    tu = _Tuning()
    _check(lib().tpg_autotune(arr, n, ctypes.byref(o), ctypes.byref(tu)))
    return _tuning_dict(tu)


def get_tuning(ws: Workspace) -> Dict[str, list]:
    tu = _Tuning()
    _check(lib().tpg_workspace_get_tuning(ws.handle, ctypes.byref(tu)))
    return _tuning_dict(tu)


def set_tuning(ws: Workspace, t: Dict[str, list]) -> None:
    tu = _Tuning()
    for i in range(7):
        tu.items[i] = int(t["items"][i])
        tu.wgs_per_cu[i] = int(t["wgs_per_cu"][i])
        tu.variant[i] = int(t.get("variant", [0] * 7)[i])
        tu.best_ms[i] = float(t.get("best_ms", [0.0] * 7)[i])
    _check(lib().tpg_workspace_set_tuning(ws.handle, ctypes.byref(tu)))
