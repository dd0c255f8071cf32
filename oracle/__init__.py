"""CPU oracle for prime paths and test paths (ctypes binding to oracle.cpp).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It
shares no code with the GPU engine.

The C++ source states which passage of the paper each routine follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, List, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.cpp with g++ (host only)."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-shared", "-fPIC",
                               "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Paths(ctypes.Structure):
    _fields_ = [("n_paths", ctypes.c_int64), ("n_vertices", ctypes.c_int64),
                ("offsets", ctypes.POINTER(ctypes.c_int64)),
                ("vertices", ctypes.POINTER(ctypes.c_int32))]


class _Stats(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_int64), ("n_cycles", ctypes.c_int64),
                ("n_extensions", ctypes.c_int64), ("n_pp", ctypes.c_int64),
                ("n_pp_local", ctypes.c_int64), ("max_len", ctypes.c_int64)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        i64p, i32p = P(ctypes.c_int64), P(ctypes.c_int32)
        _lib.orc_prime_paths.argtypes = [ctypes.c_int, i64p, i32p, ctypes.c_int,
                                         P(_Paths), P(_Stats), i64p, i64p]
        _lib.orc_prime_paths_local.argtypes = [ctypes.c_int, i64p, i32p, ctypes.c_int,
                                               ctypes.c_int, ctypes.c_int, P(_Paths),
                                               P(_Stats)]
        _lib.orc_count.argtypes = [ctypes.c_int, i64p, i32p, ctypes.c_int,
                                   ctypes.c_int64, P(_Stats), i64p, i64p, i64p]
        _lib.orc_bruteforce_pp.argtypes = [ctypes.c_int, i64p, i32p, P(_Paths), P(_Paths)]
        _lib.orc_bfs.argtypes = [ctypes.c_int, i64p, i32p, ctypes.c_int, ctypes.c_int,
                                 i32p, i32p, i32p, i32p]
        _lib.orc_bruteforce_lexmin_shortest.argtypes = [ctypes.c_int, i64p, i32p,
                                                        ctypes.c_int, ctypes.c_int, i32p,
                                                        ctypes.c_int]
        _lib.orc_test_paths.argtypes = [ctypes.c_int, i64p, i32p, ctypes.c_int,
                                        ctypes.c_int, P(_Paths), P(_Paths), i64p]
        _lib.orc_free_paths.argtypes = [P(_Paths)]
        _lib.orc_test_paths_greedy.argtypes = [ctypes.c_int, i64p, i32p, ctypes.c_int,
                                               ctypes.c_int, P(_Paths), P(_Paths)]
        _lib.orc_fnv1a64.argtypes = [ctypes.c_char_p, ctypes.c_int64]
        _lib.orc_fnv1a64.restype = ctypes.c_uint64
        _lib.orc_digest.argtypes = [ctypes.c_int64, i64p, i32p, P(ctypes.c_uint64)]
        _lib.orc_set_digests.argtypes = [ctypes.c_int, i64p, i32p, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, i64p,
                                         P(ctypes.c_uint64), i64p, i64p, P(ctypes.c_uint64)]
    return _lib


class PathList:
    """A canonical path set: offsets int64 [n+1], vertices int32 [total]."""

    def __init__(self, offsets: np.ndarray, vertices: np.ndarray) -> None:
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self.vertices = np.ascontiguousarray(vertices, dtype=np.int32)

    def __len__(self) -> int:
        return len(self.offsets) - 1

    def __getitem__(self, i: int) -> List[int]:
        return self.vertices[self.offsets[i]:self.offsets[i + 1]].tolist()

    def tolist(self) -> List[List[int]]:
        return [self[i] for i in range(len(self))]

    @staticmethod
    def from_lists(paths: List[List[int]]) -> "PathList":
        offs = np.zeros(len(paths) + 1, dtype=np.int64)
        offs[1:] = np.cumsum([len(p) for p in paths]) if paths else []
        verts = np.array([v for p in paths for v in p], dtype=np.int32)
        return PathList(offs, verts)

    def _c(self) -> _Paths:
        return _Paths(len(self), len(self.vertices),
                      self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                      self.vertices.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))


def _take(p: _Paths) -> PathList:
    n, nv = p.n_paths, p.n_vertices
    offs = np.ctypeslib.as_array(p.offsets, shape=(n + 1,)).copy()
    verts = (np.ctypeslib.as_array(p.vertices, shape=(nv,)).copy() if nv
             else np.zeros(0, np.int32))
    _load().orc_free_paths(ctypes.byref(p))
    return PathList(offs, verts)


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, np.int32)
    return (rp, ci, rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            ci.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))


def _stats(s: _Stats) -> Dict[str, int]:
    return {k: int(getattr(s, k)) for k, _ in _Stats._fields_}


def _threads(nthreads: Optional[int]) -> int:
    return int(nthreads if nthreads is not None else min(16, os.cpu_count() or 1))


def prime_paths(g, nthreads: Optional[int] = None
                ) -> Tuple[PathList, Dict[str, int], np.ndarray, np.ndarray]:
    """PPs in canonical order, stats, per-level acyclic counts, cycle counts."""
    lib = _load()
    rp, ci, prp, pci = _csr(g)
    out, st = _Paths(), _Stats()
    lv = np.zeros(g.n + 2, np.int64)
    cy = np.zeros(g.n + 2, np.int64)
    lib.orc_prime_paths(g.n, prp, pci, _threads(nthreads), ctypes.byref(out),
                        ctypes.byref(st), lv.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                        cy.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return _take(out), _stats(st), lv, cy


def prime_paths_local(g, s_lo: int, s_hi: int, nthreads: Optional[int] = None
                      ) -> Tuple[PathList, Dict[str, int]]:
    """PPs whose first vertex lies in [s_lo, s_hi), by the local rule."""
    lib = _load()
    rp, ci, prp, pci = _csr(g)
    out, st = _Paths(), _Stats()
    lib.orc_prime_paths_local(g.n, prp, pci, s_lo, s_hi, _threads(nthreads),
                              ctypes.byref(out), ctypes.byref(st))
    return _take(out), _stats(st)


def count(g, nthreads: Optional[int] = None, ext_cap: int = 0, per_start: bool = False):
    """Per-level counts and the PP count without storing paths.  With
    ext_cap > 0, returns (None, ...) once about ext_cap extensions are
    exceeded.  per_start=True appends the PP count of every first vertex."""
    lib = _load()
    rp, ci, prp, pci = _csr(g)
    st = _Stats()
    lv = np.zeros(g.n + 2, np.int64)
    cy = np.zeros(g.n + 2, np.int64)
    ps = np.zeros(g.n, np.int64)
    rc = lib.orc_count(g.n, prp, pci, _threads(nthreads), int(ext_cap), ctypes.byref(st),
                       lv.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                       cy.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                       ps.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    res = (None if rc == 1 else _stats(st), lv, cy)
    return res + (ps,) if per_start else res


def bruteforce_pp(g) -> Tuple[PathList, PathList]:
    """(prime paths, all simple paths), straight from the definitions."""
    lib = _load()
    rp, ci, prp, pci = _csr(g)
    out, allp = _Paths(), _Paths()
    rc = lib.orc_bruteforce_pp(g.n, prp, pci, ctypes.byref(out), ctypes.byref(allp))
    if rc != 0:
        raise ValueError("graph too large for brute force (<= 32 vertices, "
                         "<= 60000 simple paths)")
    return _take(out), _take(allp)


def bfs_tables(g) -> Dict[str, np.ndarray]:
    lib = _load()
    rp, ci, prp, pci = _csr(g)
    arrs = {k: np.zeros(g.n, np.int32) for k in ("dist_f", "parent", "dist_b", "next")}
    ptr = {k: v.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) for k, v in arrs.items()}
    lib.orc_bfs(g.n, prp, pci, g.entry, g.exit, ptr["dist_f"], ptr["parent"],
                ptr["dist_b"], ptr["next"])
    return arrs


def bruteforce_lexmin_shortest(g, a: int, b: int) -> Optional[List[int]]:
    lib = _load()
    rp, ci, prp, pci = _csr(g)
    buf = np.zeros(g.n + 1, np.int32)
    k = lib.orc_bruteforce_lexmin_shortest(g.n, prp, pci, a, b,
                                           buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                           g.n + 1)
    if k == -1:
        return None
    if k < 0:
        raise ValueError("graph too large for exhaustive shortest paths")
    return buf[:k].tolist()


def test_paths(g, pps: PathList) -> Tuple[PathList, int]:
    """(deduplicated sorted TPs, number spliced before dedup)."""
    lib = _load()
    rp, ci, prp, pci = _csr(g)
    src = pps._c()
    out = _Paths()
    nb = ctypes.c_int64(0)
    rc = lib.orc_test_paths(g.n, prp, pci, g.entry, g.exit, ctypes.byref(src),
                            ctypes.byref(out), ctypes.byref(nb))
    if rc != 0:
        raise ValueError("a prime path is not reachable from entry or cannot reach exit")
    return _take(out), int(nb.value)


def binarize(g):
    """The paper's input form (Sec. 3): a vertex of out-degree k > 2 keeps its
    first (smallest) successor and passes the others to a chain of k - 2 new
    decision vertices, numbered from n upward in vertex order; chain vertex i
    leads to successor i + 1 and to the next chain vertex, the last one to the
    two largest successors.  Returns a graph with the same entry and exit."""
    from paper_2210_16998_amd.cfggen import from_edges
    rp, ci = np.asarray(g.row_ptr), np.asarray(g.col_idx)
    edges, nid = [], g.n
    for v in range(g.n):
        succ = sorted(set(int(w) for w in ci[rp[v]:rp[v + 1]]))
        if len(succ) <= 2:
            edges += [(v, w) for w in succ]
            continue
        at = v
        for i in range(len(succ) - 2):
            edges += [(at, succ[i]), (at, nid)]
            at = nid
            nid += 1
        edges += [(at, succ[-2]), (at, succ[-1])]
    return from_edges(nid, edges, g.entry, g.exit, name=f"{g.name}_bin")


def group_by_last(pl: PathList) -> PathList:
    """Prime paths grouped by last vertex: ascending last vertex, the given
    (canonical) order inside a group."""
    order = sorted(range(len(pl)), key=lambda i: (int(pl.vertices[pl.offsets[i + 1] - 1]), i))
    rows = [pl.vertices[pl.offsets[i]:pl.offsets[i + 1]] for i in order]
    off = np.cumsum([0] + [len(r) for r in rows]).astype(np.int64)
    return PathList(off, np.concatenate(rows) if rows else np.zeros(0, np.int32))


def fnv1a64(data: bytes) -> int:
    """64-bit FNV-1a of a byte string."""
    return int(_load().orc_fnv1a64(data, len(data)))


def digest(pl: PathList) -> Tuple[int, int]:
    """Order-independent set digest: (sum mod 2^64, xor) of the FNV-1a 64
    hashes of each path's little-endian int32 bytes (k, v_1 .. v_k)."""
    out = (ctypes.c_uint64 * 2)()
    off = np.ascontiguousarray(pl.offsets, dtype=np.int64)
    vtx = np.ascontiguousarray(pl.vertices, dtype=np.int32)
    if vtx.size == 0:
        vtx = np.zeros(1, np.int32)
    _load().orc_digest(len(off) - 1, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                       vtx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), out)
    return int(out[0]), int(out[1])


def set_digests(g, n_buckets: int = 4, nthreads: Optional[int] = None) -> Dict[str, object]:
    """Whole-set figures without holding the sets: per-first-vertex prime
    path counts, the prime paths' set digest, and the test paths' count
    (after exact deduplication in hash buckets) and set digest.  For graphs
    whose test paths do not fit in memory at once."""
    lib = _load()
    rp, ci, prp, pci = _csr(g)
    per = np.zeros(g.n, np.int64)
    ppd = (ctypes.c_uint64 * 2)()
    tpd = (ctypes.c_uint64 * 2)()
    ntp = np.zeros(1, np.int64)
    nsp = np.zeros(1, np.int64)
    i64 = ctypes.POINTER(ctypes.c_int64)
    rc = lib.orc_set_digests(g.n, prp, pci, g.entry, g.exit, _threads(nthreads), int(n_buckets),
                             per.ctypes.data_as(i64), ppd, ntp.ctypes.data_as(i64),
                             nsp.ctypes.data_as(i64), tpd)
    if rc != 0:
        raise ValueError("a prime path is not reachable from entry or cannot reach exit")
    return {"pp_per_start": per, "n_pp": int(per.sum()), "pp_digest": (int(ppd[0]), int(ppd[1])),
            "n_tp": int(ntp[0]), "n_spliced": int(nsp[0]), "tp_digest": (int(tpd[0]), int(tpd[1]))}


def test_paths_greedy(g, pps: PathList) -> PathList:
    """Test paths by the longest-first covering (see oracle.cpp): a prime
    path already contained in a chosen test path gets no test path of its
    own.  Small graphs only (every simple window of every chosen path is
    looked up)."""
    lib = _load()
    rp, ci, prp, pci = _csr(g)
    inp = pps._c()
    out = _Paths()
    rc = lib.orc_test_paths_greedy(g.n, prp, pci, g.entry, g.exit, ctypes.byref(inp),
                                   ctypes.byref(out))
    if rc != 0:
        raise ValueError("a prime path is not reachable from the entry or cannot reach the exit")
    return _take(out)


# --- strongly connected components and the paper's path types -------------
# Types of a prime path (Sec. 2): Def. 2 CompletePP, Def. 9 SccInternalPP,
# Def. 10 SccExitPP, Def. 11 SccEntryPP; OTHER for none of them.
PP_COMPLETE, PP_SCC_INTERNAL, PP_SCC_EXIT, PP_SCC_ENTRY, PP_OTHER = 1, 2, 3, 4, 5
# Per-vertex flags: in a component with a cycle (two or more vertices, or a
# self-loop); SccEntryVertex (Def. 4: a predecessor outside its component);
# SccExitVertex (Def. 5: a successor outside its component).
SCC_CYCLIC, SCC_ENTRY_VERTEX, SCC_EXIT_VERTEX = 1, 2, 4


def scc(g) -> np.ndarray:
    """Strongly connected components (Sec. 2; Tarjan's depth-first algorithm,
    written with an explicit stack): scc[v] = the smallest vertex of v's
    component, so that the labelling is unique."""
    n = g.n
    index, low, on = [-1] * n, [0] * n, [False] * n
    stack, out, nxt = [], np.full(n, -1, np.int32), 0
    for root in range(n):
        if index[root] >= 0:
            continue
        index[root] = low[root] = nxt
        nxt += 1
        stack.append(root)
        on[root] = True
        work = [[root, 0]]
        while work:
            v, i = work[-1]
            succ = g.succ(v)
            if i < len(succ):
                work[-1][1] += 1
                w = int(succ[i])
                if index[w] < 0:
                    index[w] = low[w] = nxt
                    nxt += 1
                    stack.append(w)
                    on[w] = True
                    work.append([w, 0])
                elif on[w]:
                    low[v] = min(low[v], index[w])
                continue
            work.pop()
            if work:
                u = work[-1][0]
                low[u] = min(low[u], low[v])
            if low[v] == index[v]:
                comp = []
                while True:
                    w = stack.pop()
                    on[w] = False
                    comp.append(w)
                    if w == v:
                        break
                out[comp] = min(comp)
    return out


def scc_flags(g, comp: np.ndarray) -> np.ndarray:
    """Per-vertex SCC_CYCLIC / SCC_ENTRY_VERTEX / SCC_EXIT_VERTEX bits."""
    size = np.bincount(comp, minlength=g.n)
    fl = np.zeros(g.n, np.uint8)
    for v in range(g.n):
        for w in g.succ(v):
            w = int(w)
            if w == v:
                fl[v] |= SCC_CYCLIC
            if comp[w] != comp[v]:
                fl[v] |= SCC_EXIT_VERTEX
                fl[w] |= SCC_ENTRY_VERTEX
        if size[comp[v]] >= 2:
            fl[v] |= SCC_CYCLIC
    return fl


def ccfg(g, comp: np.ndarray):
    """Def. 3: the component graph, as a set of arcs between component
    labels (the arcs of g whose ends lie in different components)."""
    return sorted({(int(comp[v]), int(comp[w])) for v in range(g.n) for w in g.succ(v)
                   if comp[v] != comp[int(w)]})


def pp_types(g, pl: PathList) -> Tuple[np.ndarray, np.ndarray]:
    """Type of each prime path by Defs. 2, 9, 10 and 11 (first match), and the
    count of each type (index = type).  Def. 9 is read literally: start and
    end in one component with a cycle; an acyclic one must not start at an
    SccEntryVertex nor end at an SccExitVertex."""
    comp = scc(g)
    fl = scc_flags(g, comp)
    types = np.zeros(len(pl), np.uint8)
    for i in range(len(pl)):
        p = pl[i]
        a, b = p[0], p[-1]
        cyclic = len(p) > 1 and a == b
        if a == g.entry and b == g.exit:
            t = PP_COMPLETE
        elif (fl[a] & SCC_CYCLIC) and comp[a] == comp[b] and (
                cyclic or not (fl[a] & SCC_ENTRY_VERTEX or fl[b] & SCC_EXIT_VERTEX)):
            t = PP_SCC_INTERNAL
        elif (fl[a] & SCC_CYCLIC) and b == g.exit:
            t = PP_SCC_EXIT
        elif a == g.entry and (fl[b] & SCC_CYCLIC):
            t = PP_SCC_ENTRY
        else:
            t = PP_OTHER
        types[i] = t
    return types, np.bincount(types, minlength=6).astype(np.int64)


def _is_subpath(p: List[int], q: List[int]) -> bool:
    """p is a contiguous subpath of q (reading R1: subpaths are contiguous)."""
    m = len(p)
    return any(q[k:k + m] == p for k in range(len(q) - m + 1))


def _component_paths(g, comp: np.ndarray, c: int) -> List[List[int]]:
    """Every acyclic simple path that stays inside component c (depth-first
    from each of its vertices, successors inside c only)."""
    members = [v for v in range(g.n) if comp[v] == c]
    out: List[List[int]] = []
    for s in members:
        stack = [(s, [s])]
        while stack:
            v, path = stack.pop()
            out.append(path)
            for w in reversed(g.succ(v).tolist()):
                if comp[w] == c and w not in path:
                    stack.append((w, path + [w]))
    return out


def scc_path_sets(g) -> Dict[str, PathList]:
    """The intermediate paths of the compositional method (Sec. 2.1, Path
    extraction), over every component with a cycle, from Defs. 6-8:

    * entry_exit (Def. 6): acyclic simple paths inside a component from one
      of its SccEntryVertices to one of its SccExitVertices;
    * exit (Def. 7): exit paths (acyclic, inside a component, from a vertex
      that is not an SccEntryVertex to an SccExitVertex) that are not a
      proper subpath of another exit path to the same SccExitVertex;
    * entry (Def. 8): entry paths (acyclic, inside a component, from an
      SccEntryVertex to a vertex that is not an SccExitVertex) that are not a
      proper subpath of another entry path from the same SccEntryVertex.

    Maximality is taken per end vertex, as the extraction algorithms of
    Sec. 2.1 are stated for a specified exit (entry) vertex; on Fig. 1 it
    gives the same paths as maximality over all exit (entry) paths.  Each set
    in canonical (lexicographic) order."""
    comp = scc(g)
    fl = scc_flags(g, comp)
    ee: List[List[int]] = []
    ex: List[List[int]] = []
    en: List[List[int]] = []
    for c in sorted({int(x) for x in comp}):
        if not fl[c] & SCC_CYCLIC:
            continue
        paths = _component_paths(g, comp, c)
        ee += [p for p in paths if fl[p[0]] & SCC_ENTRY_VERTEX and fl[p[-1]] & SCC_EXIT_VERTEX]
        xc = [p for p in paths if not fl[p[0]] & SCC_ENTRY_VERTEX and fl[p[-1]] & SCC_EXIT_VERTEX]
        ex += [p for p in xc if not any(len(q) > len(p) and q[-1] == p[-1] and _is_subpath(p, q)
                                        for q in xc)]
        nc = [p for p in paths if fl[p[0]] & SCC_ENTRY_VERTEX and not fl[p[-1]] & SCC_EXIT_VERTEX]
        en += [p for p in nc if not any(len(q) > len(p) and q[0] == p[0] and _is_subpath(p, q)
                                        for q in nc)]
    return {k: PathList.from_lists(sorted(v)) for k, v in
            (("entry_exit", ee), ("exit", ex), ("entry", en))}


def ccfg_paths(g) -> List[List[int]]:
    """Prime paths of the component graph (Def. 3): it is acyclic with one
    source (the entry's component) and one sink (the exit's), so they are its
    paths from source to sink, as sequences of component labels."""
    comp = scc(g)
    arcs = ccfg(g, comp)
    succ: Dict[int, List[int]] = {}
    for a, b in arcs:
        succ.setdefault(a, []).append(b)
    src, dst = int(comp[g.entry]), int(comp[g.exit])
    out: List[List[int]] = []
    stack = [[src]]
    while stack:
        p = stack.pop()
        if p[-1] == dst:
            out.append(p)
            continue
        for b in sorted(succ.get(p[-1], []), reverse=True):
            stack.append(p + [b])
    return sorted(out)


def _is_prime(g, p: List[int], preds: List[List[int]]) -> bool:
    """p (a simple path or simple cycle) cannot be extended at either end."""
    if len(p) > 1 and p[0] == p[-1]:
        return True
    on = set(p)
    fwd = any(int(w) not in on or int(w) == p[0] for w in g.succ(p[-1]))
    bwd = any(u not in on or u == p[-1] for u in preds[p[0]])
    return not fwd and not bwd


def merge_pps(g) -> Dict[str, object]:
    """Sec. 2.1, Merging: the CompletePPs, SccExitPPs and SccEntryPPs built
    from the component graph's prime paths and the extracted paths.

    * complete: each component-graph path with every component replaced by
      one of its paths that the arcs of g join to its neighbours (the entry's
      and exit's components are single vertices; a component without a cycle
      contributes its vertex; a component with a cycle one of its
      SccEntryExitPaths);
    * exit: for each complete path and each component with a cycle it
      leaves, at SccExitVertex x, the path's rest from x, prefixed by every
      SccExitPath of that component that ends at x;
    * entry: for each complete path and each component with a cycle it
      enters, at SccEntryVertex y, the path's part before y, followed by
      every SccEntryPath of that component that starts at y.

    A merged path that can still be extended at one of its ends (this
    happens when an exit path's first vertex has a predecessor, necessarily
    an SccEntryVertex, off the path, or an entry path's last vertex a
    successor, necessarily an SccExitVertex, off it) is not a prime path and
    is dropped; the numbers dropped are returned too (none on Fig. 1)."""
    comp = scc(g)
    fl = scc_flags(g, comp)
    sets = scc_path_sets(g)
    preds: List[List[int]] = [[] for _ in range(g.n)]
    for v in range(g.n):
        for w in g.succ(v):
            preds[int(w)].append(v)
    arc = {(v, int(w)) for v in range(g.n) for w in g.succ(v)}
    ee_by_comp: Dict[int, List[List[int]]] = {}
    for p in sets["entry_exit"].tolist():
        ee_by_comp.setdefault(int(comp[p[0]]), []).append(p)
    ex_by_end: Dict[int, List[List[int]]] = {}
    for p in sets["exit"].tolist():
        ex_by_end.setdefault(p[-1], []).append(p)
    en_by_start: Dict[int, List[List[int]]] = {}
    for p in sets["entry"].tolist():
        en_by_start.setdefault(p[0], []).append(p)

    def pieces(c: int) -> List[List[int]]:
        if fl[c] & SCC_CYCLIC:
            return ee_by_comp.get(c, [])
        return [[c]]  # a component without a cycle is its one vertex (label = vertex)

    complete: List[List[int]] = []
    for cp in ccfg_paths(g):
        partial = [[]]
        for c in cp:
            nxt = []
            for pre in partial:
                for piece in pieces(c):
                    if not pre or (pre[-1], piece[0]) in arc:
                        nxt.append(pre + piece)
            partial = nxt
        complete += partial
    complete = sorted({tuple(p) for p in complete})
    cand_ex, cand_en = set(), set()
    for p in complete:
        p = list(p)
        for i, v in enumerate(p):
            if not fl[v] & SCC_CYCLIC:
                continue
            if i + 1 < len(p) and comp[p[i + 1]] != comp[v]:  # leaves the component at v
                for e in ex_by_end.get(v, []):
                    cand_ex.add(tuple(e + p[i + 1:]))
            if i > 0 and comp[p[i - 1]] != comp[v]:  # enters it at v
                for f in en_by_start.get(v, []):
                    cand_en.add(tuple(p[:i] + f))
    ex_pps = sorted(q for q in cand_ex if _is_prime(g, list(q), preds))
    en_pps = sorted(q for q in cand_en if _is_prime(g, list(q), preds))
    return {"complete": PathList.from_lists([list(p) for p in complete]),
            "exit": PathList.from_lists([list(p) for p in ex_pps]),
            "entry": PathList.from_lists([list(p) for p in en_pps]),
            "dropped_exit": len(cand_ex) - len(ex_pps),
            "dropped_entry": len(cand_en) - len(en_pps)}


def canonical_bytes(pl: PathList) -> bytes:
    """n (int64 LE) + offsets (int64 LE) + vertices (int32 LE)."""
    return (np.int64(len(pl)).tobytes() + pl.offsets.astype("<i8").tobytes()
            + pl.vertices.astype("<i4").tobytes())


def sha256(pl: PathList) -> str:
    import hashlib
    return hashlib.sha256(canonical_bytes(pl)).hexdigest()
