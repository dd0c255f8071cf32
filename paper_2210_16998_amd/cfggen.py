"""Seeded synthetic control-flow-graph generators.

This module only builds input graphs; it holds none of the path arithmetic
(no path extension, no prime-path test, no test-path splice).  Both the GPU
engine's tests and the CPU oracle draw their inputs from here.

A CFG is built from a small block grammar (sequence, if-else, while,
switch, straight-line statement) and lowered to a digraph with one entry
vertex (in-degree 0, id 0) and one exit vertex (out-degree 0, id V-1); the
paper's problem statement fixes exactly this input shape (Problem 1 and the
assumptions after it).  Vertex ids follow creation order of the lowering,
so structurally close blocks get close ids, as in compiler-numbered CFGs.

Every generator is a pure function of its integer seed (numpy PCG64).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class CFG:
    """A digraph in CSR form with designated entry and exit vertices."""

    n: int
    row_ptr: np.ndarray  # int64 [n+1]
    col_idx: np.ndarray  # int32 [E]
    entry: int
    exit: int
    name: str = ""

    @property
    def n_edges(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def cyclomatic(self) -> int:
        return self.n_edges - self.n + 2

    def succ(self, v: int) -> np.ndarray:
        return self.col_idx[self.row_ptr[v]:self.row_ptr[v + 1]]

    def edges(self) -> List[Tuple[int, int]]:
        return [(v, int(w)) for v in range(self.n) for w in self.succ(v)]


def from_edges(n: int, edges: Sequence[Tuple[int, int]], entry: int = 0,
               exit: Optional[int] = None, name: str = "") -> CFG:
    """CSR with rows sorted ascending and duplicate arcs removed."""
    rows: List[set] = [set() for _ in range(n)]
    for a, b in edges:
        if not (0 <= a < n and 0 <= b < n):
            raise ValueError(f"arc ({a},{b}) out of range for n={n}")
        rows[a].add(int(b))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    cols: List[int] = []
    for v in range(n):
        s = sorted(rows[v])
        cols.extend(s)
        row_ptr[v + 1] = len(cols)
    return CFG(n, row_ptr, np.asarray(cols, dtype=np.int32), int(entry),
               int(n - 1 if exit is None else exit), name)


# ---------------------------------------------------------------------------
# Block grammar and lowering
# ---------------------------------------------------------------------------
# AST nodes are tuples:
#   ('stmt',)
#   ('seq', [nodes])
#   ('if', then_seq, else_seq, join)      join: bool -> explicit join vertex
#   ('while', body_seq)
#   ('switch', [arm_seq, ...], join)

class _Lower:
    def __init__(self) -> None:
        self.n = 0
        self.edges: List[Tuple[int, int]] = []

    def new(self) -> int:
        v = self.n
        self.n += 1
        return v

    def seq(self, items) -> Optional[Tuple[int, List[int]]]:
        entry = None
        exits: List[int] = []
        for it in items:
            e, x = self.node(it)
            if entry is None:
                entry = e
            else:
                for a in exits:
                    self.edges.append((a, e))
            exits = x
        if entry is None:
            return None
        return entry, exits

    def node(self, nd) -> Tuple[int, List[int]]:
        kind = nd[0]
        if kind == 'stmt':
            v = self.new()
            return v, [v]
        if kind == 'seq':
            r = self.seq(nd[1])
            if r is None:
                raise ValueError("empty sequence node")
            return r
        if kind == 'if':
            c = self.new()
            exits: List[int] = []
            for arm in (nd[1], nd[2]):
                r = self.seq(arm)
                if r is None:
                    exits.append(c)
                else:
                    self.edges.append((c, r[0]))
                    exits.extend(r[1])
            if nd[3]:
                j = self.new()
                for a in exits:
                    self.edges.append((a, j))
                return c, [j]
            return c, exits
        if kind == 'while':
            h = self.new()
            r = self.seq(nd[1])
            if r is None:
                raise ValueError("while with empty body")
            self.edges.append((h, r[0]))
            for a in r[1]:
                self.edges.append((a, h))
            return h, [h]
        if kind == 'switch':
            s = self.new()
            exits = []
            for arm in nd[1]:
                r = self.seq(arm)
                if r is None:
                    raise ValueError("switch arm must be non-empty")
                self.edges.append((s, r[0]))
                exits.extend(r[1])
            if nd[2]:
                j = self.new()
                for a in exits:
                    self.edges.append((a, j))
                return s, [j]
            return s, exits
        raise ValueError(f"unknown node {kind}")


def lower_program(body: list, name: str = "") -> CFG:
    """Entry statement, ``body``, exit statement -> CFG (entry 0, exit V-1)."""
    lw = _Lower()
    r = lw.seq([('stmt',)] + list(body) + [('stmt',)])
    assert r is not None
    return from_edges(lw.n, lw.edges, 0, lw.n - 1, name)


def _diamond():
    return ('if', [('stmt',)], [('stmt',)], False)


# ---------------------------------------------------------------------------
# Fixed small layouts
# ---------------------------------------------------------------------------

def fig1_cfg() -> CFG:
    """The example CFG of the paper's Fig. 1 (binarySearch0), whose drawing is
    not available: rebuilt arc by arc from the paths the paper prints (Def. 1
    and 2 examples, the SCC / CCFG walk-through of Sec. 2.1).  Start = 0,
    blocks 1..9 keep the paper's numbers, End = 10."""
    edges = [(0, 1), (1, 2), (2, 3), (2, 9), (3, 4), (3, 5), (4, 8), (5, 6),
             (5, 7), (6, 8), (7, 10), (8, 2), (9, 10)]
    return from_edges(11, edges, 0, 10, "fig1")


def fig1_scc_cfg() -> CFG:
    """The SCC {2,3,4,5,6,8} of the Fig. 1 CFG taken alone, relabelled in
    ascending order to 0..5 (2->0, 3->1, 4->2, 5->3, 6->4, 8->5).  Not a CFG
    (no entry/exit); used for the SCC-only prime-path example of Sec. 2.1."""
    m = {2: 0, 3: 1, 4: 2, 5: 3, 6: 4, 8: 5}
    src = fig1_cfg()
    edges = [(m[a], m[b]) for a, b in src.edges() if a in m and b in m]
    return from_edges(6, edges, 0, 5, "fig1_scc")


FIG1_SCC_LABELS = [2, 3, 4, 5, 6, 8]


def c1_cfg(seed: int = 0) -> CFG:
    """20-vertex structured CFG: entry -> 3 sequential if-else diamonds ->
    while { while { if-else } } -> exit 19.  Seed 0 is the identity layout;
    seeds >= 1 relabel the 18 internal vertices by a seeded permutation."""
    inner = ('while', [('if', [('stmt',)], [('stmt',)], True)])
    outer = ('while', [inner, ('stmt',)])
    g = lower_program([_diamond(), _diamond(), _diamond(), ('stmt',), outer,
                       ('stmt',)], name="c1")
    assert g.n == 20
    if seed == 0:
        return g
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = np.arange(g.n)
    perm[1:g.n - 1] = 1 + rng.permutation(g.n - 2)
    return relabel(g, perm, name=f"c1_s{seed}")


def relabel(g: CFG, perm: np.ndarray, name: str = "") -> CFG:
    """Vertex v becomes perm[v]."""
    edges = [(int(perm[a]), int(perm[b])) for a, b in g.edges()]
    return from_edges(g.n, edges, int(perm[g.entry]), int(perm[g.exit]),
                      name or g.name)


def diamond_chain(k: int) -> CFG:
    return lower_program([_diamond() for _ in range(k)], name=f"dchain{k}")


def loop_diamond_chain(k: int) -> CFG:
    """entry -> while { k chained diamonds, the last one with a join vertex }
    -> stmt -> exit  (V = 3k + 5)."""
    body = [_diamond() for _ in range(k - 1)] + \
        [('if', [('stmt',)], [('stmt',)], True)]
    return lower_program([('while', body), ('stmt',)], name=f"loopdchain{k}")


def complete_digraph(n: int) -> CFG:
    edges = [(a, b) for a in range(n) for b in range(n) if a != b]
    return from_edges(n, edges, 0, n - 1, f"K{n}")


def cycle_graph(n: int) -> CFG:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)], 0, n - 1, f"C{n}")


def path_graph(n: int) -> CFG:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)], 0, n - 1, f"P{n}")


def random_digraph(seed: int, n: int, p: float, self_loops: bool = True) -> CFG:
    """Erdos-Renyi digraph (not necessarily a valid CFG)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = rng.random((n, n)) < p
    if not self_loops:
        np.fill_diagonal(m, False)
    edges = [(a, b) for a in range(n) for b in range(n) if m[a, b]]
    return from_edges(n, edges, 0, n - 1, f"er{n}_{seed}")


def random_small_cfg(seed: int, n: int, extra: int = 3) -> CFG:
    """A random valid CFG on n >= 2 vertices: entry 0 (in-degree 0), exit n-1
    (out-degree 0), every vertex reachable from entry and reaching exit.
    A random spine 0 -> ... -> n-1 through all vertices, plus ``extra``
    random arcs (back arcs included) that respect the entry/exit rules."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mid = list(1 + rng.permutation(n - 2)) if n > 2 else []
    order = [0] + [int(x) for x in mid] + [n - 1]
    edges = [(order[i], order[i + 1]) for i in range(n - 1)]
    for _ in range(extra):
        a = int(rng.integers(0, n - 1))      # any vertex but exit
        b = int(rng.integers(1, n))          # any vertex but entry
        edges.append((a, b))
    return from_edges(n, edges, 0, n - 1, f"rs{n}_{seed}")


# ---------------------------------------------------------------------------
# Random structured grammar
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class GrammarParams:
    size: int                      # target vertex count (approximate)
    max_loop_depth: int = 4
    switch_fanout: Tuple[int, int] = (3, 8)
    p_if: float = 0.30
    p_while: float = 0.12
    p_switch: float = 0.04
    p_join: float = 0.5            # if-else gets an explicit join vertex
    p_else: float = 0.8            # if-else has a non-empty else arm
    max_block: int = 24            # cap on a compound block's vertex budget
    branch_bits: float = math.inf  # total decision bits allowed in the graph


class _Gen:
    def __init__(self, rng: np.random.Generator, P: GrammarParams) -> None:
        self.rng = rng
        self.P = P
        self.bits = P.branch_bits

    def seq(self, size: int, depth: int) -> list:
        out: list = []
        while size > 0:
            node, used = self.block(size, depth)
            out.append(node)
            size -= used
        return out

    def _take_bits(self, b: float) -> bool:
        if self.bits >= b:
            self.bits -= b
            return True
        return False

    def block(self, size: int, depth: int):
        P, rng = self.P, self.rng
        u = rng.random()
        cap = min(size, P.max_block)
        if u < P.p_while and depth < P.max_loop_depth and cap >= 3 \
                and self._take_bits(1.0):
            s = int(rng.integers(3, cap + 1))
            return ('while', self.seq(s - 1, depth + 1)), s
        u -= P.p_while
        lo, hi = P.switch_fanout
        if u < P.p_switch and cap >= lo + 2:
            k = int(rng.integers(lo, min(hi, cap - 2) + 1))
            if self._take_bits(math.log2(k)):
                s = int(rng.integers(k + 2, cap + 1))
                arms_budget = s - 2
                share = self._split(arms_budget, k)
                arms = [self.seq(b, depth) for b in share]
                return ('switch', arms, True), s
        u -= P.p_switch
        if u < P.p_if and cap >= 3 and self._take_bits(1.0):
            join = rng.random() < P.p_join
            has_else = rng.random() < P.p_else
            need = 1 + int(join) + 1 + int(has_else)
            if cap >= need:
                s = int(rng.integers(need, cap + 1))
                body = s - 1 - int(join)
                if has_else:
                    a, b = self._split(body, 2)
                    return ('if', self.seq(a, depth), self.seq(b, depth), join), s
                if not join:
                    # an if without else and without join would leave the
                    # cond vertex as an exit of the construct; keep it simple
                    join = True
                    s = max(s, 3)
                    body = s - 2
                return ('if', self.seq(body, depth), [], join), s
            self.bits += 1.0
        return ('stmt',), 1

    def _split(self, total: int, k: int) -> List[int]:
        """Split ``total`` into k positive parts at random."""
        if k > total:
            raise ValueError("cannot split")
        cuts = np.sort(self.rng.choice(np.arange(1, total), size=k - 1,
                                       replace=False)) if k > 1 else []
        parts = np.diff(np.concatenate([[0], cuts, [total]])).astype(int)
        return [int(x) for x in parts]


def structured_cfg(seed: int, P: GrammarParams, name: str = "") -> CFG:
    rng = np.random.Generator(np.random.PCG64(seed))
    g = _Gen(rng, P)
    body = g.seq(max(P.size - 2, 1), 0)
    return lower_program(body, name=name or f"g{seed}")


# ---------------------------------------------------------------------------
# Workload recipes
# ---------------------------------------------------------------------------

def c2_params(seed: int) -> GrammarParams:
    rng = np.random.Generator(np.random.PCG64(seed ^ 0x5EED))
    return GrammarParams(size=int(rng.integers(180, 221)), max_loop_depth=4,
                         switch_fanout=(3, 8), p_if=0.22, p_while=0.12,
                         p_switch=0.03)


def c2_shape_ok(g: CFG) -> bool:
    """Shape window of the single ~200-vertex workload (Table 1, CFGs 1-2:
    V 180-215, CC 35-44)."""
    return 180 <= g.n <= 220 and 36 <= g.cyclomatic <= 44


def c2_cfg(seed: int) -> CFG:
    """~200-vertex structured CFG (sequence/if-else/while/switch fan-out
    3..8, loop nesting depth <= 4)."""
    return structured_cfg(seed, c2_params(seed), name=f"c2_s{seed}")


C3_SEED_BASE = 3_000_000
C4_SEED_BASE = 4_000_000


def batch_member_params(seed: int) -> GrammarParams:
    """Per-graph parameters of the batched workload: vertex count lognormal
    (median 40, sigma 0.6) clipped to [10, 300]; loop depth uniform 1..5; a
    total branching budget of 18 decision bits per graph."""
    rng = np.random.Generator(np.random.PCG64(seed ^ 0xBA7C4))
    z = rng.standard_normal()
    v = int(np.clip(round(math.exp(math.log(40.0) + 0.6 * z)), 10, 300))
    depth = int(rng.integers(1, 6))
    return GrammarParams(size=v, max_loop_depth=depth, switch_fanout=(3, 8),
                         branch_bits=18.0)


def batch_member_cfg(seed: int) -> CFG:
    return structured_cfg(seed, batch_member_params(seed), name=f"b{seed}")


def c3_batch(count: int = 4096, base: int = C3_SEED_BASE) -> List[CFG]:
    return [batch_member_cfg(base + i) for i in range(count)]


def c5_cfg(per_arm: int = 3, chain: Tuple[int, int, int] = (1, 1, 1),
           tail: int = 9, pad_to: int = 400) -> CFG:
    """High-NPath stress layout: 3 nested while loops, one 16-way switch and
    60 if-else diamonds, padded with straight-line statements to ~400
    vertices.  Chaining all 60 diamonds along one path would give more than
    2^60 prime paths, so the diamonds are placed so that only a bounded
    number lie on any simple path: ``per_arm`` in each of the 16 switch arms
    (parallel), ``chain[i]`` before the next nested loop at level i, and
    ``tail`` after the switch inside the innermost loop."""
    def stmts(k):
        return [('stmt',) for _ in range(k)]

    arms = [[_diamond() for _ in range(per_arm)] or [('stmt',)] for _ in range(16)]
    switch = ('switch', arms, True)
    lvl3 = ('while', [_diamond() for _ in range(chain[2])] + [switch]
            + [_diamond() for _ in range(tail)] + [('stmt',)])
    lvl2 = ('while', [_diamond() for _ in range(chain[1])] + [lvl3, ('stmt',)])
    lvl1 = ('while', [_diamond() for _ in range(chain[0])] + [lvl2, ('stmt',)])
    g = lower_program([lvl1], name="c5")
    pad = max(0, pad_to - g.n)
    pre, post = pad // 2, pad - pad // 2
    return lower_program(stmts(pre) + [lvl1] + stmts(post), name="c5")
