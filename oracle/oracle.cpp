// CPU oracle for prime paths (PP) and test paths (TP).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
// execute this code: only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark use it.  It shares no code, header, table or helper
// with the GPU engine; both read the same seeded input graphs and nothing
// else.
//
// What it computes, and from which passage of the paper:
//  * A simple path is a vertex sequence v1..vk (k > 0) along arcs in which no
//    vertex repeats, except that v1 = vk is allowed (Sec. 2, Preliminaries).
//  * A prime path is a simple path that is not a proper subpath of any other
//    simple path (Def. 1; Sec. 1 and Sec. 7.1 restate it as "maximal").
//  * The enumeration follows the edge-based method the paper attributes to
//    Ammann and Offutt (Sec. 7.2): start from every single vertex, extend by
//    one arc while the path stays simple, stop a path when it cannot be
//    extended (or when it has closed a cycle), then prune every candidate
//    that is covered by another one.  Enumeration here is a depth-first
//    walk with ascending successors, which visits exactly the same tree of
//    simple paths as the level-by-level extension.
//  * Pruning: a candidate that cannot be extended forward can only be covered
//    as a proper suffix of another non-extendable candidate (a path that
//    follows it would extend it), and a closed cycle is never covered.  So the
//    prune pass sorts the reversed acyclic candidates and drops each one that
//    is a proper prefix of its successor in that order.
//  * Test paths (Problem 1 output; Sec. 7.3 describes extending every prime
//    path to the initial and final nodes): prefix = the lexicographically
//    smallest shortest path from the entry to the first vertex, suffix = the
//    lexicographically smallest shortest path from the last vertex to the
//    exit, shared endpoints kept once; duplicates removed; sorted.
//  * Canonical order of every path set: lexicographic on the vertex ids.
//
// A second, independent prime-path test (the "local rule": an acyclic
// non-extendable path is prime iff every predecessor of its first vertex lies
// on it) is provided for counting runs that must not hold every candidate in
// memory; tests check that it agrees with the prune pass.
//
// Brute-force routines for graphs of <= 12 vertices enumerate simple paths by
// length (breadth first, a different routine from the DFS) and test
// subsumption directly against the definition.

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <vector>

namespace {

struct Digraph {
  int n = 0;
  std::vector<std::vector<int>> succ;  // ascending, unique
  std::vector<std::vector<int>> pred;  // ascending, unique
};

Digraph make_graph(int n, const int64_t* row_ptr, const int32_t* col_idx) {
  Digraph g;
  g.n = n;
  g.succ.assign(n, {});
  g.pred.assign(n, {});
  for (int v = 0; v < n; ++v) {
    for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) g.succ[v].push_back(col_idx[k]);
    std::sort(g.succ[v].begin(), g.succ[v].end());
    g.succ[v].erase(std::unique(g.succ[v].begin(), g.succ[v].end()), g.succ[v].end());
    for (int w : g.succ[v]) g.pred[w].push_back(v);
  }
  for (int v = 0; v < n; ++v) std::sort(g.pred[v].begin(), g.pred[v].end());
  return g;
}

using Path = std::vector<int32_t>;

// Per-start-vertex result of the DFS enumeration.
struct StartResult {
  std::vector<int32_t> verts;     // concatenated candidate paths
  std::vector<int64_t> offs;      // starts (size = count + 1)
  std::vector<uint8_t> is_cycle;  // per candidate
  std::vector<uint8_t> local_pp;  // per candidate: local-rule verdict
  std::vector<int64_t> level;     // level[L] = acyclic paths with L vertices
  std::vector<int64_t> cyc;       // cyc[L] = cycles with L entries (L-1 distinct)
};

// Depth-first enumeration of every simple path that starts at s.
// Emits every candidate that cannot be extended (acyclic) and every closed
// cycle, in lexicographic order.  When `store` is false only counters are
// kept (the candidate list stays empty) and the local-rule PP count is
// accumulated into *n_local_pp.
void dfs_from(const Digraph& g, int s, bool store, StartResult& r, int64_t* n_local_pp,
              std::atomic<int64_t>* budget = nullptr) {
  const int n = g.n;
  std::vector<char> on(n, 0);
  std::vector<int32_t> path;
  std::vector<size_t> it;  // next successor index per depth
  std::vector<char> grew;  // did the path at this depth produce an extension
  r.level.assign(n + 2, 0);
  r.cyc.assign(n + 2, 0);
  if (store) r.offs.push_back(0);
  path.push_back(s);
  on[s] = 1;
  it.push_back(0);
  grew.push_back(0);
  r.level[1] += 1;
  auto emit = [&](const std::vector<int32_t>& p, bool cycle, bool local) {
    if (store) {
      r.verts.insert(r.verts.end(), p.begin(), p.end());
      r.offs.push_back((int64_t)r.verts.size());
      r.is_cycle.push_back(cycle ? 1 : 0);
      r.local_pp.push_back(local ? 1 : 0);
    }
    if (local && n_local_pp) *n_local_pp += 1;
  };
  while (!path.empty()) {
    const int u = path.back();
    const size_t d = path.size() - 1;
    const auto& su = g.succ[u];
    if (it[d] < su.size()) {
      const int w = su[it[d]++];
      if (w == s) {
        grew[d] = 1;
        path.push_back(w);
        r.cyc[path.size()] += 1;
        emit(path, true, true);
        path.pop_back();
      } else if (!on[w]) {
        if (budget && (r.level[path.size() + 1] & 0xFFF) == 0 &&
            budget->fetch_sub(4096) < 0)
          return;  // counting run over its extension cap: abandon
        grew[d] = 1;
        path.push_back(w);
        on[w] = 1;
        it.push_back(0);
        grew.push_back(0);
        r.level[path.size()] += 1;
      }
      continue;
    }
    if (!grew[d]) {
      // cannot be extended forward: candidate; local rule for the verdict
      bool all_in = true;
      for (int p : g.pred[s])
        if (!on[p]) { all_in = false; break; }
      emit(path, false, all_in);
    }
    on[u] = 0;
    path.pop_back();
    it.pop_back();
    grew.pop_back();
  }
}

template <class F>
void parallel_over_starts(int n, int nthreads, F&& fn) {
  if (nthreads <= 1) {
    for (int s = 0; s < n; ++s) fn(s);
    return;
  }
  std::atomic<int> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < nthreads; ++t)
    pool.emplace_back([&]() {
      for (;;) {
        int s = next.fetch_add(1);
        if (s >= n) break;
        fn(s);
      }
    });
  for (auto& th : pool) th.join();
}

struct PathSet {
  std::vector<int64_t> offs{0};
  std::vector<int32_t> verts;
  void add(const int32_t* b, const int32_t* e) {
    verts.insert(verts.end(), b, e);
    offs.push_back((int64_t)verts.size());
  }
  int64_t size() const { return (int64_t)offs.size() - 1; }
};

}  // namespace

extern "C" {

typedef struct orc_paths {
  int64_t n_paths;
  int64_t n_vertices;
  int64_t* offsets;   // n_paths + 1, malloc'ed
  int32_t* vertices;  // n_vertices, malloc'ed
} orc_paths;

typedef struct orc_stats {
  int64_t n_candidates;   // non-extendable acyclic paths + closed cycles
  int64_t n_cycles;
  int64_t n_extensions;   // simple paths with >= 2 entries (cycles included)
  int64_t n_pp;
  int64_t n_pp_local;     // PPs by the local rule (must equal n_pp)
  int64_t max_len;        // longest PP, in entries
} orc_stats;

static void to_out(const PathSet& ps, orc_paths* out) {
  out->n_paths = ps.size();
  out->n_vertices = (int64_t)ps.verts.size();
  out->offsets = (int64_t*)malloc(sizeof(int64_t) * (ps.offs.size()));
  out->vertices = (int32_t*)malloc(sizeof(int32_t) * (ps.verts.size() + 1));
  memcpy(out->offsets, ps.offs.data(), sizeof(int64_t) * ps.offs.size());
  if (!ps.verts.empty()) memcpy(out->vertices, ps.verts.data(), sizeof(int32_t) * ps.verts.size());
}

void orc_free_paths(orc_paths* p) {
  if (!p) return;
  free(p->offsets);
  free(p->vertices);
  p->offsets = nullptr;
  p->vertices = nullptr;
  p->n_paths = p->n_vertices = 0;
}

// Prime paths of an arbitrary digraph (rows of col_idx need not be sorted).
// level_counts[L] (L = 0..n+1) receives the number of acyclic simple paths
// with L vertices; cycle_counts[L] the number of closed cycles with L entries.
// Either array may be NULL.  Returns 0.
int orc_prime_paths(int n, const int64_t* row_ptr, const int32_t* col_idx, int nthreads,
                    orc_paths* out, orc_stats* st, int64_t* level_counts, int64_t* cycle_counts) {
  Digraph g = make_graph(n, row_ptr, col_idx);
  std::vector<StartResult> res(n);
  parallel_over_starts(n, nthreads, [&](int s) { dfs_from(g, s, true, res[s], nullptr); });

  // Gather the candidates in start-vertex order (which is lexicographic).
  std::vector<const int32_t*> cb;
  std::vector<int64_t> cl;
  std::vector<uint8_t> ccyc, clocal;
  for (int s = 0; s < n; ++s) {
    const auto& r = res[s];
    for (size_t i = 0; i + 1 < r.offs.size(); ++i) {
      cb.push_back(r.verts.data() + r.offs[i]);
      cl.push_back(r.offs[i + 1] - r.offs[i]);
      ccyc.push_back(r.is_cycle[i]);
      clocal.push_back(r.local_pp[i]);
    }
  }
  const int64_t m = (int64_t)cb.size();

  // Prune pass: reversed acyclic candidates, sorted; a candidate whose
  // reversal is a proper prefix of the next reversal is a proper suffix of
  // another candidate, hence covered.
  std::vector<int64_t> acyc;
  for (int64_t i = 0; i < m; ++i)
    if (!ccyc[i]) acyc.push_back(i);
  std::vector<std::vector<int32_t>> rev(acyc.size());
  for (size_t k = 0; k < acyc.size(); ++k) {
    const int64_t i = acyc[k];
    rev[k].assign(cb[i], cb[i] + cl[i]);
    std::reverse(rev[k].begin(), rev[k].end());
  }
  std::vector<size_t> ord(acyc.size());
  for (size_t k = 0; k < ord.size(); ++k) ord[k] = k;
  std::sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return rev[a] < rev[b]; });
  std::vector<uint8_t> covered(m, 0);
  for (size_t t = 0; t + 1 < ord.size(); ++t) {
    const auto& a = rev[ord[t]];
    const auto& b = rev[ord[t + 1]];
    if (b.size() > a.size() && std::equal(a.begin(), a.end(), b.begin())) covered[acyc[ord[t]]] = 1;
  }

  PathSet pp;
  int64_t n_local = 0, max_len = 0;
  for (int64_t i = 0; i < m; ++i) {
    n_local += clocal[i];
    if (covered[i]) continue;
    pp.add(cb[i], cb[i] + cl[i]);
    max_len = std::max(max_len, cl[i]);
  }
  if (out) to_out(pp, out);
  int64_t cycles = 0, ext = 0;
  std::vector<int64_t> lv(n + 2, 0), cy(n + 2, 0);
  for (int s = 0; s < n; ++s)
    for (int L = 0; L < n + 2; ++L) {
      lv[L] += res[s].level[L];
      cy[L] += res[s].cyc[L];
    }
  for (int L = 0; L < n + 2; ++L) {
    cycles += cy[L];
    if (L >= 2) ext += lv[L];
  }
  ext += cycles;
  if (level_counts) memcpy(level_counts, lv.data(), sizeof(int64_t) * (n + 2));
  if (cycle_counts) memcpy(cycle_counts, cy.data(), sizeof(int64_t) * (n + 2));
  if (st) {
    st->n_candidates = m;
    st->n_cycles = cycles;
    st->n_extensions = ext;
    st->n_pp = pp.size();
    st->n_pp_local = n_local;
    st->max_len = max_len;
  }
  return 0;
}

// Prime paths whose first vertex lies in [s_lo, s_hi), by the local rule, in
// lexicographic order.  Used where the full candidate set is too large to
// hold (it needs no candidate from other start vertices).
int orc_prime_paths_local(int n, const int64_t* row_ptr, const int32_t* col_idx, int s_lo,
                          int s_hi, int nthreads, orc_paths* out, orc_stats* st) {
  Digraph g = make_graph(n, row_ptr, col_idx);
  s_lo = std::max(0, s_lo);
  s_hi = std::min(n, s_hi);
  const int cnt = std::max(0, s_hi - s_lo);
  std::vector<StartResult> res(cnt);
  parallel_over_starts(cnt, nthreads, [&](int i) { dfs_from(g, s_lo + i, true, res[i], nullptr); });
  PathSet pp;
  int64_t cycles = 0, ext = 0, cand = 0, max_len = 0;
  for (int i = 0; i < cnt; ++i) {
    const auto& r = res[i];
    for (size_t k = 0; k + 1 < r.offs.size(); ++k) {
      ++cand;
      if (!r.local_pp[k]) continue;
      pp.add(r.verts.data() + r.offs[k], r.verts.data() + r.offs[k + 1]);
      max_len = std::max<int64_t>(max_len, r.offs[k + 1] - r.offs[k]);
    }
    for (int L = 0; L < n + 2; ++L) {
      cycles += r.cyc[L];
      if (L >= 2) ext += r.level[L];
    }
  }
  if (out) to_out(pp, out);
  if (st) {
    st->n_candidates = cand;
    st->n_cycles = cycles;
    st->n_extensions = ext + cycles;
    st->n_pp = pp.size();
    st->n_pp_local = pp.size();
    st->max_len = max_len;
  }
  return 0;
}

// Counting run: per-level acyclic path counts, cycles and the local-rule PP
// count, without storing any path.  level_counts / cycle_counts: n+2 entries.
// ext_cap > 0 bounds the work: past about that many extensions the run stops
// and returns 1 (counts are then incomplete).
int orc_count(int n, const int64_t* row_ptr, const int32_t* col_idx, int nthreads,
              int64_t ext_cap, orc_stats* st, int64_t* level_counts, int64_t* cycle_counts,
              int64_t* pp_per_start) {
  Digraph g = make_graph(n, row_ptr, col_idx);
  std::vector<StartResult> res(n);
  std::vector<int64_t> npp(n, 0);
  std::atomic<int64_t> budget{ext_cap > 0 ? ext_cap : 0};
  parallel_over_starts(n, nthreads, [&](int s) {
    dfs_from(g, s, false, res[s], &npp[s], ext_cap > 0 ? &budget : nullptr);
  });
  if (ext_cap > 0 && budget.load() < 0) return 1;
  if (pp_per_start) memcpy(pp_per_start, npp.data(), sizeof(int64_t) * n);
  std::vector<int64_t> lv(n + 2, 0), cy(n + 2, 0);
  int64_t pp = 0;
  for (int s = 0; s < n; ++s) {
    pp += npp[s];
    for (int L = 0; L < n + 2; ++L) {
      lv[L] += res[s].level[L];
      cy[L] += res[s].cyc[L];
    }
  }
  int64_t cycles = 0, ext = 0;
  for (int L = 0; L < n + 2; ++L) {
    cycles += cy[L];
    if (L >= 2) ext += lv[L];
  }
  if (level_counts) memcpy(level_counts, lv.data(), sizeof(int64_t) * (n + 2));
  if (cycle_counts) memcpy(cycle_counts, cy.data(), sizeof(int64_t) * (n + 2));
  if (st) {
    st->n_candidates = -1;
    st->n_cycles = cycles;
    st->n_extensions = ext + cycles;
    st->n_pp = pp;
    st->n_pp_local = pp;
    st->max_len = -1;
  }
  return 0;
}

// Brute force, straight from the definitions (graphs of <= 12 vertices):
// every simple path, grown breadth first by length; a path is prime iff no
// other simple path contains it as a proper contiguous subpath.
// Also returns all simple paths when `all` is non-NULL.
int orc_bruteforce_pp(int n, const int64_t* row_ptr, const int32_t* col_idx, orc_paths* out,
                      orc_paths* all) {
  if (n > 32) return -1;
  Digraph g = make_graph(n, row_ptr, col_idx);
  // Def. of a simple path (Sec. 2): no vertex repeats, except v1 = vk.
  auto is_simple = [](const Path& q) {
    const size_t k = q.size();
    for (size_t i = 0; i < k; ++i)
      for (size_t j = i + 1; j < k; ++j)
        if (q[i] == q[j] && !(i == 0 && j == k - 1)) return false;
    return true;
  };
  std::vector<Path> paths, frontier;
  for (int v = 0; v < n; ++v) frontier.push_back({v});
  while (!frontier.empty()) {
    std::vector<Path> next;
    for (const Path& p : frontier) {
      paths.push_back(p);
      for (int w : g.succ[p.back()]) {
        Path q = p;
        q.push_back(w);
        if (is_simple(q)) next.push_back(q);
      }
    }
    frontier.swap(next);
    if (paths.size() > 60000) return -2;  // too many simple paths for O(N^2)
  }
  // subsumption
  PathSet pp;
  std::sort(paths.begin(), paths.end());
  for (const Path& p : paths) {
    bool sub = false;
    for (const Path& q : paths) {
      if (q.size() <= p.size()) continue;
      for (size_t off = 0; off + p.size() <= q.size() && !sub; ++off)
        if (std::equal(p.begin(), p.end(), q.begin() + off)) sub = true;
      if (sub) break;
    }
    if (!sub) pp.add(p.data(), p.data() + p.size());
  }
  if (out) to_out(pp, out);
  if (all) {
    PathSet a;
    for (const Path& p : paths) a.add(p.data(), p.data() + p.size());
    to_out(a, all);
  }
  return 0;
}

// BFS tables.  dist_f[v]: arcs from entry (-1 if unreachable); parent[v]: the
// first vertex to discover v in a FIFO search that scans successors in
// ascending order (-1 for entry/unreached); dist_b[v]: arcs from v to exit
// (-1 if exit unreachable); next[v]: smallest successor w with
// dist_b[w] = dist_b[v] - 1 (-1 for exit/none).
int orc_bfs(int n, const int64_t* row_ptr, const int32_t* col_idx, int entry, int exit,
            int32_t* dist_f, int32_t* parent, int32_t* dist_b, int32_t* next) {
  Digraph g = make_graph(n, row_ptr, col_idx);
  for (int v = 0; v < n; ++v) dist_f[v] = parent[v] = dist_b[v] = next[v] = -1;
  std::deque<int> q;
  dist_f[entry] = 0;
  q.push_back(entry);
  while (!q.empty()) {
    int u = q.front();
    q.pop_front();
    for (int w : g.succ[u])
      if (dist_f[w] < 0) {
        dist_f[w] = dist_f[u] + 1;
        parent[w] = u;
        q.push_back(w);
      }
  }
  dist_b[exit] = 0;
  q.push_back(exit);
  while (!q.empty()) {
    int u = q.front();
    q.pop_front();
    for (int w : g.pred[u])
      if (dist_b[w] < 0) {
        dist_b[w] = dist_b[u] + 1;
        q.push_back(w);
      }
  }
  for (int v = 0; v < n; ++v) {
    if (v == exit || dist_b[v] < 0) continue;
    for (int w : g.succ[v])
      if (dist_b[w] == dist_b[v] - 1) {
        next[v] = w;
        break;
      }
  }
  return 0;
}

// Lexicographically smallest shortest path from a to b by exhaustive search
// over all shortest paths (small graphs only).  Writes up to cap vertices into
// out and returns the length in vertices, or -1 if b is unreachable.
int orc_bruteforce_lexmin_shortest(int n, const int64_t* row_ptr, const int32_t* col_idx, int a,
                                   int b, int32_t* out, int cap) {
  if (n > 32) return -2;
  Digraph g = make_graph(n, row_ptr, col_idx);
  // all walks of increasing length until b is reached; shortest ones are simple
  std::vector<Path> layer{{a}};
  for (int len = 0; len <= n; ++len) {
    std::vector<Path> hits;
    for (const Path& p : layer)
      if (p.back() == b) hits.push_back(p);
    if (!hits.empty()) {
      const Path& best = *std::min_element(hits.begin(), hits.end());
      if ((int)best.size() > cap) return -3;
      std::copy(best.begin(), best.end(), out);
      return (int)best.size();
    }
    std::vector<Path> nl;
    for (const Path& p : layer)
      for (int w : g.succ[p.back()]) {
        if (std::find(p.begin(), p.end(), w) != p.end()) continue;
        Path q = p;
        q.push_back(w);
        nl.push_back(q);
      }
    layer.swap(nl);
    if (layer.empty()) break;
  }
  return -1;
}

// Test paths of the given prime paths: splice + dedup + lexicographic sort.
// n_spliced receives the count before deduplication.
int orc_test_paths(int n, const int64_t* row_ptr, const int32_t* col_idx, int entry, int exit,
                   const orc_paths* pp, orc_paths* out, int64_t* n_spliced) {
  std::vector<int32_t> df(n), par(n), db(n), nx(n);
  orc_bfs(n, row_ptr, col_idx, entry, exit, df.data(), par.data(), db.data(), nx.data());
  std::vector<Path> tps;
  tps.reserve(pp->n_paths);
  for (int64_t i = 0; i < pp->n_paths; ++i) {
    const int32_t* p = pp->vertices + pp->offsets[i];
    const int64_t len = pp->offsets[i + 1] - pp->offsets[i];
    const int v1 = p[0], vk = p[len - 1];
    if (df[v1] < 0 || db[vk] < 0) return -1;
    Path pre;
    for (int v = v1; v != entry; v = par[v]) pre.push_back(par[v]);
    std::reverse(pre.begin(), pre.end());
    Path t = pre;
    t.insert(t.end(), p, p + len);
    for (int v = vk; v != exit; v = nx[v]) t.push_back(nx[v]);
    tps.push_back(std::move(t));
  }
  if (n_spliced) *n_spliced = (int64_t)tps.size();
  std::sort(tps.begin(), tps.end());
  tps.erase(std::unique(tps.begin(), tps.end()), tps.end());
  PathSet ps;
  for (const Path& t : tps) ps.add(t.data(), t.data() + t.size());
  to_out(ps, out);
  return 0;
}

// Test paths by the longest-first covering that the paper cites for
// generating TPs (Ammann and Offutt, in its survey of TP generation): the
// prime paths are taken in order of decreasing length (ties: the given
// canonical order); a prime path that is already a contiguous subpath of a
// chosen test path gets none of its own, any other gets its spliced test
// path (prefix + path + suffix, as above) chosen.  Every simple contiguous
// subpath and simple cycle of a chosen test path is looked up in the prime
// path set.  Output: the chosen test paths in lexicographic order.
int orc_test_paths_greedy(int n, const int64_t* row_ptr, const int32_t* col_idx, int entry,
                          int exit, const orc_paths* pp, orc_paths* out) {
  std::vector<int32_t> df(n), par(n), db(n), nx(n);
  orc_bfs(n, row_ptr, col_idx, entry, exit, df.data(), par.data(), db.data(), nx.data());
  const int64_t np = pp->n_paths;
  std::map<Path, int64_t> id;
  std::vector<int64_t> order(np);
  for (int64_t i = 0; i < np; ++i) {
    const int32_t* p = pp->vertices + pp->offsets[i];
    id[Path(p, p + (pp->offsets[i + 1] - pp->offsets[i]))] = i;
    order[i] = i;
  }
  auto len = [&](int64_t i) { return pp->offsets[i + 1] - pp->offsets[i]; };
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return len(a) > len(b); });
  std::vector<char> covered(np, 0);
  std::vector<Path> chosen;
  for (int64_t i : order) {
    if (covered[i]) continue;
    const int32_t* p = pp->vertices + pp->offsets[i];
    const int v1 = p[0], vk = p[len(i) - 1];
    if (df[v1] < 0 || db[vk] < 0) return -1;
    Path t;
    for (int v = v1; v != entry; v = par[v]) t.push_back(par[v]);
    std::reverse(t.begin(), t.end());
    t.insert(t.end(), p, p + len(i));
    for (int v = vk; v != exit; v = nx[v]) t.push_back(nx[v]);
    for (size_t a = 0; a < t.size(); ++a) {
      Path w;
      std::vector<char> on(n, 0);
      for (size_t b = a; b < t.size(); ++b) {
        const int x = t[b];
        const bool closes = b > a && x == t[a];
        if (on[x] && !closes) break;  // prime paths are simple paths or simple cycles
        w.push_back(x);
        auto it = id.find(w);
        if (it != id.end()) covered[it->second] = 1;
        if (closes) break;
        on[x] = 1;
      }
    }
    chosen.push_back(std::move(t));
  }
  std::sort(chosen.begin(), chosen.end());
  chosen.erase(std::unique(chosen.begin(), chosen.end()), chosen.end());
  PathSet ps;
  for (const Path& t : chosen) ps.add(t.data(), t.data() + t.size());
  to_out(ps, out);
  return 0;
}

// FNV-1a, 64-bit (Fowler, Noll and Vo): start from the offset basis
// 14695981039346656037; for every byte, xor it in, then multiply by the FNV
// prime 1099511628211 (mod 2^64).
uint64_t orc_fnv1a64(const uint8_t* bytes, int64_t n) {
  uint64_t h = 14695981039346656037ull;
  for (int64_t i = 0; i < n; ++i) {
    h ^= bytes[i];
    h *= 1099511628211ull;
  }
  return h;
}

// Set digest of a path set: for each path p with k entries the hash of the
// little-endian int32 byte string (k, p_1, .., p_k); out[0] = their sum mod
// 2^64, out[1] = their xor.
void orc_digest(int64_t n_paths, const int64_t* offsets, const int32_t* vertices, uint64_t* out) {
  uint64_t sum = 0, x = 0;
  std::vector<uint8_t> buf;
  for (int64_t i = 0; i < n_paths; ++i) {
    const int64_t k = offsets[i + 1] - offsets[i];
    buf.clear();
    auto put = [&](uint32_t w) {
      for (int b = 0; b < 4; ++b) buf.push_back((uint8_t)(w >> (8 * b)));
    };
    put((uint32_t)k);
    for (int64_t j = offsets[i]; j < offsets[i + 1]; ++j) put((uint32_t)vertices[j]);
    const uint64_t h = orc_fnv1a64(buf.data(), (int64_t)buf.size());
    sum += h;
    x ^= h;
  }
  out[0] = sum;
  out[1] = x;
}


// Whole-set figures of a graph too large to hold its test paths at once:
// the prime paths (local rule) of every first vertex, their per-start counts
// and set digest, and the test paths' count and set digest after exact
// deduplication.  Duplicates are removed bucket by bucket: a test path goes
// to bucket (its FNV-1a 64 hash mod n_buckets), so equal test paths always
// meet in one bucket, and each bucket's paths are sorted and made unique by
// plain sequence comparison.  Every bucket enumerates the prime paths again,
// first vertices a chunk at a time, so memory is bounded by one bucket's
// test paths plus one chunk's candidates.
// pp_per_start: n entries; pp_digest, tp_digest: 2 entries (sum, xor).
int orc_set_digests(int n, const int64_t* row_ptr, const int32_t* col_idx, int entry, int exit,
                    int nthreads, int n_buckets, int64_t* pp_per_start, uint64_t* pp_digest,
                    int64_t* n_tp, int64_t* n_spliced, uint64_t* tp_digest) {
  Digraph g = make_graph(n, row_ptr, col_idx);
  std::vector<int32_t> df(n), par(n), db(n), nx(n);
  orc_bfs(n, row_ptr, col_idx, entry, exit, df.data(), par.data(), db.data(), nx.data());
  if (n_buckets < 1) n_buckets = 1;
  auto path_hash = [](const int32_t* p, int64_t k) {
    std::vector<uint8_t> buf;
    auto put = [&](uint32_t w) {
      for (int b = 0; b < 4; ++b) buf.push_back((uint8_t)(w >> (8 * b)));
    };
    put((uint32_t)k);
    for (int64_t j = 0; j < k; ++j) put((uint32_t)p[j]);
    return orc_fnv1a64(buf.data(), (int64_t)buf.size());
  };
  const int chunk = 16;
  uint64_t ps = 0, px = 0, ts = 0, tx = 0;
  int64_t kept = 0, spliced = 0;
  for (int v = 0; v < n; ++v) pp_per_start[v] = 0;
  for (int b = 0; b < n_buckets; ++b) {
    std::vector<Path> bucket;
    for (int s0 = 0; s0 < n; s0 += chunk) {
      const int cnt = std::min(chunk, n - s0);
      std::vector<StartResult> res(cnt);
      std::vector<std::vector<Path>> tps(cnt);
      std::vector<uint64_t> hs(cnt, 0), hx(cnt, 0);
      std::vector<int64_t> np(cnt, 0);
      std::atomic<int> bad{0};
      parallel_over_starts(cnt, nthreads, [&](int i) {
        StartResult& r = res[i];
        dfs_from(g, s0 + i, true, r, nullptr);
        for (size_t k = 0; k + 1 < r.offs.size(); ++k) {
          if (!r.local_pp[k]) continue;
          const int32_t* p = r.verts.data() + r.offs[k];
          const int64_t len = r.offs[k + 1] - r.offs[k];
          np[i] += 1;
          if (b == 0) {
            const uint64_t h = path_hash(p, len);
            hs[i] += h;
            hx[i] ^= h;
          }
          const int v1 = p[0], vk = p[len - 1];
          if (df[v1] < 0 || db[vk] < 0) {
            bad = 1;
            return;
          }
          Path t;
          for (int v = v1; v != entry; v = par[v]) t.push_back(par[v]);
          std::reverse(t.begin(), t.end());
          t.insert(t.end(), p, p + len);
          for (int v = vk; v != exit; v = nx[v]) t.push_back(nx[v]);
          if (path_hash(t.data(), (int64_t)t.size()) % (uint64_t)n_buckets == (uint64_t)b)
            tps[i].push_back(std::move(t));
        }
        r = StartResult();  // free the candidates of this start
      });
      if (bad) return -1;
      for (int i = 0; i < cnt; ++i) {
        if (b == 0) {
          pp_per_start[s0 + i] = np[i];
          ps += hs[i];
          px ^= hx[i];
          spliced += np[i];
        }
        for (auto& t : tps[i]) bucket.push_back(std::move(t));
      }
    }
    std::sort(bucket.begin(), bucket.end());
    bucket.erase(std::unique(bucket.begin(), bucket.end()), bucket.end());
    kept += (int64_t)bucket.size();
    for (const Path& t : bucket) {
      const uint64_t h = path_hash(t.data(), (int64_t)t.size());
      ts += h;
      tx ^= h;
    }
  }
  pp_digest[0] = ps;
  pp_digest[1] = px;
  tp_digest[0] = ts;
  tp_digest[1] = tx;
  *n_tp = kept;
  *n_spliced = spliced;
  return 0;
}

}  // extern "C"
