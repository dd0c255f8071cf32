// Structural features of a CFG for the path-count predictor (host only).
//
// 32 numbers computed from the CSR alone: sizes, cyclomatic complexity,
// branching, loop nesting (natural loops of DFS back arcs), strongly
// connected components, if-else diamonds, switch fan-outs, distances and the
// number of entry-to-exit paths of the component DAG.  Counts that grow
// exponentially enter as logarithms.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>
#include <cstring>
#include <deque>
#include <vector>

#include "internal.h"

using namespace tpg;

namespace {

void sccs(const tpg_graph* g, std::vector<int32_t>& comp, int32_t& ncomp) {
  // iterative Tarjan
  const int32_t n = g->n;
  std::vector<int32_t> idx(n, -1), low(n, 0), stk;
  std::vector<char> on(n, 0);
  comp.assign(n, -1);
  ncomp = 0;
  int32_t counter = 0;
  std::vector<std::pair<int32_t, int32_t>> call;  // (vertex, next arc)
  for (int32_t s = 0; s < n; ++s) {
    if (idx[s] >= 0) continue;
    call.push_back({s, g->succ_ptr[s]});
    idx[s] = low[s] = counter++;
    stk.push_back(s);
    on[s] = 1;
    while (!call.empty()) {
      auto& fr = call.back();
      const int32_t v = fr.first;
      if (fr.second < g->succ_ptr[v + 1]) {
        const int32_t w = g->succ[fr.second++];
        if (idx[w] < 0) {
          idx[w] = low[w] = counter++;
          stk.push_back(w);
          on[w] = 1;
          call.push_back({w, g->succ_ptr[w]});
        } else if (on[w]) {
          low[v] = std::min(low[v], idx[w]);
        }
        continue;
      }
      if (low[v] == idx[v]) {
        for (;;) {
          const int32_t w = stk.back();
          stk.pop_back();
          on[w] = 0;
          comp[w] = ncomp;
          if (w == v) break;
        }
        ++ncomp;
      }
      call.pop_back();
      if (!call.empty()) low[call.back().first] = std::min(low[call.back().first], low[v]);
    }
  }
}

std::vector<int32_t> bfs_dist(const tpg_graph* g, int32_t src, bool forward) {
  std::vector<int32_t> d(g->n, -1);
  std::deque<int32_t> q{src};
  d[src] = 0;
  const auto& ptr = forward ? g->succ_ptr : g->pred_ptr;
  const auto& adj = forward ? g->succ : g->pred;
  while (!q.empty()) {
    const int32_t u = q.front();
    q.pop_front();
    for (int32_t k = ptr[u]; k < ptr[u + 1]; ++k)
      if (d[adj[k]] < 0) d[adj[k]] = d[u] + 1, q.push_back(adj[k]);
  }
  return d;
}

void features_of(const tpg_graph* g, float* f) {
  const int32_t n = g->n;
  const double m = (double)g->succ.size();
  std::vector<double> x(32, 0.0);
  x[0] = std::log1p((double)n);
  x[1] = std::log1p(m);
  const double cc = m - n + 2;
  x[2] = std::log1p(std::max(0.0, cc));
  x[3] = m / n;
  int32_t maxdeg = 0, ndec = 0, diamonds = 0, sw[4] = {0, 0, 0, 0};
  double bits = 0;
  for (int32_t v = 0; v < n; ++v) {
    const int32_t d = g->succ_ptr[v + 1] - g->succ_ptr[v];
    maxdeg = std::max(maxdeg, d);
    if (d >= 2) {
      ++ndec;
      bits += std::log2((double)d);
    }
    if (d == 2) {
      const int32_t a = g->succ[g->succ_ptr[v]], b = g->succ[g->succ_ptr[v] + 1];
      bool common = false;
      for (int32_t i = g->succ_ptr[a]; i < g->succ_ptr[a + 1] && !common; ++i)
        for (int32_t j = g->succ_ptr[b]; j < g->succ_ptr[b + 1]; ++j)
          if (g->succ[i] == g->succ[j]) common = true;
      diamonds += common;
    }
    if (d >= 3 && d <= 4) ++sw[0];
    else if (d >= 5 && d <= 8) ++sw[1];
    else if (d >= 9 && d <= 16) ++sw[2];
    else if (d > 16) ++sw[3];
  }
  x[4] = maxdeg;
  x[5] = (double)ndec / n;
  x[6] = std::log1p((double)ndec);
  x[7] = bits;
  // natural loops of back arcs found by an iterative DFS from the entry
  std::vector<int32_t> depth(n, 0);
  int32_t n_back = 0;
  {
    std::vector<char> state(n, 0);  // 0 new, 1 on stack, 2 done
    std::vector<std::pair<int32_t, int32_t>> st{{g->entry, g->succ_ptr[g->entry]}};
    state[g->entry] = 1;
    std::vector<std::vector<int32_t>> latches(n);
    while (!st.empty()) {
      auto& fr = st.back();
      const int32_t v = fr.first;
      if (fr.second < g->succ_ptr[v + 1]) {
        const int32_t w = g->succ[fr.second++];
        if (state[w] == 0) {
          state[w] = 1;
          st.push_back({w, g->succ_ptr[w]});
        } else if (state[w] == 1) {
          latches[w].push_back(v);
          ++n_back;
        }
        continue;
      }
      state[v] = 2;
      st.pop_back();
    }
    std::vector<char> in(n, 0);
    for (int32_t h = 0; h < n; ++h) {
      if (latches[h].empty()) continue;
      std::fill(in.begin(), in.end(), 0);
      in[h] = 1;
      std::deque<int32_t> q;
      for (int32_t u : latches[h])
        if (!in[u]) in[u] = 1, q.push_back(u);
      while (!q.empty()) {
        const int32_t u = q.front();
        q.pop_front();
        for (int32_t k = g->pred_ptr[u]; k < g->pred_ptr[u + 1]; ++k)
          if (!in[g->pred[k]]) in[g->pred[k]] = 1, q.push_back(g->pred[k]);
      }
      for (int32_t v = 0; v < n; ++v) depth[v] += in[v];
    }
  }
  int32_t maxdepth = 0;
  double hist[5] = {0, 0, 0, 0, 0};
  for (int32_t v = 0; v < n; ++v) {
    maxdepth = std::max(maxdepth, depth[v]);
    hist[std::min(depth[v], 4)] += 1.0;
  }
  x[8] = n_back;
  for (int k = 0; k < 5; ++k) x[9 + k] = hist[k] / n;
  x[14] = maxdepth;
  // strongly connected components
  std::vector<int32_t> comp;
  int32_t ncomp = 0;
  sccs(g, comp, ncomp);
  std::vector<int32_t> csize(ncomp, 0);
  std::vector<double> cbits(ncomp, 0.0);
  for (int32_t v = 0; v < n; ++v) {
    csize[comp[v]]++;
    const int32_t d = g->succ_ptr[v + 1] - g->succ_ptr[v];
    if (d >= 2) cbits[comp[v]] += std::log2((double)d);
  }
  int32_t nontriv = 0, largest = 0, in_scc = 0;
  double sq = 0, bits_in = 0, bits_max = 0;
  for (int32_t c = 0; c < ncomp; ++c) {
    if (csize[c] > 1) {
      ++nontriv;
      in_scc += csize[c];
      bits_in += cbits[c];
      bits_max = std::max(bits_max, cbits[c]);
    }
    largest = std::max(largest, csize[c]);
    sq += (double)csize[c] * csize[c];
  }
  x[15] = nontriv;
  x[16] = (double)largest / n;
  x[17] = sq / n;
  x[18] = diamonds;
  for (int k = 0; k < 4; ++k) x[19 + k] = sw[k];
  const auto df = bfs_dist(g, g->entry, true);
  const auto db = bfs_dist(g, g->exit, false);
  int32_t mdf = 0, mdb = 0;
  for (int32_t v = 0; v < n; ++v) {
    mdf = std::max(mdf, df[v]);
    mdb = std::max(mdb, db[v]);
  }
  x[23] = mdf;
  x[24] = mdb;
  x[25] = bits_max;
  x[26] = bits_in;
  x[27] = (double)in_scc / n;
  // log of the number of entry-to-exit paths in the component DAG
  {
    // Tarjan numbers components in reverse topological order
    std::vector<double> lp(ncomp, -INFINITY);
    lp[comp[g->entry]] = 0.0;
    std::vector<int32_t> cstart(ncomp + 1, 0), members(n);
    for (int32_t v = 0; v < n; ++v) cstart[comp[v] + 1]++;
    for (int32_t c = 0; c < ncomp; ++c) cstart[c + 1] += cstart[c];
    {
      std::vector<int32_t> fill(cstart.begin(), cstart.end() - 1);
      for (int32_t v = 0; v < n; ++v) members[fill[comp[v]]++] = v;
    }
    for (int32_t c = ncomp - 1; c >= 0; --c) {
      if (lp[c] == -INFINITY) continue;
      for (int32_t mi = cstart[c]; mi < cstart[c + 1]; ++mi) {
        const int32_t v = members[mi];
        for (int32_t k = g->succ_ptr[v]; k < g->succ_ptr[v + 1]; ++k) {
          const int32_t d = comp[g->succ[k]];
          if (d == c) continue;
          const double a = lp[d], b = lp[c];
          lp[d] = (a == -INFINITY) ? b : std::max(a, b) + std::log1p(std::exp(-std::fabs(a - b)));
        }
      }
    }
    const double e = lp[comp[g->exit]];
    x[28] = e == -INFINITY ? 0.0 : e;
  }
  double indeg_scc = 0;
  for (int32_t v = 0; v < n; ++v)
    if (csize[comp[v]] > 1) indeg_scc += g->pred_ptr[v + 1] - g->pred_ptr[v];
  x[29] = in_scc ? indeg_scc / in_scc : 0.0;
  x[30] = bits_in * (double)maxdepth;
  x[31] = std::log1p((double)n * std::exp2(std::min(bits_max, 60.0)));
  for (int k = 0; k < 32; ++k) f[k] = (float)x[k];
}

}  // namespace

extern "C" {

tpg_status tpg_features(const tpg_graph* const* graphs, int32_t n_graphs, float* out) {
  if (!graphs || !out || n_graphs < 0) return fail(TPG_ERR_INVALID_ARG, "NULL argument");
  for (int32_t i = 0; i < n_graphs; ++i)
    if (!graphs[i]) return fail(TPG_ERR_INVALID_ARG, "graph %d is NULL", i);
  // each graph's features are computed once (graphs are immutable), in
  // parallel over host threads
  auto one = [&](int32_t i) {
    const tpg_graph* g = graphs[i];
    std::call_once(g->feat_once, [g]() { features_of(g, g->feat); });
    memcpy(out + (size_t)32 * i, g->feat, sizeof(float) * 32);
  };
  const int nt = (int)std::min<unsigned>(16, std::max(1u, std::thread::hardware_concurrency()));
  if (n_graphs < 64 || nt == 1) {
    for (int32_t i = 0; i < n_graphs; ++i) one(i);
    return TPG_OK;
  }
  std::atomic<int32_t> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&]() {
      for (;;) {
        const int32_t i = next.fetch_add(16);
        if (i >= n_graphs) break;
        for (int32_t k = i; k < std::min(n_graphs, i + 16); ++k) one(k);
      }
    });
  for (auto& th : pool) th.join();
  return TPG_OK;
}

}  // extern "C"
