// CFG loading, validation and canonicalization (host only).
//
// Input model: the paper's Problem 1 (Sec. 3) - a digraph with a start vertex
// of in-degree 0 and an end vertex of out-degree 0, stored as CSR (Sec. 4.1).
// The engine accepts any out-degree up to TPG_MAX_OUT_DEGREE (the paper's
// out-degree-2 restriction is not applied: switch vertices are processed as
// given).

#include <atomic>
#include <cstdarg>
#include <cstring>
#include <deque>
#include <new>
#include <algorithm>

#include "internal.h"

namespace tpg {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

tpg_status fail(tpg_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return s;
}

static std::atomic<uint64_t> g_uid{1};

}  // namespace tpg

using namespace tpg;

extern "C" {

const char* tpg_last_error(void) { return g_err; }

const char* tpg_status_str(tpg_status s) {
  switch (s) {
    case TPG_OK: return "ok";
    case TPG_ERR_INVALID_ARG: return "invalid argument";
    case TPG_ERR_BAD_CSR: return "malformed CSR";
    case TPG_ERR_BAD_ENTRY_EXIT: return "bad entry/exit vertex";
    case TPG_ERR_UNREACHABLE: return "vertex unreachable from entry or cannot reach exit";
    case TPG_ERR_OOM_HOST: return "host out of memory";
    case TPG_ERR_OOM_DEVICE: return "device out of memory";
    case TPG_ERR_CAPACITY: return "pool capacity exceeded";
    case TPG_ERR_DEVICE: return "device error";
    case TPG_ERR_UNSUPPORTED: return "unsupported input";
    case TPG_ERR_CALLBACK: return "stopped by the chunk callback";
  }
  return "unknown status";
}

const char* tpg_version(void) { return "tpg 0.1 (gfx950)"; }

tpg_status tpg_load_cfg_csr(int32_t n, const int64_t* row_ptr, const int32_t* col_idx,
                            int32_t entry, int32_t exit, uint32_t load_flags,
                            tpg_graph** out) {
  if (!out) return fail(TPG_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!row_ptr) return fail(TPG_ERR_INVALID_ARG, "row_ptr is NULL");
  if (n < 1) return fail(TPG_ERR_INVALID_ARG, "n must be >= 1 (got %d)", n);
  if (n > TPG_MAX_VERTICES)
    return fail(TPG_ERR_UNSUPPORTED, "n = %d exceeds %d vertices", n, TPG_MAX_VERTICES);
  if (row_ptr[0] != 0) return fail(TPG_ERR_BAD_CSR, "row_ptr[0] must be 0");
  for (int32_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] < row_ptr[v]) return fail(TPG_ERR_BAD_CSR, "row_ptr decreases at %d", v);
  const int64_t m = row_ptr[n];
  if (m > 0 && !col_idx) return fail(TPG_ERR_INVALID_ARG, "col_idx is NULL");
  if (m > (int64_t)1 << 30) return fail(TPG_ERR_UNSUPPORTED, "too many arcs");
  for (int64_t k = 0; k < m; ++k)
    if (col_idx[k] < 0 || col_idx[k] >= n)
      return fail(TPG_ERR_BAD_CSR, "col_idx[%lld] = %d out of range", (long long)k, col_idx[k]);
  if (entry < 0 || entry >= n || exit < 0 || exit >= n)
    return fail(TPG_ERR_BAD_ENTRY_EXIT, "entry %d / exit %d out of range", entry, exit);

  tpg_graph* g = new (std::nothrow) tpg_graph;
  if (!g) return fail(TPG_ERR_OOM_HOST, "graph handle");
  g->n = n;
  g->entry = entry;
  g->exit = exit;
  g->load_flags = load_flags;
  g->uid = g_uid.fetch_add(1);
  g->succ_ptr.assign(n + 1, 0);
  std::vector<int32_t> row;
  int32_t maxdeg = 0;
  for (int32_t v = 0; v < n; ++v) {
    row.assign(col_idx + row_ptr[v], col_idx + row_ptr[v + 1]);
    std::sort(row.begin(), row.end());
    const size_t before = row.size();
    row.erase(std::unique(row.begin(), row.end()), row.end());
    if (row.size() != before && (load_flags & TPG_LOAD_STRICT)) {
      delete g;
      return fail(TPG_ERR_BAD_CSR, "duplicate arc out of vertex %d", v);
    }
    g->succ.insert(g->succ.end(), row.begin(), row.end());
    g->succ_ptr[v + 1] = (int32_t)g->succ.size();
    maxdeg = std::max<int32_t>(maxdeg, (int32_t)row.size());
  }
  if (load_flags & TPG_LOAD_BINARIZE) {
    // out-degree <= 2 (Sec. 3): vertex v with successors s_1 < .. < s_k, k > 2,
    // keeps s_1 and hands s_2 .. s_k to a chain of new decision vertices
    int64_t extra = 0;
    for (int32_t v = 0; v < n; ++v)
      extra += std::max<int32_t>(0, g->succ_ptr[v + 1] - g->succ_ptr[v] - 2);
    if (n + extra > TPG_MAX_VERTICES) {
      delete g;
      return fail(TPG_ERR_UNSUPPORTED, "binarized graph has %lld vertices (max %d)",
                  (long long)(n + extra), TPG_MAX_VERTICES);
    }
    const int32_t nb = n + (int32_t)extra;
    std::vector<std::vector<int32_t>> rows(nb);
    int32_t next_id = n;
    for (int32_t v = 0; v < n; ++v) {
      const int32_t* sv = g->succ.data() + g->succ_ptr[v];
      const int32_t k = g->succ_ptr[v + 1] - g->succ_ptr[v];
      if (k <= 2) {
        rows[v].assign(sv, sv + k);
        continue;
      }
      int32_t at = v;
      for (int32_t i = 0; i < k - 2; ++i) {
        const int32_t x = next_id++;
        rows[at] = {sv[i], x};
        at = x;
      }
      rows[at] = {sv[k - 2], sv[k - 1]};
    }
    g->n = n = nb;
    g->succ.clear();
    g->succ_ptr.assign(n + 1, 0);
    for (int32_t v = 0; v < n; ++v) {
      g->succ.insert(g->succ.end(), rows[v].begin(), rows[v].end());
      g->succ_ptr[v + 1] = (int32_t)g->succ.size();
    }
    maxdeg = std::min<int32_t>(maxdeg, 2);
  }
  g->max_out_degree = maxdeg;
  if (maxdeg > TPG_MAX_OUT_DEGREE) {
    delete g;
    return fail(TPG_ERR_UNSUPPORTED, "out-degree %d exceeds %d", maxdeg, TPG_MAX_OUT_DEGREE);
  }
  // reverse CSR, rows ascending (counting sort by target keeps sources ascending)
  g->pred_ptr.assign(n + 1, 0);
  for (int32_t w : g->succ) g->pred_ptr[w + 1]++;
  for (int32_t v = 0; v < n; ++v) g->pred_ptr[v + 1] += g->pred_ptr[v];
  g->pred.assign(g->succ.size(), 0);
  {
    std::vector<int32_t> fill(g->pred_ptr.begin(), g->pred_ptr.end() - 1);
    for (int32_t v = 0; v < n; ++v)
      for (int32_t k = g->succ_ptr[v]; k < g->succ_ptr[v + 1]; ++k)
        g->pred[fill[g->succ[k]]++] = v;
  }
  if (!(load_flags & TPG_LOAD_ANY_DIGRAPH)) {
    if (g->pred_ptr[entry + 1] != g->pred_ptr[entry]) {
      delete g;
      return fail(TPG_ERR_BAD_ENTRY_EXIT, "entry %d has predecessors", entry);
    }
    if (g->succ_ptr[exit + 1] != g->succ_ptr[exit]) {
      delete g;
      return fail(TPG_ERR_BAD_ENTRY_EXIT, "exit %d has successors", exit);
    }
    std::vector<char> seen(n, 0);
    std::deque<int32_t> q{entry};
    seen[entry] = 1;
    while (!q.empty()) {
      int32_t u = q.front();
      q.pop_front();
      for (int32_t k = g->succ_ptr[u]; k < g->succ_ptr[u + 1]; ++k)
        if (!seen[g->succ[k]]) seen[g->succ[k]] = 1, q.push_back(g->succ[k]);
    }
    std::vector<char> back(n, 0);
    q.push_back(exit);
    back[exit] = 1;
    while (!q.empty()) {
      int32_t u = q.front();
      q.pop_front();
      for (int32_t k = g->pred_ptr[u]; k < g->pred_ptr[u + 1]; ++k)
        if (!back[g->pred[k]]) back[g->pred[k]] = 1, q.push_back(g->pred[k]);
    }
    for (int32_t v = 0; v < n; ++v)
      if (!seen[v] || !back[v]) {
        delete g;
        return fail(TPG_ERR_UNREACHABLE, "vertex %d is %s", v,
                    !seen[v] ? "unreachable from entry" : "unable to reach exit");
      }
  }
  *out = g;
  return TPG_OK;
}

void tpg_graph_free(tpg_graph* g) { delete g; }

tpg_status tpg_graph_info(const tpg_graph* g, int32_t* n, int64_t* n_arcs, int32_t* entry,
                          int32_t* exit) {
  if (!g) return fail(TPG_ERR_INVALID_ARG, "graph is NULL");
  if (n) *n = g->n;
  if (n_arcs) *n_arcs = (int64_t)g->succ.size();
  if (entry) *entry = g->entry;
  if (exit) *exit = g->exit;
  return TPG_OK;
}

tpg_status tpg_graph_csr(const tpg_graph* g, int64_t* row_ptr, int32_t* col_idx) {
  if (!g || !row_ptr || (!col_idx && !g->succ.empty()))
    return fail(TPG_ERR_INVALID_ARG, "NULL argument");
  for (int32_t v = 0; v <= g->n; ++v) row_ptr[v] = g->succ_ptr[v];
  if (!g->succ.empty()) memcpy(col_idx, g->succ.data(), sizeof(int32_t) * g->succ.size());
  return TPG_OK;
}

void tpg_paths_free(tpg_paths* p) {
  if (!p) return;
  if (!p->on_device) {
    free(p->offsets);
    free(p->vertices);
  }
  memset(p, 0, sizeof *p);
}

}  // extern "C"
