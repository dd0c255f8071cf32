// Host orchestration: workspace (grow-only device arena + stream), unions of
// CFGs, level loop (device-sized one-pass or plain two-pass), ranking,
// materialization, test paths, and the batched entry point.

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "sizing.h"

using namespace tpg;

namespace {

// Outputs of one union of CFGs (graph-wide ids until localized).
struct OutSet {
  DevBuf pp_off, pp_vtx, tp_off, tp_vtx;
  DevBuf ppg_off, ppg_vtx;  // prime paths grouped by last vertex (TPG_ORDER_BY_LAST)
  DevBuf comp_starts;  // int64 [4][n_comp+1]: pp, pp vertices, tp, tp vertices
  int64_t n_pp = 0, n_ppv = 0, n_tp = 0, n_tpv = 0;
};

// A disjoint union of CFGs laid out as one graph (host side).
struct HostUnion {
  int32_t n = 0, n_comp = 0, W = 1;  // W: visited-set words in registers (power of two)
  int32_t Wu = 1;                     // words stored per visited set: ceil(largest component / 64)
  std::vector<int32_t> sp{0}, s, pp{0}, p, loc, comp, cbase{0}, centry, cexit;
  std::vector<uint64_t> uids;
};

int pow2_words(int n) {
  int w = (n + 63) / 64;
  int q = 1;
  while (q < w) q <<= 1;
  return q;
}

}  // namespace

// The batched form's whole call as one HIP graph (see tpg_batch_test_paths):
// what the call depended on, every value the host read from the device
// during the recorded call, the host-side results it produced, and the
// instantiated graph.
struct CallGraph {
  std::vector<uint8_t> key;
  std::vector<uint8_t> vals;    // host reads of the recorded call, in order
  size_t stage_bytes = 0;       // host data the call uploaded
  uint64_t gen = 0;             // the workspace's allocation generation after the record
  bool recorded = false;
  bool failed = false;          // capture did not work for this key: stay eager
  hipGraphExec_t exec = nullptr;
  // host results of the call
  std::vector<int64_t> pp_first, tp_first;
  int64_t ppv = 0, tpv = 0;
  tpg_stats stats{};
};

struct tpg_workspace {
  int device = 0;
  hipStream_t own_stream = nullptr;
  // BFS tables run on a side stream, forked after the graph upload and
  // joined before the splice, so they overlap the extension
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool bfs_pending = false;
  int num_cus = 256;
  size_t bytes = 0;
  uint64_t cap = 0;  // pool cap of the running call (0: none)

  // Host <-> device traffic of a call whose device work may be captured
  // into one graph: io_mode 0 an ordinary call; 1 an ordinary call that
  // records every value the host reads from the device and the host data
  // it uploads; 2 capture, where the reads come from the record (the graph
  // copies the device's values into io_check for the check after each
  // replay) and uploads come from pinned staging that the graph keeps.
  int io_mode = 0;
  const std::vector<uint8_t>* io_rec = nullptr;  // mode 2: the recorded reads
  std::vector<uint8_t> io_vals;                  // mode 1: reads being recorded
  size_t io_pos = 0;
  uint8_t* io_check = nullptr;
  size_t io_check_cap = 0, io_check_used = 0;
  uint8_t* io_stage = nullptr;
  size_t io_stage_cap = 0, io_stage_used = 0;
  bool io_diverged = false;  // a capture left the recorded call's path
  uint64_t alloc_gen = 0;    // bumped by every device allocation and release
  CallGraph cg;

  // union on the device
  std::vector<uint64_t> union_uids;
  // level count of the last one-pass run on this union (sizes the first batch)
  std::vector<uint64_t> levels_uids;
  int levels_last = 0;
  // unions (by graph uids) whose predicted capacities could not be allocated
  std::vector<std::vector<uint64_t>> pred_failed;
  DevBuf g_csr;
  DGraph dg{};

  // path tree
  DevBuf par, info, cstart, nch, mask0, mask1, ls;
  int64_t rec_cap = 0, mask_cap = 0;
  int mask_words = 0;
  // ranking
  DevBuf sub_cnt, pp_len, leaf_by_rank, totals, cycles;
  // scans
  DevBuf scan_status, scan_ctr, scalars;
  DevBuf scan2_status, scalars2;  // the side stream's own scan scratch
  // test paths
  DevBuf bfs_i32, pfx_off, sfx_off, pfx, sfx, pfx_pk, sfx_pk;
  DevBuf tp_len, tp_off, tp_vtx, tp_key, tp_pk, idx0, idx1, grp_cnt, rb0, rb1, merge_split, tp_lead;
  bool tp_len_ready = false;  // the prime-path writer filled tp_len and tp_lead for this union
  bool rb_ready = false;      // the root ranking wrote the runs by first vertex into rb0
  DevBuf keep_cnt, keep_len, keep_pos, keep_voff, comp_cnt;
  // per-level, per-component counts (batched labels)
  DevBuf lvl_comp;
  // outputs: out[0] single-graph calls, out[k] the unions of a batch
  std::vector<OutSet> out;
  DevBuf b_pp_off, b_pp_vtx, b_tp_off, b_tp_vtx, b_desc;

  // pinned host mirrors
  LevelState* h_ls = nullptr;
  int64_t* h_scalars = nullptr;

  std::vector<hipEvent_t> ev_pool;

  // captured level loops: a graph of `len` identical extension launches per
  // batch length, valid while the launch arguments stay the same
  struct LevelGraph {
    int len = 0;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<LevelGraph> level_graphs;
  // captured launch sequences keyed by every argument they were captured with
  // (the ranking sweeps): replayed only when a call repeats them exactly
  struct SeqGraph {
    std::vector<uint8_t> key;
    hipGraphExec_t exec = nullptr;
  };
  SeqGraph rank_up, rank_down;
  // level-1 seeds of the next build: first vertices seed_lo .. seed_lo + seed_n - 1
  // (seed_n < 0: every vertex of the union)
  int32_t seed_lo = 0, seed_n = -1;
  DevBuf digest;  // [2] set digest of the last digest_set call
  DevBuf grp_key, grp_hist;  // last-vertex grouping: keys, per-tile histograms
  // longest-first covering: prime-path hash table, covering pairs, order,
  // coverers per path, round states, chosen list
  DevBuf cov_keys, cov_vals, cov_misc, pair_p, pair_q, cov_pos, gstate0, gstate1, cov_flag;
  // components and prime-path types: Tarjan scratch, labels, flags, counters
  // (n_comp int32 at 0, type counts u64 at 64), a host path set's copy, types
  DevBuf scc_work, scc_comp, scc_flags, scc_misc, ty_off, ty_vtx, ty_types;
  // compositional method: component-graph arcs; extraction marks, counts,
  // emitted nodes and lengths, per-vertex flags and ids; the extracted sets
  // (entry-exit, exit, entry); the macro graph's vertex kinds and ids, its
  // paths' classes and lengths, selection scans; the merged sets
  DevBuf cg_cnt, cg_off, cg_src, cg_dst, cx_qb, cx_cnt0, cx_cnt1, cx_node, cx_len, cx_vfl, cx_orig;
  DevBuf cx_off[3], cx_vtx[3];
  DevBuf cm_kind, cm_orig, cm_cls, cm_len, cm_flag, cm_lens, cm_pos, cm_voff;
  DevBuf cm_off[3], cm_vtx[3];
  // the per-vertex schedule: two rounds of rows, their offsets and marks,
  // per-vertex counts, prime flags and their positions
  DevBuf pv_rows0, pv_rows1, pv_voff0, pv_voff1, pv_ext, pv_cnt, pv_flag, pv_pos;
  ExtArgs graph_args{};
  int graph_W = 0, graph_grid = 0, graph_items = 0, graph_variant = 0;
  hipStream_t graph_stream = nullptr;

  // extension-kernel launch shape per visited-set width (index = log2 of the
  // register width W): parents per thread (tile = threads * items, one output
  // claim per tile), persistent workgroups per CU and kernel variant;
  // defaults from sweeps on MI355X
  int tune_items[7] = {2, 1, 1, 1, 2, 1, 1};
  int tune_wgs[7] = {2, 2, 2, 4, 2, 2, 4};
  int tune_variant[7] = {2, 2, 2, 2, 2, 2, 0};
  double tune_ms[7] = {0, 0, 0, 0, 0, 0, 0};
};

namespace {

tpg_status ws_reserve(tpg_workspace* ws, DevBuf& b, size_t bytes, bool keep = false,
                      hipStream_t st = nullptr, size_t keep_bytes = 0) {
  if (bytes == 0) bytes = 16;
  if (b.cap >= bytes) return TPG_OK;
  if (ws->io_mode == 2) {
    ws->io_diverged = true;
    return fail(TPG_ERR_UNSUPPORTED, "the captured call needed a larger buffer");
  }
  ws->alloc_gen += 1;
  size_t want = std::max(bytes, b.cap + b.cap / 2);
  want = (want + 255) & ~(size_t)255;
  if (ws->cap && ws->bytes - b.cap + want > ws->cap) {
    want = (bytes + 255) & ~(size_t)255;
    if (ws->bytes - b.cap + want > ws->cap)
      return fail(TPG_ERR_CAPACITY, "device pool would need %zu bytes (cap %llu)",
                  ws->bytes - b.cap + want, (unsigned long long)ws->cap);
  }
  void* ptr = nullptr;
  hipError_t e = hipMalloc(&ptr, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(TPG_ERR_OOM_DEVICE, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
  }
  if (keep && b.p && keep_bytes) {
    TPG_HIP(hipMemcpyAsync(ptr, b.p, std::min(keep_bytes, b.cap), hipMemcpyDeviceToDevice, st));
    TPG_HIP(hipStreamSynchronize(st));
  }
  if (b.p) {
    TPG_HIP(hipFree(b.p));
    ws->bytes -= b.cap;
  }
  b.p = ptr;
  b.cap = want;
  ws->bytes += want;
  return TPG_OK;
}

void ws_release(tpg_workspace* ws, DevBuf& b) {
  if (b.p) {
    if (ws->io_mode == 2) {  // no free under capture; the capture is abandoned
      ws->io_diverged = true;
      return;
    }
    (void)hipFree(b.p);
    ws->bytes -= b.cap;
    ws->alloc_gen += 1;
  }
  b.p = nullptr;
  b.cap = 0;
}

// The host's reads of device values on the batched path.  An ordinary call
// copies and waits (recording the bytes in io_mode 1).  Under capture the
// value comes from the record and the graph copies the device's value into
// io_check, compared with the record after every replay.
tpg_status io_read(tpg_workspace* ws, hipStream_t st, void* dst, const void* dev, size_t bytes) {
  if (ws->io_mode == 2) {
    if (!ws->io_rec || ws->io_pos + bytes > ws->io_rec->size() ||
        ws->io_check_used + bytes > ws->io_check_cap) {
      ws->io_diverged = true;
      memset(dst, 0, bytes);
      return fail(TPG_ERR_UNSUPPORTED, "the captured call read more than the recorded one");
    }
    TPG_HIP(hipMemcpyAsync(ws->io_check + ws->io_check_used, dev, bytes, hipMemcpyDeviceToHost,
                           st));
    memcpy(dst, ws->io_rec->data() + ws->io_pos, bytes);
    ws->io_pos += bytes;
    ws->io_check_used += bytes;
    return TPG_OK;
  }
  TPG_HIP(hipMemcpyAsync(dst, dev, bytes, hipMemcpyDeviceToHost, st));
  TPG_HIP(hipStreamSynchronize(st));
  if (ws->io_mode == 1) {
    const uint8_t* p = static_cast<const uint8_t*>(dst);
    ws->io_vals.insert(ws->io_vals.end(), p, p + bytes);
  }
  return TPG_OK;
}

// A value the host decides from device state it queries (free memory):
// recorded in io_mode 1, taken from the record under capture.
void io_value(tpg_workspace* ws, int64_t& v) {
  if (ws->io_mode == 1) {
    const uint8_t* p = reinterpret_cast<const uint8_t*>(&v);
    ws->io_vals.insert(ws->io_vals.end(), p, p + sizeof v);
  } else if (ws->io_mode == 2) {
    if (!ws->io_rec || ws->io_pos + sizeof v > ws->io_rec->size() ||
        ws->io_check_used + sizeof v > ws->io_check_cap) {
      ws->io_diverged = true;
      return;
    }
    memcpy(&v, ws->io_rec->data() + ws->io_pos, sizeof v);
    // the check buffer holds it too (no device copy writes there), so the
    // values after a replay line up with the record
    memcpy(ws->io_check + ws->io_check_used, &v, sizeof v);
    ws->io_pos += sizeof v;
    ws->io_check_used += sizeof v;
  }
}

// Host data about to be uploaded on the batched path: under capture it is
// copied to pinned staging that the graph reads at every replay (in io_mode
// 1 its size is counted for that staging).
const void* io_src(tpg_workspace* ws, const void* host, size_t bytes) {
  const size_t b = (bytes + 255) & ~(size_t)255;
  if (ws->io_mode == 1) ws->io_stage_used += b;
  if (ws->io_mode != 2) return host;
  if (ws->io_stage_used + b > ws->io_stage_cap) {
    ws->io_diverged = true;
    return host;
  }
  uint8_t* at = ws->io_stage + ws->io_stage_used;
  memcpy(at, host, bytes);
  ws->io_stage_used += b;
  return at;
}

// Predicted number of paths with L + 1 entries of graph i (index 63: all
// deeper levels), from the predictor's log1p output; a value that is not a
// finite number counts as no prediction, and the log is capped so the
// count stays finite.
double predicted_paths(const float* predicted, int32_t i, int L) {
  const double x = (double)predicted[(size_t)i * 65 + L];
  if (!std::isfinite(x) || x <= 0.0) return 0.0;
  return std::expm1(std::min(x, 40.0));
}

void add_component(HostUnion& U, const tpg_graph* g) {
  const int32_t base = U.n;
  for (int32_t v = 0; v < g->n; ++v) {
    for (int32_t k = g->succ_ptr[v]; k < g->succ_ptr[v + 1]; ++k) U.s.push_back(base + g->succ[k]);
    U.sp.push_back((int32_t)U.s.size());
    for (int32_t k = g->pred_ptr[v]; k < g->pred_ptr[v + 1]; ++k) U.p.push_back(base + g->pred[k]);
    U.pp.push_back((int32_t)U.p.size());
    U.loc.push_back(v);
    U.comp.push_back(U.n_comp);
  }
  U.centry.push_back(base + g->entry);
  U.cexit.push_back(base + g->exit);
  U.n += g->n;
  U.cbase.push_back(U.n);
  U.n_comp += 1;
  U.W = std::max(U.W, pow2_words(g->n));
  U.Wu = std::max(U.Wu, (g->n + 63) / 64);
  U.uids.push_back(g->uid);
}

tpg_status upload_union(tpg_workspace* ws, const HostUnion& U, hipStream_t st) {
  // a recorded or captured call always uploads, so that every replay does
  if (ws->io_mode == 0 && ws->union_uids == U.uids) return TPG_OK;
  const size_t n1 = (size_t)U.n + 1, m = U.s.size(), nc = (size_t)U.n_comp;
  const size_t words = 2 * n1 + 2 * (m + 1) + 2 * (size_t)U.n + (nc + 1) + 2 * nc + 8;
  TPG_TRY(ws_reserve(ws, ws->g_csr, sizeof(int32_t) * words));
  int32_t* q = ws->g_csr.as<int32_t>();
  hipError_t err = hipSuccess;
  auto put = [&](const std::vector<int32_t>& v, size_t pad) -> int32_t* {
    int32_t* at = q;
    if (!v.empty() && err == hipSuccess)
      err = hipMemcpyAsync(at, io_src(ws, v.data(), sizeof(int32_t) * v.size()),
                           sizeof(int32_t) * v.size(), hipMemcpyHostToDevice, st);
    q += v.size() + pad;
    return at;
  };
  DGraph d{};
  d.sp = put(U.sp, 0);
  d.s = put(U.s, 1);
  d.pp = put(U.pp, 0);
  d.p = put(U.p, 1);
  d.loc = put(U.loc, 0);
  d.comp = put(U.comp, 0);
  d.cbase = put(U.cbase, 0);
  d.centry = put(U.centry, 0);
  d.cexit = put(U.cexit, 0);
  d.n = U.n;
  d.n_comp = U.n_comp;
  d.n_stage = (int32_t)(d.comp - d.sp);
  TPG_HIP(err);
  if (ws->io_mode != 2) TPG_HIP(hipStreamSynchronize(st));  // the host vectors are freed after
  ws->dg = d;
  ws->union_uids = U.uids;
  return TPG_OK;
}

// Buffer of the stored (odd) level L's visited sets.
int mask_buf_host(int L) { return ((L - 1) >> 1) & 1; }

// W here: words stored per visited set.
tpg_status reserve_tree(tpg_workspace* ws, int64_t rec, int64_t msk, int W, hipStream_t st,
                        int64_t keep_rec, int keep_parity, int64_t keep_mask) {
  if (rec > (int64_t)INT32_MAX - 2)
    return fail(TPG_ERR_UNSUPPORTED, "more than 2^31 simple paths in one run");
  TPG_TRY(ws_reserve(ws, ws->par, sizeof(int32_t) * rec, keep_rec > 0, st, sizeof(int32_t) * keep_rec));
  TPG_TRY(ws_reserve(ws, ws->info, sizeof(uint32_t) * rec, keep_rec > 0, st, sizeof(uint32_t) * keep_rec));
  TPG_TRY(ws_reserve(ws, ws->cstart, sizeof(int32_t) * (rec + 1), keep_rec > 0, st,
                     sizeof(int32_t) * (keep_rec + 1)));
  TPG_TRY(ws_reserve(ws, ws->nch, (size_t)rec, keep_rec > 0, st, (size_t)keep_rec));
  ws->rec_cap = std::min<int64_t>(ws->par.cap / sizeof(int32_t), ws->cstart.cap / sizeof(int32_t) - 1);
  ws->rec_cap = std::min<int64_t>(ws->rec_cap, ws->info.cap / sizeof(uint32_t));
  ws->rec_cap = std::min<int64_t>(ws->rec_cap, (int64_t)ws->nch.cap);
  ws->rec_cap = std::min<int64_t>(ws->rec_cap, kMaxTreeNodes);  // buffers may hold more
  // Visited sets are word-major (word q of slot j at q * mask_cap + j), so the
  // stride is the capacity: both buffers always have the same size, and the
  // kept level is copied to the new stride when they grow.
  const size_t need = sizeof(uint64_t) * (size_t)msk * W;
  if (ws->mask0.cap < need || ws->mask1.cap < need) {
    size_t want = std::max(need, std::max(ws->mask0.cap, ws->mask1.cap) * 3 / 2);
    want = (want + 255) & ~(size_t)255;
    const bool keep = keep_mask > 0 && keep_parity >= 0 && ws->mask_words == W;
    DevBuf& kb = keep_parity == 1 ? ws->mask1 : ws->mask0;
    DevBuf& ob = keep_parity == 1 ? ws->mask0 : ws->mask1;
    ws_release(ws, ob);
    TPG_TRY(ws_reserve(ws, ob, want));
    if (keep) {
      DevBuf nb;
      // the old buffer is freed right after the copy, as in a plain regrow
      const uint64_t cap_save = ws->cap;
      if (ws->cap) ws->cap += kb.cap;
      const tpg_status rc = ws_reserve(ws, nb, want);
      ws->cap = cap_save;
      TPG_TRY(rc);
      const size_t S_old = sizeof(uint64_t) * (size_t)ws->mask_cap;
      const size_t S_new = sizeof(uint64_t) * (want / (sizeof(uint64_t) * W));
      TPG_HIP(hipMemcpy2DAsync(nb.p, S_new, kb.p, S_old, sizeof(uint64_t) * (size_t)keep_mask, W,
                               hipMemcpyDeviceToDevice, st));
      TPG_HIP(hipStreamSynchronize(st));
      ws_release(ws, kb);
      kb = nb;
    } else {
      ws_release(ws, kb);
      TPG_TRY(ws_reserve(ws, kb, want));
    }
  }
  ws->mask_cap = (int64_t)(std::min(ws->mask0.cap, ws->mask1.cap) / (sizeof(uint64_t) * W));
  TPG_TRY(ws_reserve(ws, ws->ls, sizeof(LevelState)));
  ws->mask_words = W;
  return TPG_OK;
}

ExtArgs make_args(tpg_workspace* ws, int grid = 0) {
  ExtArgs a{};
  a.tiles_target = std::max(64, grid / 2);
  a.g = ws->dg;
  a.t.par = ws->par.as<int32_t>();
  a.t.info = ws->info.as<uint32_t>();
  a.t.cstart = ws->cstart.as<int32_t>();
  a.t.nch = ws->nch.as<uint8_t>();
  a.t.mask[0] = ws->mask0.as<uint64_t>();
  a.t.mask[1] = ws->mask1.as<uint64_t>();
  a.t.rec_cap = ws->rec_cap;
  a.t.mask_cap = ws->mask_cap;
  a.t.mask_words = ws->mask_words;
  a.ls = ws->ls.as<LevelState>();
  a.seed_lo = ws->seed_n >= 0 ? ws->seed_lo : 0;
  a.seed_n = ws->seed_n >= 0 ? ws->seed_n : ws->dg.n;
  return a;
}

tpg_status reserve_scan(tpg_workspace* ws, int64_t n) {
  TPG_TRY(ws_reserve(ws, ws->scan_status, sizeof(uint64_t) * (scan_tiles(n) + 2)));
  TPG_TRY(ws_reserve(ws, ws->scan_ctr, sizeof(uint32_t) * 4));
  TPG_TRY(ws_reserve(ws, ws->scalars, sizeof(int64_t) * 16));
  return TPG_OK;
}

struct Timer {
  tpg_workspace* ws;
  hipStream_t st;
  bool on;
  size_t next = 0;
  // an unrecorded event from the pool (for dispatch-recorded kernel timing)
  hipEvent_t event() {
    if (!on) return nullptr;
    if (next >= ws->ev_pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ws->ev_pool.push_back(e);
    }
    return ws->ev_pool[next++];
  }
  hipEvent_t mark() {
    hipEvent_t e = event();
    if (e) (void)hipEventRecord(e, st);
    return e;
  }
  static double ms(hipEvent_t a, hipEvent_t b) {
    if (!a || !b) return 0.0;
    float t = 0.f;
    if (hipEventElapsedTime(&t, a, b) != hipSuccess) return 0.0;
    return (double)t;
  }
};

struct TreeResult {
  int Lmax = 0;  // deepest level holding nodes
  std::vector<int64_t> count, off;
  int64_t n_nodes = 0;
  int64_t n_overflows = 0;
  int64_t peak = 0;
  double ms_kernel = 0.0;
  int64_t launches = 0;
};

void drop_level_graphs(tpg_workspace* ws) {
  for (auto& lg : ws->level_graphs)
    if (lg.exec) (void)hipGraphExecDestroy(lg.exec);
  ws->level_graphs.clear();
}

void drop_seq_graph(tpg_workspace::SeqGraph& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  g.exec = nullptr;
  g.key.clear();
}

template <class T>
void key_add(std::vector<uint8_t>& k, const T& v) {
  const uint8_t* p = reinterpret_cast<const uint8_t*>(&v);
  k.insert(k.end(), p, p + sizeof(T));
}

// A sequence of short launches (one per level) is issued directly the first
// time; when the next call repeats it with the same arguments it is captured
// once and from then on replayed as one graph, which removes the host's
// per-launch gap between short kernels.
template <class F>
tpg_status run_seq(tpg_workspace* ws, tpg_workspace::SeqGraph& g, std::vector<uint8_t>&& key,
                   hipStream_t st, F&& launches) {
  if (ws->io_mode == 2) {  // inside a whole-call capture: plain launches
    TPG_HIP(launches());
    return TPG_OK;
  }
  if (key != g.key) {
    drop_seq_graph(g);
    g.key = std::move(key);
    TPG_HIP(launches());
    return TPG_OK;
  }
  if (!g.exec) {
    hipGraph_t graph = nullptr;
    TPG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const hipError_t e = launches();
    const hipError_t e2 = hipStreamEndCapture(st, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      g.key.clear();
      return fail(TPG_ERR_DEVICE, "capture of a launch sequence failed: %s",
                  hipGetErrorString(e != hipSuccess ? e : e2));
    }
    const hipError_t e3 = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) {
      g.exec = nullptr;
      g.key.clear();
      TPG_HIP(e3);
    }
  }
  TPG_HIP(hipGraphLaunch(g.exec, st));
  return TPG_OK;
}

// `len` extension launches (launch li extends level batch_start + li),
// replayed from a captured HIP graph (launch arguments are baked in; a change
// of buffers or stream drops the graphs).
tpg_status launch_levels_graph(tpg_workspace* ws, const ExtArgs& a, int W, int items,
                               int variant, int grid, int len, hipStream_t st) {
  if (ws->io_mode == 2) {  // inside a whole-call capture: plain launches
    for (int i = 0; i < len; ++i) TPG_HIP(launch_extend(W, items, variant, a, grid, i, st));
    return TPG_OK;
  }
  if (memcmp(&ws->graph_args, &a, sizeof a) != 0 || ws->graph_W != W || ws->graph_grid != grid ||
      ws->graph_items != items || ws->graph_variant != variant || ws->graph_stream != st) {
    drop_level_graphs(ws);
    ws->graph_args = a;
    ws->graph_W = W;
    ws->graph_grid = grid;
    ws->graph_items = items;
    ws->graph_variant = variant;
    ws->graph_stream = st;
  }
  for (auto& lg : ws->level_graphs)
    if (lg.len == len) {
      TPG_HIP(hipGraphLaunch(lg.exec, st));
      return TPG_OK;
    }
  hipGraph_t graph = nullptr;
  TPG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  for (int i = 0; i < len; ++i) {
    hipError_t e = launch_extend(W, items, variant, a, grid, i, st);
    if (e != hipSuccess) {
      hipGraph_t g2 = nullptr;
      (void)hipStreamEndCapture(st, &g2);
      if (g2) (void)hipGraphDestroy(g2);
      return fail(TPG_ERR_DEVICE, "capture of the level loop failed: %s", hipGetErrorString(e));
    }
  }
  TPG_HIP(hipStreamEndCapture(st, &graph));
  tpg_workspace::LevelGraph lg;
  lg.len = len;
  hipError_t e = hipGraphInstantiate(&lg.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  TPG_HIP(e);
  ws->level_graphs.push_back(lg);
  TPG_HIP(hipGraphLaunch(lg.exec, st));
  return TPG_OK;
}

// Frees the path tree and the visited-set buffers (capacities back to zero).
void release_tree(tpg_workspace* ws) {
  for (DevBuf* b : {&ws->par, &ws->info, &ws->cstart, &ws->nch, &ws->mask0, &ws->mask1})
    ws_release(ws, *b);
  ws->rec_cap = 0;
  ws->mask_cap = 0;
  ws->mask_words = 0;
  drop_level_graphs(ws);
  ws->levels_uids.clear();
  ws->levels_last = 0;
}

// The device side of the one-pass level loop (see sizing.h): buffers of the
// workspace, extension launches (replayed from captured graphs, or issued
// one by one with an event pair each when the call is timed), and the level
// sizes read back after each batch.
struct OnePassDev {
  tpg_workspace* ws;
  const HostUnion& U;
  hipStream_t st;
  Timer& tm;
  TreeResult& R;
  int W, items, variant, grid;
  ExtArgs a{};
  tpg_status err = TPG_OK;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> evs;

  int64_t rec_cap() const { return ws->rec_cap; }
  int64_t mask_cap() const { return ws->mask_cap; }
  bool ok(tpg_status s) {
    err = s;
    return s == TPG_OK;
  }
  bool hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return true;
    err = fail(e == hipErrorOutOfMemory ? TPG_ERR_OOM_DEVICE : TPG_ERR_DEVICE, "%s: %s", what,
               hipGetErrorString(e));
    return false;
  }
  bool reserve(const TreeCaps& c, int64_t keep_rec, int keep_level, int64_t keep_mask) {
    if (!ok(reserve_tree(ws, c.rec, c.msk, U.Wu, st, keep_rec,
                         keep_level > 0 ? mask_buf_host(keep_level) : -1, keep_mask)))
      return false;
    a = make_args(ws, grid);
    return true;
  }
  bool run(int L0, int len, BatchReport& r) {
    LevelState* dls = ws->ls.as<LevelState>();
    ws->h_scalars[8] = L0;
    if (!hip(hipMemcpyAsync(&dls->batch_start, io_src(ws, &ws->h_scalars[8], sizeof(int32_t)),
                            sizeof(int32_t), hipMemcpyHostToDevice, st), "batch start"))
      return false;
    evs.clear();
    if (tm.on) {
      for (int b = 0; b < len; ++b) {
        hipEvent_t e0 = tm.event(), e1 = tm.event();
        if (!hip(launch_extend(W, items, variant, a, grid, b, st, e0, e1), "extension launch"))
          return false;
        evs.emplace_back(e0, e1);
      }
    } else if (!ok(launch_levels_graph(ws, a, W, items, variant, grid, len, st))) {
      return false;
    }
    // header + sizes of levels L0 .. L0 + len
    if (!ok(io_read(ws, st, ws->h_ls, dls, 32)) ||
        !ok(io_read(ws, st, ws->h_ls->count + L0, dls->count + L0, sizeof(int64_t) * (len + 1))))
      return false;
    const LevelState& h = *ws->h_ls;
    r.overflow = h.overflow != 0;
    r.overflow_level = h.overflow_level;
    r.count = h.count;
    // kernel time of the launches that extended a level for good
    const int last_ok = r.overflow ? r.overflow_level - 1 : L0 + len - 1;
    for (int b = 0; b < (int)evs.size() && L0 + b <= last_ok && h.count[L0 + b] > 0; ++b) {
      R.ms_kernel += Timer::ms(evs[b].first, evs[b].second);
      R.launches += 1;
    }
    tm.next = 0;
    return true;
  }
  bool resume(int Lo) { return hip(launch_resume_fix(a, Lo, st), "replay"); }
};

// Level loop, one-pass device-sized form.  rec0 / msk0: initial capacities
// (nodes overall / nodes of one level); 0 = what the workspace already has.
// Levels run in batches of launches (4, 8, ... 64); the host learns the
// sizes of a batch's levels after it, and grows and replays on overflow.
tpg_status build_tree_onepass(tpg_workspace* ws, const HostUnion& U, hipStream_t st, Timer& tm,
                              TreeResult& R, int64_t rec0, int64_t msk0) {
  const int W = U.W;
  const int64_t held_msk =
      (ws->mask_words && ws->mask_cap) ? ws->mask_cap * ws->mask_words / U.Wu : 0;
  const TreeCaps first = onepass_first_caps(ws->rec_cap, held_msk, U.n, rec0, msk0);
  TPG_TRY(reserve_tree(ws, first.rec, first.msk, U.Wu, st, 0, -1, 0));
  int wi = 0;
  while ((1 << wi) < W) ++wi;
  const int grid = ws->num_cus * ws->tune_wgs[wi];
  OnePassDev d{ws, U, st, tm, R, W, ws->tune_items[wi], ws->tune_variant[wi], grid};
  d.a = make_args(ws, grid);
  TPG_HIP(launch_seed(d.a, st));
  std::vector<int64_t> cnt(kMaxLevels + 1, 0);
  cnt[1] = d.a.seed_n;
  // a union seen before: one batch covers its levels and the empty one after
  const int first_batch =
      (ws->levels_uids == U.uids && ws->levels_last > 0) ? ws->levels_last + 1 : 4;
  int Lmax = 0;
  LoopFailure why;
  switch (onepass_levels(d, first_batch, kMaxLevels, cnt, Lmax, R.n_overflows, why)) {
    case LoopEnd::ok:
      break;
    case LoopEnd::device_failed:
      return d.err != TPG_OK ? d.err : fail(TPG_ERR_DEVICE, "level loop failed");
    case LoopEnd::too_deep:
      return fail(TPG_ERR_UNSUPPORTED, "more levels than vertices + 1");
    case LoopEnd::bad_report:
      return fail(TPG_ERR_DEVICE, "the device reported an overflow at level %d, outside the batch",
                  why.level);
    case LoopEnd::repeated_overflow:
      return fail(TPG_ERR_DEVICE,
                  "level %d overflowed again after growing to its exact size (base %lld, "
                  "%lld paths, %lld children; capacities %lld nodes, %lld sets)",
                  why.level, (long long)why.base, (long long)why.F, (long long)why.nxt,
                  (long long)why.rec_cap, (long long)why.mask_cap);
  }
  ws->levels_uids = U.uids;
  ws->levels_last = Lmax;
  R.count.assign(kMaxLevels, 0);
  R.off.assign(kMaxLevels, 0);
  R.Lmax = Lmax;
  int64_t off = 0;
  for (int L = 1; L <= Lmax + 1 && L < kMaxLevels; ++L) {
    R.count[L] = L <= Lmax ? cnt[L] : 0;
    R.off[L] = off;
    off += R.count[L];
    R.peak = std::max(R.peak, R.count[L]);
  }
  R.n_nodes = off;
  return TPG_OK;
}

// Level loop, plain two-pass form: count -> scan -> host reads the size -> fill.
tpg_status build_tree_twopass(tpg_workspace* ws, const HostUnion& U, hipStream_t st, Timer& tm,
                              TreeResult& R) {
  const int W = U.W;
  int64_t rec = std::max<int64_t>(ws->rec_cap, (int64_t)U.n + 4096);
  int64_t msk = (int64_t)U.n + 1024;
  if (ws->mask_words && ws->mask_cap)
    msk = std::max<int64_t>(msk, ws->mask_cap * ws->mask_words / U.Wu);
  TPG_TRY(reserve_tree(ws, rec, msk, U.Wu, st, 0, -1, 0));
  ExtArgs a = make_args(ws);
  TPG_HIP(launch_seed(a, st));
  R.count.assign(kMaxLevels, 0);
  R.off.assign(kMaxLevels, 0);
  int L = 1;
  int64_t base = 0, F = a.seed_n, prev = 0;
  R.count[1] = F;
  R.peak = F;
  for (;;) {
    TPG_TRY(reserve_scan(ws, F));
    hipEvent_t e0 = tm.mark();
    TPG_HIP(launch_count(W, a, L, prev, base, F, st));
    int32_t* cs = ws->cstart.as<int32_t>() + base;
    TPG_HIP(scan_i32_to_i32(cs, cs, F, base + F, ws->scalars.as<int64_t>(),
                            ws->scan_status.as<uint64_t>(), ws->scan_ctr.as<uint32_t>(), st));
    TPG_HIP(hipMemcpyAsync(ws->h_scalars, ws->scalars.p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    TPG_HIP(hipStreamSynchronize(st));
    const int64_t total = ws->h_scalars[0] - (base + F);
    if (total == 0) {
      hipEvent_t e1 = tm.mark();
      R.ms_kernel += Timer::ms(e0, e1);
      tm.next = 0;
      break;
    }
    // the children's visited sets are stored when they form an odd level
    const bool store_next = (L + 1) & 1;
    if (base + F + total + 1 > ws->rec_cap || (store_next && total > ws->mask_cap)) {
      const int64_t need = base + F + total + 1;
      const int Ls = (L & 1) ? L : L - 1;  // the stored level the fill reads
      TPG_TRY(reserve_tree(ws, std::max(need, std::min(std::max<int64_t>(ws->rec_cap, need + need / 2),
                                                       kMaxTreeNodes)),
                           store_next ? std::max<int64_t>(ws->mask_cap, total + total / 2) : ws->mask_cap,
                           U.Wu, st, base + F + 1, mask_buf_host(Ls), R.count[Ls]));
      a = make_args(ws);
    }
    TPG_HIP(launch_fill(W, a, L, prev, base, F, st));
    hipEvent_t e1 = tm.mark();
    TPG_HIP(hipStreamSynchronize(st));
    R.ms_kernel += Timer::ms(e0, e1);
    tm.next = 0;
    R.launches += 1;
    R.off[L + 1] = base + F;
    R.count[L + 1] = total;
    R.peak = std::max(R.peak, total);
    prev = base;
    base += F;
    F = total;
    ++L;
  }
  R.Lmax = L;
  R.off[L + 1] = base + F;
  R.n_nodes = base + F;
  return TPG_OK;
}

struct PPResult {
  int64_t n_pp = 0, n_vtx = 0, n_cycles = 0;
};

BfsOut bfs_views(tpg_workspace* ws, int n);

tpg_status rank_and_materialize(tpg_workspace* ws, const HostUnion& U, hipStream_t st,
                                const TreeResult& R, PPResult& P, OutSet& o) {
  ExtArgs a = make_args(ws);
  const int64_t N = R.n_nodes;
  TPG_TRY(ws_reserve(ws, ws->sub_cnt, sizeof(uint32_t) * N));
  TPG_TRY(ws_reserve(ws, ws->totals, sizeof(int64_t) * 4));
  TPG_TRY(ws_reserve(ws, ws->cycles, sizeof(uint64_t) * (kCycleSlots + 1)));
  uint32_t* sc = ws->sub_cnt.as<uint32_t>();
  // the levels' ranges and every buffer the sweeps touch key their graphs
  std::vector<uint8_t> key;
  key_add(key, a);
  key_add(key, sc);
  key_add(key, ws->cycles.p);
  key_add(key, ws->totals.p);
  key_add(key, U.n);
  key_add(key, R.Lmax);
  for (int L = 1; L <= R.Lmax; ++L) {
    key_add(key, R.off[L]);
    key_add(key, R.count[L]);
  }
  std::vector<uint8_t> key_down = key;
  // both sweeps take up to kRun levels per launch (a launch costs ~7 us
  // however little it does)
  constexpr int kRun = 2;  // 3 measured slower: deeper per-thread chains
  TPG_TRY(run_seq(ws, ws->rank_up, std::move(key), st, [&]() -> hipError_t {
    hipError_t e = launch_zero_u64(ws->cycles.as<uint64_t>(), kCycleSlots, st);
    unsigned long long* ncyc = ws->cycles.as<unsigned long long>();
    for (int L = R.Lmax; L >= 1 && e == hipSuccess;) {
      const int n = std::min(kRun, L);  // levels L - n + 1 .. L
      const int top = L - n + 1;
      e = n > 1 ? launch_up_run(a, n - 1, R.off[top], R.count[top], sc, ncyc, st)
                : launch_up(a, top, R.off[top], R.count[top], sc, ncyc, st);
      L -= n;
    }
    if (e == hipSuccess)
      e = launch_roots(a, R.count[1], sc, nullptr, nullptr, ws->totals.as<int64_t>(), 0, nullptr, ncyc,
                       st);
    return e;
  }));
  TPG_TRY(io_read(ws, st, ws->h_scalars, ws->totals.p, sizeof(int64_t)));
  TPG_TRY(io_read(ws, st, ws->h_scalars + 2, ws->cycles.as<uint64_t>() + kCycleSlots,
                  sizeof(int64_t)));
  P.n_pp = ws->h_scalars[0];
  P.n_cycles = ws->h_scalars[2];
  TPG_TRY(ws_reserve(ws, ws->leaf_by_rank, sizeof(int64_t) * (P.n_pp + 1)));
  TPG_TRY(ws_reserve(ws, ws->pp_len, sizeof(int32_t) * (P.n_pp + 1)));
  TPG_TRY(ws_reserve(ws, o.pp_off, sizeof(int64_t) * (P.n_pp + 1)));
  TPG_TRY(ws_reserve(ws, o.comp_starts, sizeof(int64_t) * 4 * (U.n_comp + 1)));
  TPG_TRY(reserve_scan(ws, P.n_pp));
  int64_t* lbr = ws->leaf_by_rank.as<int64_t>();
  int32_t* len = ws->pp_len.as<int32_t>();
  // with every vertex a root (in id order) the root ranks are also the test
  // paths' runs by first vertex
  int64_t* rbw = nullptr;
  if (ws->seed_lo == 0 && R.count[1] == U.n) {
    TPG_TRY(ws_reserve(ws, ws->rb0, sizeof(int64_t) * (U.n + 2)));
    rbw = ws->rb0.as<int64_t>();
  }
  ws->rb_ready = rbw != nullptr;
  key_add(key_down, lbr);
  key_add(key_down, len);
  key_add(key_down, rbw);
  TPG_TRY(run_seq(ws, ws->rank_down, std::move(key_down), st, [&]() -> hipError_t {
    hipError_t e =
        launch_roots(a, R.count[1], sc, lbr, len, ws->totals.as<int64_t>(), 1, rbw, nullptr, st);
    for (int L = 1; L < R.Lmax && e == hipSuccess;) {
      const int n = std::min(kRun, R.Lmax - L);  // parents of levels L .. L + n - 1
      e = n > 1 ? launch_down_run(a, n - 1, L, R.off[L], R.count[L], sc, lbr, len, st)
                : launch_down(a, L, R.off[L], R.count[L], sc, lbr, len, st);
      L += n;
    }
    return e;
  }));
  // offsets of the prime paths: a scan of their lengths
  int64_t* scal = ws->scalars.as<int64_t>();
  TPG_HIP(scan_i32_to_i64(len, o.pp_off.as<int64_t>(), P.n_pp, 0, scal + 6,
                          ws->scan_status.as<uint64_t>(), ws->scan_ctr.as<uint32_t>(), st));
  int64_t* cs = o.comp_starts.as<int64_t>();
  TPG_HIP(launch_comp_pp_starts(ws->dg, sc, o.pp_off.as<int64_t>(), ws->totals.as<int64_t>(), cs,
                                cs + (U.n_comp + 1), st));
  TPG_TRY(io_read(ws, st, ws->h_scalars + 6, scal + 6, sizeof(int64_t)));
  P.n_vtx = ws->h_scalars[6];
  TPG_TRY(ws_reserve(ws, o.pp_vtx, sizeof(int32_t) * (P.n_vtx + 1)));
  // with the BFS under way (test paths follow), the writer also records each
  // test path's length and where its prime path leaves the BFS tree, with
  // the entries around that point; the BFS ran beside the extension and is
  // long done
  PPWriteTp tpx{};
  ws->tp_len_ready = false;
  if (ws->bfs_pending) {
    TPG_TRY(ws_reserve(ws, ws->tp_len, sizeof(int64_t) * (P.n_pp + 1)));
    TPG_TRY(ws_reserve(ws, ws->tp_lead, sizeof(int4) * (P.n_pp + 1)));
    TPG_HIP(hipStreamWaitEvent(st, ws->ev_join, 0));
    const BfsOut bv = bfs_views(ws, U.n);
    tpx = PPWriteTp{bv.parent, bv.pfx_off, bv.sfx_off, ws->tp_len.as<int64_t>(),
                    ws->tp_lead.as<int4>()};
    ws->tp_len_ready = true;
  }
  TPG_HIP(launch_pp_write(a, lbr, o.pp_off.as<int64_t>(), P.n_pp, o.pp_vtx.as<int32_t>(), tpx,
                          st));
  o.n_pp = P.n_pp;
  o.n_ppv = P.n_vtx;
  return TPG_OK;
}

struct TPResult {
  int64_t n_spliced = 0, n_tp = 0, n_vtx = 0;
};

BfsOut bfs_views(tpg_workspace* ws, int n) {
  BfsOut b{};
  int32_t* bi = ws->bfs_i32.as<int32_t>();
  b.dist_f = bi;
  b.parent = bi + n;
  b.dist_b = bi + 2 * n;
  b.next = bi + 3 * n;
  b.pre = bi + 4 * n;
  b.pend = bi + 5 * n;
  b.cfirst = bi + 6 * n;
  b.ccnt = bi + 7 * n;
  b.bq = bi + 8 * n;
  b.pfx_off = ws->pfx_off.as<int64_t>();
  b.sfx_off = ws->sfx_off.as<int64_t>();
  return b;
}

// BFS distances, tree ranks and prefix/suffix table offsets of the uploaded
// union, on the side stream after everything already queued on `st`.
tpg_status bfs_start(tpg_workspace* ws, const HostUnion& U, hipStream_t st) {
  const int n = U.n;
  TPG_TRY(ws_reserve(ws, ws->bfs_i32, sizeof(int32_t) * 9 * (size_t)n));
  TPG_TRY(ws_reserve(ws, ws->pfx_off, sizeof(int64_t) * (n + 1)));
  TPG_TRY(ws_reserve(ws, ws->sfx_off, sizeof(int64_t) * (n + 1)));
  TPG_TRY(ws_reserve(ws, ws->scan2_status, sizeof(uint64_t) * (scan_tiles(n) + 2)));
  TPG_TRY(ws_reserve(ws, ws->scalars2, sizeof(int64_t) * 8));
  const BfsOut b = bfs_views(ws, n);
  hipStream_t side = ws->side_stream;
  int64_t* sc2 = ws->scalars2.as<int64_t>();
  TPG_HIP(hipEventRecord(ws->ev_fork, st));
  TPG_HIP(hipStreamWaitEvent(side, ws->ev_fork, 0));
  TPG_HIP(launch_bfs_dist(ws->dg, b, side));
  TPG_HIP(scan_i32_to_i64(b.dist_f, b.pfx_off, n, 0, sc2 + 0, ws->scan2_status.as<uint64_t>(),
                          nullptr, side));
  TPG_HIP(scan_i32_to_i64(b.dist_b, b.sfx_off, n, 0, sc2 + 1, ws->scan2_status.as<uint64_t>(),
                          nullptr, side));
  TPG_HIP(hipEventRecord(ws->ev_join, side));
  ws->bfs_pending = true;
  return TPG_OK;
}

// Longest-first covering (see kernels_cover.hip): from the spliced test
// paths of all np prime paths, the chosen ones in prime-path order into idx0
// and their per-first-vertex runs into rb0; *n_sel their number.
tpg_status greedy_select(tpg_workspace* ws, const HostUnion& U, hipStream_t st, int64_t np,
                         const OutSet& o, int64_t* n_sel) {
  const int n = U.n;
  int64_t* sc = ws->scalars.as<int64_t>();
  int64_t* hs = ws->h_scalars;
  TPG_TRY(ws_reserve(ws, ws->cov_misc, sizeof(uint64_t) * 4));
  uint64_t* misc = ws->cov_misc.as<uint64_t>();  // [0] shared hashes, [1] missing windows, [2] undecided
  // hash table of the prime paths, load factor <= 1/2
  int64_t slots = 1024;
  while (slots < 2 * np) slots <<= 1;
  TPG_TRY(ws_reserve(ws, ws->cov_keys, sizeof(uint64_t) * slots));
  TPG_TRY(ws_reserve(ws, ws->cov_vals, sizeof(int32_t) * slots));
  uint64_t mul = 0;
  for (int attempt = 0;; ++attempt) {
    if (attempt == 4) return fail(TPG_ERR_UNSUPPORTED, "prime-path hashes collide for 4 multipliers");
    mul = cover_hash_mul(attempt);
    TPG_HIP(launch_zero_u64(ws->cov_keys.as<uint64_t>(), slots, st));
    TPG_HIP(launch_zero_u64(misc, 4, st));
    TPG_HIP(launch_pp_hash_insert(o.pp_off.as<int64_t>(), o.pp_vtx.as<int32_t>(), np, mul,
                                  ws->cov_keys.as<uint64_t>(), ws->cov_vals.as<int32_t>(), slots - 1,
                                  misc, st));
    TPG_HIP(hipMemcpyAsync(hs + 10, misc, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    TPG_HIP(hipStreamSynchronize(st));
    if (hs[10] == 0) break;
  }
  // covering pairs: count, offsets, write
  const int64_t* tp_off = ws->tp_off.as<int64_t>();
  const int32_t* tp_vtx = ws->tp_vtx.as<int32_t>();
  TPG_TRY(ws_reserve(ws, ws->keep_cnt, sizeof(int64_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->keep_pos, sizeof(int64_t) * (np + 1)));
  int64_t* cnt = ws->keep_cnt.as<int64_t>();
  int64_t* at = ws->keep_pos.as<int64_t>();
  TPG_HIP(launch_cover(U.W, ws->dg, tp_off, tp_vtx, np, mul, ws->cov_keys.as<uint64_t>(),
                       ws->cov_vals.as<int32_t>(), slots - 1, cnt, at, nullptr, nullptr, 0, misc + 1,
                       st));
  TPG_HIP(scan_i64(cnt, at, np, 0, sc + 12, ws->scan_status.as<uint64_t>(),
                   ws->scan_ctr.as<uint32_t>(), st));
  TPG_HIP(hipMemcpyAsync(hs + 10, sc + 12, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  TPG_HIP(hipStreamSynchronize(st));
  const int64_t npairs = hs[10];
  TPG_TRY(ws_reserve(ws, ws->pair_p, sizeof(int32_t) * (npairs + 1)));
  TPG_TRY(ws_reserve(ws, ws->pair_q, sizeof(int32_t) * (npairs + 1)));
  TPG_HIP(launch_cover(U.W, ws->dg, tp_off, tp_vtx, np, mul, ws->cov_keys.as<uint64_t>(),
                       ws->cov_vals.as<int32_t>(), slots - 1, cnt, at, ws->pair_p.as<int32_t>(),
                       ws->pair_q.as<int32_t>(), 1, misc + 1, st));
  TPG_HIP(hipMemcpyAsync(hs + 11, misc + 1, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
  TPG_HIP(hipStreamSynchronize(st));
  if (hs[11] != 0)
    return fail(TPG_ERR_DEVICE, "%lld accepted windows are not prime paths", (long long)hs[11]);
  // order: decreasing length, canonical order among equal lengths
  const int64_t nt = group_tiles(np);
  const int64_t nkeys = (int64_t)n + 2;
  const int64_t nh = nkeys * std::max<int64_t>(nt, 1);
  TPG_TRY(ws_reserve(ws, ws->grp_key, sizeof(int32_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->grp_hist, sizeof(int64_t) * (nh + 1)));
  TPG_TRY(ws_reserve(ws, ws->keep_len, sizeof(int64_t) * (nh + 1)));
  TPG_TRY(ws_reserve(ws, ws->idx1, sizeof(int32_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->cov_pos, sizeof(int32_t) * (np + 1)));
  TPG_TRY(reserve_scan(ws, std::max(np, nh)));
  int32_t* key = ws->grp_key.as<int32_t>();
  int32_t* perm = ws->idx1.as<int32_t>();
  TPG_HIP(launch_len_key(o.pp_off.as<int64_t>(), np, (int64_t)n + 1, key, st));
  TPG_HIP(launch_zero_u64(ws->grp_hist.as<uint64_t>(), nh, st));
  TPG_HIP(launch_key_hist(key, np, nt, ws->grp_hist.as<uint64_t>(), st));
  TPG_HIP(scan_i64(ws->grp_hist.as<int64_t>(), ws->keep_len.as<int64_t>(), nh, 0, sc + 13,
                   ws->scan_status.as<uint64_t>(), ws->scan_ctr.as<uint32_t>(), st));
  TPG_HIP(launch_last_place(key, np, nt, ws->keep_len.as<int64_t>(), perm, st));
  TPG_HIP(launch_invert(perm, np, ws->cov_pos.as<int32_t>(), st));
  // rounds until every path is decided
  TPG_TRY(ws_reserve(ws, ws->gstate0, (size_t)np + 8));
  TPG_TRY(ws_reserve(ws, ws->gstate1, (size_t)2 * np + 16));
  uint8_t* state = ws->gstate0.as<uint8_t>();
  uint8_t* drop = ws->gstate1.as<uint8_t>();
  uint8_t* block = drop + np + 8;
  TPG_HIP(launch_zero_u32(reinterpret_cast<uint32_t*>(state), (np + 4) / 4, st));
  TPG_HIP(launch_zero_u32(reinterpret_cast<uint32_t*>(drop), (2 * np + 16) / 4, st));
  for (int64_t round = 0;; ++round) {
    if (round > np + 1) return fail(TPG_ERR_DEVICE, "covering rounds did not settle");
    TPG_HIP(launch_zero_u64(misc + 2, 1, st));
    TPG_HIP(launch_round_pairs(ws->pair_p.as<int32_t>(), ws->pair_q.as<int32_t>(), npairs,
                               ws->cov_pos.as<int32_t>(), state, drop, block, st));
    TPG_HIP(launch_round_decide(np, state, drop, block, misc + 2, st));
    TPG_HIP(hipMemcpyAsync(hs + 10, misc + 2, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    TPG_HIP(hipStreamSynchronize(st));
    if (hs[10] == 0) break;
  }
  // the chosen paths in prime-path order and their runs by first vertex
  TPG_TRY(ws_reserve(ws, ws->cov_flag, sizeof(int32_t) * (np + 1)));
  TPG_HIP(launch_chosen_flags(state, np, ws->cov_flag.as<int32_t>(), st));
  TPG_HIP(scan_i32_to_i64(ws->cov_flag.as<int32_t>(), at, np, 0, sc + 15,
                          ws->scan_status.as<uint64_t>(), ws->scan_ctr.as<uint32_t>(), st));
  TPG_HIP(launch_chosen_list(state, at, np, ws->idx0.as<int32_t>(), st));
  TPG_HIP(hipMemcpyAsync(hs + 10, sc + 15, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  TPG_HIP(hipStreamSynchronize(st));
  TPG_HIP(launch_chosen_runs(ws->idx0.as<int32_t>(), hs[10], o.pp_off.as<int64_t>(),
                             o.pp_vtx.as<int32_t>(), n, ws->rb0.as<int64_t>(), st));
  *n_sel = hs[10];
  return TPG_OK;
}

tpg_status test_paths_device(tpg_workspace* ws, const HostUnion& U, hipStream_t st,
                             const PPResult& P, TPResult& T, OutSet& o, bool greedy = false) {
  const int n = U.n;
  const int nc = U.n_comp;
  if (!ws->bfs_pending) TPG_TRY(bfs_start(ws, U, st));
  ws->bfs_pending = false;
  TPG_HIP(hipStreamWaitEvent(st, ws->ev_join, 0));
  const int64_t np = P.n_pp;
  T.n_spliced = np;
  const int eb = n > 1 ? 32 - __builtin_clz((unsigned)n) : 1;  // bits of entry + 1 <= n
  TPG_TRY(reserve_scan(ws, std::max<int64_t>(np, n)));
  BfsOut b = bfs_views(ws, n);
  int64_t* sc = ws->scalars.as<int64_t>();

  TPG_TRY(ws_reserve(ws, ws->tp_len, sizeof(int64_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->tp_off, sizeof(int64_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->rb0, sizeof(int64_t) * (n + 2)));
  TPG_TRY(ws_reserve(ws, ws->rb1, sizeof(int64_t) * (n + 2)));
  TPG_TRY(ws_reserve(ws, ws->idx0, sizeof(int32_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->idx1, sizeof(int32_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->tp_key, sizeof(uint64_t) * kTpKeyWords * (np + 1)));
  const bool from_writer = ws->tp_len_ready, rb_from_roots = ws->rb_ready;
  ws->tp_len_ready = false;
  ws->rb_ready = false;
  TPG_HIP(launch_tp_len(o.pp_off.as<int64_t>(), o.pp_vtx.as<int32_t>(), np, n, b,
                        from_writer ? nullptr : ws->tp_len.as<int64_t>(),
                        rb_from_roots ? nullptr : ws->rb0.as<int64_t>(), st));
  TPG_HIP(scan_i64(ws->tp_len.as<int64_t>(), ws->tp_off.as<int64_t>(), np, 0, sc,
                   ws->scan_status.as<uint64_t>(), ws->scan_ctr.as<uint32_t>(), st));
  TPG_TRY(io_read(ws, st, ws->h_scalars, sc, sizeof(int64_t)));
  TPG_TRY(io_read(ws, st, ws->h_scalars + 4, ws->scalars2.p, 2 * sizeof(int64_t)));
  const int64_t tp_total = ws->h_scalars[0];
  TPG_TRY(ws_reserve(ws, ws->pfx, sizeof(int32_t) * (ws->h_scalars[4] + 1)));
  TPG_TRY(ws_reserve(ws, ws->sfx, sizeof(int32_t) * (ws->h_scalars[5] + 1)));
  b.pfx = ws->pfx.as<int32_t>();
  b.sfx = ws->sfx.as<int32_t>();
  TPG_HIP(launch_bfs_tables(ws->dg, b, st));
  const int pe = 64 / eb;
  // packed rows: row v at off[v] / pe + 2 v, ceil(len / pe) + 1 words each
  TPG_TRY(ws_reserve(ws, ws->pfx_pk, sizeof(uint64_t) * (ws->h_scalars[4] / pe + 2 * (int64_t)n + 4)));
  TPG_TRY(ws_reserve(ws, ws->sfx_pk, sizeof(uint64_t) * (ws->h_scalars[5] / pe + 2 * (int64_t)n + 4)));
  b.pfx_pk = ws->pfx_pk.as<uint64_t>();
  b.sfx_pk = ws->sfx_pk.as<uint64_t>();
  TPG_HIP(launch_pack_tables(n, b, eb, st));
  // the plain spliced entries only for the covering, which reads them
  if (greedy) TPG_TRY(ws_reserve(ws, ws->tp_vtx, sizeof(int32_t) * (tp_total + 1)));
  TPG_TRY(ws_reserve(ws, ws->tp_pk, sizeof(uint64_t) * ((tp_total + pe - 1) / pe + 2 * np + 4)));
  TPG_HIP(launch_tp_write(o.pp_off.as<int64_t>(), o.pp_vtx.as<int32_t>(), np, b,
                          ws->tp_off.as<int64_t>(), greedy ? ws->tp_vtx.as<int32_t>() : nullptr,
                          ws->tp_key.as<uint64_t>(), ws->tp_pk.as<uint64_t>(), eb,
                          ws->idx0.as<int32_t>(), from_writer ? ws->tp_lead.as<int4>() : nullptr,
                          st));
  // with longest-first covering only the chosen test paths are sorted
  int64_t nm = np;
  if (greedy) TPG_TRY(greedy_select(ws, U, st, np, o, &nm));
  // merge the per-first-vertex runs
  TpOrder K{ws->tp_off.as<int64_t>(), ws->tp_key.as<uint64_t>(), ws->tp_pk.as<uint64_t>(), eb,
            pe};
  int64_t runs = n, final_runs = 1;
  TPG_TRY(ws_reserve(ws, ws->merge_split, sizeof(int64_t) * merge_split_slots(nm)));
  DevBuf* ri = &ws->rb0;
  DevBuf* ro = &ws->rb1;
  DevBuf* ii = &ws->idx0;
  DevBuf* io = &ws->idx1;
  if (nc > 1) {
    // a union of graphs: merge within each graph only (its runs padded to a
    // power of two), as the graphs' test paths already follow each other in
    // order; worth it when that takes fewer rounds
    int32_t largest = 1;
    for (int c = 0; c < nc; ++c) largest = std::max(largest, U.cbase[c + 1] - U.cbase[c]);
    int R = 0;
    while ((1 << R) < largest) ++R;
    int R_all = 0;
    while ((int64_t)1 << R_all < n) ++R_all;
    if (R < R_all) {
      const int64_t P = (int64_t)nc << R;
      TPG_TRY(ws_reserve(ws, ws->rb0, sizeof(int64_t) * (std::max<int64_t>(P, n) + 2), true, st,
                         sizeof(int64_t) * (n + 1)));
      TPG_TRY(ws_reserve(ws, ws->rb1, sizeof(int64_t) * (std::max<int64_t>(P, n) + 2)));
      TPG_HIP(launch_pad_runs(ws->dg, ws->rb0.as<int64_t>(), R, P, ws->rb1.as<int64_t>(), st));
      std::swap(ri, ro);
      runs = P;
      final_runs = nc;
    }
  }
  while (runs > final_runs) {
    TPG_HIP(launch_merge_round(K, ii->as<int32_t>(), io->as<int32_t>(), ri->as<int64_t>(), runs,
                               nm, ws->merge_split.as<int64_t>(), st));
    TPG_HIP(launch_next_runs(ri->as<int64_t>(), runs, ro->as<int64_t>(), st));
    std::swap(ri, ro);
    std::swap(ii, io);
    runs = (runs + 1) / 2;
  }
  // dedup
  TPG_TRY(ws_reserve(ws, ws->keep_cnt, sizeof(int64_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->keep_len, sizeof(int64_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->keep_pos, sizeof(int64_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->keep_voff, sizeof(int64_t) * (np + 1)));
  TPG_HIP(launch_dedup_flags(K, ii->as<int32_t>(), nm, ws->keep_cnt.as<int64_t>(),
                             ws->keep_len.as<int64_t>(), st));
  TPG_HIP(scan_i64(ws->keep_cnt.as<int64_t>(), ws->keep_pos.as<int64_t>(), nm, 0, sc + 2,
                   ws->scan_status.as<uint64_t>(), ws->scan_ctr.as<uint32_t>(), st));
  TPG_HIP(scan_i64(ws->keep_len.as<int64_t>(), ws->keep_voff.as<int64_t>(), nm, 0, sc + 3,
                   ws->scan_status.as<uint64_t>(), ws->scan_ctr.as<uint32_t>(), st));
  TPG_TRY(io_read(ws, st, ws->h_scalars + 2, sc + 2, 2 * sizeof(int64_t)));
  T.n_tp = ws->h_scalars[2];
  T.n_vtx = ws->h_scalars[3];
  TPG_TRY(ws_reserve(ws, o.tp_off, sizeof(int64_t) * (T.n_tp + 1)));
  TPG_TRY(ws_reserve(ws, o.tp_vtx, sizeof(int32_t) * (T.n_vtx + 1)));
  TPG_HIP(launch_unpack_gather(ws->tp_off.as<int64_t>(), ws->tp_pk.as<uint64_t>(),
                               o.pp_off.as<int64_t>(), o.pp_vtx.as<int32_t>(), b, eb,
                               ii->as<int32_t>(), nm, ws->keep_pos.as<int64_t>(),
                               ws->keep_voff.as<int64_t>(), ws->keep_len.as<int64_t>(),
                               o.tp_off.as<int64_t>(), o.tp_vtx.as<int32_t>(), st));
  TPG_HIP(launch_set_i64(o.tp_off.as<int64_t>() + T.n_tp, sc + 3, st));
  int64_t* cs = o.comp_starts.as<int64_t>();
  if (nc > 1)
    TPG_HIP(launch_comp_bounds(o.tp_off.as<int64_t>(), o.tp_vtx.as<int32_t>(), T.n_tp, ws->dg.comp,
                               nc, cs + 2 * (nc + 1), cs + 3 * (nc + 1), st));
  o.n_tp = T.n_tp;
  o.n_tpv = T.n_vtx;
  return TPG_OK;
}

tpg_status export_paths(const DevBuf& off, const DevBuf& vtx, int64_t n, int64_t nv, bool device,
                        hipStream_t st, tpg_paths* out) {
  memset(out, 0, sizeof *out);
  out->n_paths = n;
  out->n_vertices = nv;
  if (device) {
    out->on_device = 1;
    out->offsets = off.as<int64_t>();
    out->vertices = vtx.as<int32_t>();
    return TPG_OK;
  }
  out->offsets = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
  out->vertices = (int32_t*)malloc(sizeof(int32_t) * (nv > 0 ? nv : 1));
  if (!out->offsets || !out->vertices) {
    free(out->offsets);
    free(out->vertices);
    memset(out, 0, sizeof *out);
    return fail(TPG_ERR_OOM_HOST, "result arrays");
  }
  TPG_HIP(hipMemcpyAsync(out->offsets, off.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, st));
  if (nv)
    TPG_HIP(hipMemcpyAsync(out->vertices, vtx.p, sizeof(int32_t) * nv, hipMemcpyDeviceToHost, st));
  TPG_HIP(hipStreamSynchronize(st));
  return TPG_OK;
}

// The canonical prime paths regrouped by last vertex (stable, so each
// group keeps the canonical order) into o.ppg_off / o.ppg_vtx: a counting
// sort over n_keys vertex ids, then a flattened gather of the rows.
tpg_status group_by_last(tpg_workspace* ws, int32_t n_keys, hipStream_t st, OutSet& o, int64_t np,
                         int64_t nv) {
  const int64_t nt = group_tiles(np);
  const int64_t nh = (int64_t)n_keys * std::max<int64_t>(nt, 1);
  TPG_TRY(ws_reserve(ws, ws->grp_key, sizeof(int32_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->grp_hist, sizeof(int64_t) * (nh + 1)));
  TPG_TRY(ws_reserve(ws, ws->keep_len, sizeof(int64_t) * (std::max(np, nh) + 1)));
  TPG_TRY(ws_reserve(ws, ws->keep_pos, sizeof(int64_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->keep_voff, sizeof(int64_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->idx0, sizeof(int32_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, o.ppg_off, sizeof(int64_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, o.ppg_vtx, sizeof(int32_t) * (nv + 1)));
  TPG_TRY(reserve_scan(ws, std::max(np, nh)));
  int64_t* sc = ws->scalars.as<int64_t>();
  uint64_t* hist = ws->grp_hist.as<uint64_t>();
  int64_t* base = ws->keep_len.as<int64_t>();  // the scanned histograms
  int32_t* perm = ws->idx0.as<int32_t>();
  TPG_HIP(launch_zero_u64(hist, nh, st));
  TPG_HIP(launch_last_hist(o.pp_off.as<int64_t>(), o.pp_vtx.as<int32_t>(), np, nt,
                           ws->grp_key.as<int32_t>(), hist, st));
  TPG_HIP(scan_i64(reinterpret_cast<const int64_t*>(hist), base, nh, 0, sc + 10,
                   ws->scan_status.as<uint64_t>(), ws->scan_ctr.as<uint32_t>(), st));
  TPG_HIP(launch_last_place(ws->grp_key.as<int32_t>(), np, nt, base, perm, st));
  // row lengths in the new order (reusing the histogram buffer is safe: the
  // placement above has consumed it), their offsets, then the rows
  int64_t* len = ws->keep_len.as<int64_t>();
  TPG_HIP(launch_perm_lens(o.pp_off.as<int64_t>(), perm, np, len, ws->keep_pos.as<int64_t>(), st));
  TPG_HIP(scan_i64(len, ws->keep_voff.as<int64_t>(), np, 0, sc + 11, ws->scan_status.as<uint64_t>(),
                   ws->scan_ctr.as<uint32_t>(), st));
  TPG_HIP(launch_gather(o.pp_off.as<int64_t>(), o.pp_vtx.as<int32_t>(), perm, np,
                        ws->keep_pos.as<int64_t>(), ws->keep_voff.as<int64_t>(), len,
                        o.ppg_off.as<int64_t>(), o.ppg_vtx.as<int32_t>(), st));
  TPG_HIP(launch_set_i64(o.ppg_off.as<int64_t>() + np, sc + 11, st));
  return TPG_OK;
}

// Digest of paths [0, n) of a device set (see tpg_paths.digest).
tpg_status digest_set(tpg_workspace* ws, const DevBuf& off, const DevBuf& vtx, int64_t n,
                      hipStream_t st, uint64_t out[2]) {
  TPG_TRY(ws_reserve(ws, ws->digest, 2 * sizeof(uint64_t)));
  TPG_HIP(launch_digest(off.as<int64_t>(), vtx.as<int32_t>(), n, ws->digest.as<uint64_t>(), st));
  TPG_HIP(hipMemcpyAsync(ws->h_scalars + 12, ws->digest.p, 2 * sizeof(uint64_t),
                         hipMemcpyDeviceToHost, st));
  TPG_HIP(hipStreamSynchronize(st));
  out[0] = (uint64_t)ws->h_scalars[12];
  out[1] = (uint64_t)ws->h_scalars[13];
  return TPG_OK;
}

// Result set into *out as the flags ask: arrays (host or device), digest.
tpg_status deliver_set(tpg_workspace* ws, const DevBuf& off, const DevBuf& vtx, int64_t n,
                       int64_t nv, uint32_t flags, hipStream_t st, tpg_paths* out) {
  uint64_t dg[2] = {0, 0};
  if (flags & (TPG_DIGEST | TPG_DIGEST_ONLY)) TPG_TRY(digest_set(ws, off, vtx, n, st, dg));
  if (flags & TPG_DIGEST_ONLY) {
    memset(out, 0, sizeof *out);
    out->n_paths = n;
    out->n_vertices = nv;
  } else {
    TPG_TRY(export_paths(off, vtx, n, nv, flags & TPG_OUT_DEVICE, st, out));
  }
  out->digest[0] = dg[0];
  out->digest[1] = dg[1];
  return TPG_OK;
}

struct CallCtx {
  tpg_workspace* ws = nullptr;
  bool own_ws = false;
  hipStream_t st = nullptr;
  uint32_t flags = 0;
  tpg_stats* stats = nullptr;
  const tpg_opts* opts = nullptr;
  ~CallCtx() {
    if (own_ws && ws) tpg_workspace_free(ws);
  }
};

tpg_status begin_call(const tpg_opts* opts, CallCtx& c) {
  if (opts && opts->struct_size != sizeof(tpg_opts))
    return fail(TPG_ERR_INVALID_ARG, "opts.struct_size = %u, expected %zu", opts->struct_size,
                sizeof(tpg_opts));
  c.opts = opts;
  c.flags = opts ? opts->flags : 0;
  c.stats = opts ? opts->stats : nullptr;
  if (opts && opts->ws) {
    c.ws = opts->ws;
  } else {
    TPG_TRY(tpg_workspace_create(-1, &c.ws));
    c.own_ws = true;
  }
  TPG_HIP(hipSetDevice(c.ws->device));
  c.st = (opts && opts->stream) ? (hipStream_t)opts->stream : c.ws->own_stream;
  c.ws->cap = opts ? opts->pool_cap_bytes : 0;
  if (c.ws->cap && c.ws->bytes > c.ws->cap)
    return fail(TPG_ERR_CAPACITY, "workspace already holds %zu bytes (cap %llu)", c.ws->bytes,
                (unsigned long long)c.ws->cap);
  if (c.ws->out.empty()) c.ws->out.resize(1);
  c.ws->seed_lo = 0;
  c.ws->seed_n = -1;
  return TPG_OK;
}

tpg_status run_pp(const HostUnion& U, CallCtx& c, Timer& tm, TreeResult& R, PPResult& P,
                  OutSet& o, hipEvent_t* e_ext, int64_t rec0 = 0, int64_t msk0 = 0,
                  bool with_bfs = false) {
  TPG_TRY(upload_union(c.ws, U, c.st));
  c.ws->bfs_pending = false;
  if (with_bfs) TPG_TRY(bfs_start(c.ws, U, c.st));
  if (c.flags & TPG_FORCE_TWO_PASS)
    TPG_TRY(build_tree_twopass(c.ws, U, c.st, tm, R));
  else
    TPG_TRY(build_tree_onepass(c.ws, U, c.st, tm, R, rec0, msk0));
  if (e_ext) *e_ext = tm.mark();
  TPG_TRY(rank_and_materialize(c.ws, U, c.st, R, P, o));
  return TPG_OK;
}

void add_stats(tpg_stats* s, const HostUnion& U, const TreeResult& R, const PPResult& P,
               const TPResult* T) {
  s->n_levels = std::max<int64_t>(s->n_levels, R.Lmax);
  s->n_nodes += R.n_nodes;
  s->n_extensions += R.n_nodes - R.count[1];
  s->n_cycles += P.n_cycles;
  s->n_pp += P.n_pp;
  s->n_pp_vertices += P.n_vtx;
  if (T) {
    s->n_tp_spliced += T->n_spliced;
    s->n_tp += T->n_tp;
    s->n_tp_vertices += T->n_vtx;
  }
  s->n_overflows += R.n_overflows;
  s->ms_extend_kernel += R.ms_kernel;
  s->n_extend_launches += R.launches;
  s->peak_level_nodes = std::max<int64_t>(s->peak_level_nodes, R.peak);
  s->n_unions += 1;
}

tpg_status check_graph(const tpg_graph* g) {
  if (!g) return fail(TPG_ERR_INVALID_ARG, "graph is NULL");
  return TPG_OK;
}

// Hands one chunk to the caller: host copies (freed right after the call)
// or device pointers.
tpg_status call_chunk(CallCtx& c, const tpg_paths& chunk, int64_t first, int64_t end) {
  const int32_t r = c.opts->on_chunk(c.opts->chunk_ctx, &chunk, first, end);
  if (r != 0) return fail(TPG_ERR_CALLBACK, "on_chunk returned %d for [%lld, %lld)", r,
                          (long long)first, (long long)end);
  return TPG_OK;
}

// TPG_STREAM for prime paths: the first vertices in ranges of
// chunk_vertices, each range a fresh path tree (so device memory is bounded
// by the largest range's tree); prime paths grouped by first vertex are
// exactly the canonical order's consecutive blocks, so the chunks
// concatenate to the canonical set.
tpg_status prime_paths_stream(const tpg_graph* g, CallCtx& c, tpg_paths* out) {
  if (!c.opts || !c.opts->on_chunk) return fail(TPG_ERR_INVALID_ARG, "TPG_STREAM needs opts.on_chunk");
  if (c.opts->chunk_vertices < 0) return fail(TPG_ERR_INVALID_ARG, "chunk_vertices < 0");
  HostUnion U;
  add_component(U, g);
  const int32_t cv = c.opts->chunk_vertices > 0 ? c.opts->chunk_vertices : 32;
  Timer tm{c.ws, c.st, false};
  tpg_stats acc{};
  std::vector<int64_t> levels;
  uint64_t dg[2] = {0, 0};
  OutSet& o = c.ws->out[0];
  for (int32_t lo = 0; lo < U.n; lo += cv) {
    c.ws->seed_lo = lo;
    c.ws->seed_n = std::min(cv, U.n - lo);
    TreeResult R;
    PPResult P;
    TPG_TRY(run_pp(U, c, tm, R, P, o, nullptr));
    uint64_t cd[2];
    TPG_TRY(digest_set(c.ws, o.pp_off, o.pp_vtx, P.n_pp, c.st, cd));
    dg[0] += cd[0];
    dg[1] ^= cd[1];
    tpg_paths chunk;
    TPG_TRY(export_paths(o.pp_off, o.pp_vtx, P.n_pp, P.n_vtx, c.flags & TPG_OUT_DEVICE, c.st, &chunk));
    chunk.digest[0] = cd[0];
    chunk.digest[1] = cd[1];
    const tpg_status rc = call_chunk(c, chunk, lo, lo + c.ws->seed_n);
    tpg_paths_free(&chunk);
    TPG_TRY(rc);
    out->n_paths += P.n_pp;
    out->n_vertices += P.n_vtx;
    add_stats(&acc, U, R, P, nullptr);
    if ((int)levels.size() <= R.Lmax) levels.resize(R.Lmax + 1, 0);
    for (int L = 1; L <= R.Lmax; ++L) levels[L] += R.count[L];
  }
  c.ws->seed_n = -1;
  out->digest[0] = dg[0];
  out->digest[1] = dg[1];
  if (c.stats) {
    *c.stats = acc;
    c.stats->n_unions = 1;
    c.stats->device_bytes = (int64_t)c.ws->bytes;
  }
  if (c.opts->level_counts)
    for (int L = 0; L < c.opts->level_counts_len; ++L)
      c.opts->level_counts[L] = L < (int)levels.size() ? levels[L] : 0;
  return TPG_OK;
}

// TPG_STREAM for test paths: the canonical set in chunks of chunk_paths,
// each with offsets rebased to its own entries.
tpg_status test_paths_stream_out(CallCtx& c, const OutSet& o, int64_t n_tp) {
  if (c.opts->chunk_paths < 0) return fail(TPG_ERR_INVALID_ARG, "chunk_paths < 0");
  const int64_t cp = c.opts->chunk_paths > 0 ? c.opts->chunk_paths : (int64_t)1 << 20;
  const bool dev = c.flags & TPG_OUT_DEVICE;
  std::vector<int64_t> off;
  std::vector<int32_t> vtx;
  DevBuf& doff = c.ws->tp_len;  // scratch for rebased device offsets (free after the sort)
  if (dev) TPG_TRY(ws_reserve(c.ws, doff, sizeof(int64_t) * (std::min(cp, n_tp) + 1)));
  for (int64_t k = 0; k < n_tp; k += cp) {
    const int64_t cnt = std::min(cp, n_tp - k);
    off.resize(cnt + 1);
    TPG_HIP(hipMemcpyAsync(off.data(), o.tp_off.as<int64_t>() + k, sizeof(int64_t) * (cnt + 1),
                           hipMemcpyDeviceToHost, c.st));
    TPG_HIP(hipStreamSynchronize(c.st));
    const int64_t v0 = off[0], nv = off[cnt] - v0;
    for (auto& x : off) x -= v0;
    tpg_paths chunk;
    memset(&chunk, 0, sizeof chunk);
    chunk.n_paths = cnt;
    chunk.n_vertices = nv;
    if (dev) {
      TPG_HIP(hipMemcpyAsync(doff.p, off.data(), sizeof(int64_t) * (cnt + 1), hipMemcpyHostToDevice,
                             c.st));
      TPG_HIP(hipStreamSynchronize(c.st));
      chunk.on_device = 1;
      chunk.offsets = doff.as<int64_t>();
      chunk.vertices = o.tp_vtx.as<int32_t>() + v0;
    } else {
      vtx.resize(nv > 0 ? nv : 1);
      if (nv)
        TPG_HIP(hipMemcpyAsync(vtx.data(), o.tp_vtx.as<int32_t>() + v0, sizeof(int32_t) * nv,
                               hipMemcpyDeviceToHost, c.st));
      TPG_HIP(hipStreamSynchronize(c.st));
      chunk.offsets = off.data();
      chunk.vertices = vtx.data();
    }
    TPG_TRY(call_chunk(c, chunk, k, k + cnt));
  }
  return TPG_OK;
}

}  // namespace

extern "C" {

int32_t tpg_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

tpg_status tpg_workspace_create(int32_t device, tpg_workspace** out) {
  if (!out) return fail(TPG_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return fail(TPG_ERR_DEVICE, "no HIP device available");
  }
  if (device < 0) TPG_HIP(hipGetDevice(&device));
  if (device >= ndev) return fail(TPG_ERR_INVALID_ARG, "device %d of %d", device, ndev);
  tpg_workspace* ws = new (std::nothrow) tpg_workspace;
  if (!ws) return fail(TPG_ERR_OOM_HOST, "workspace");
  ws->device = device;
  TPG_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) ws->num_cus = prop.multiProcessorCount;
  if (hipStreamCreateWithFlags(&ws->own_stream, hipStreamNonBlocking) != hipSuccess) {
    delete ws;
    return fail(TPG_ERR_DEVICE, "hipStreamCreate failed");
  }
  if (hipStreamCreateWithFlags(&ws->side_stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&ws->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ws->ev_join, hipEventDisableTiming) != hipSuccess) {
    tpg_workspace_free(ws);
    return fail(TPG_ERR_DEVICE, "side stream / events");
  }
  if (hipHostMalloc((void**)&ws->h_ls, sizeof(LevelState), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&ws->h_scalars, sizeof(int64_t) * 16, hipHostMallocDefault) != hipSuccess) {
    tpg_workspace_free(ws);
    return fail(TPG_ERR_OOM_HOST, "pinned host buffers");
  }
  ws->out.resize(1);
  *out = ws;
  return TPG_OK;
}

void tpg_workspace_free(tpg_workspace* ws) {
  if (!ws) return;
  (void)hipSetDevice(ws->device);
  if (ws->own_stream) (void)hipStreamSynchronize(ws->own_stream);
  if (ws->side_stream) (void)hipStreamSynchronize(ws->side_stream);
  if (ws->cg.exec) (void)hipGraphExecDestroy(ws->cg.exec);
  if (ws->io_check) (void)hipHostFree(ws->io_check);
  if (ws->io_stage) (void)hipHostFree(ws->io_stage);
  DevBuf* bufs[] = {&ws->g_csr, &ws->par, &ws->info, &ws->cstart, &ws->nch, &ws->mask0,
                    &ws->mask1, &ws->ls, &ws->sub_cnt, &ws->pp_len,
                    &ws->leaf_by_rank, &ws->totals, &ws->cycles, &ws->scan_status,
                    &ws->scan_ctr, &ws->scalars, &ws->bfs_i32, &ws->pfx_off, &ws->sfx_off,
                    &ws->pfx, &ws->sfx, &ws->pfx_pk, &ws->sfx_pk, &ws->tp_len, &ws->tp_off, &ws->tp_vtx, &ws->tp_key, &ws->tp_pk, &ws->idx0,
                    &ws->idx1, &ws->grp_cnt, &ws->rb0, &ws->rb1, &ws->merge_split, &ws->tp_lead, &ws->keep_cnt, &ws->keep_len,
                    &ws->keep_pos, &ws->keep_voff, &ws->comp_cnt, &ws->lvl_comp, &ws->b_pp_off,
                    &ws->scan2_status, &ws->scalars2, &ws->digest, &ws->grp_key, &ws->grp_hist,
                    &ws->cov_keys, &ws->cov_vals, &ws->cov_misc, &ws->pair_p, &ws->pair_q,
                    &ws->cov_pos, &ws->gstate0, &ws->gstate1, &ws->cov_flag,
                    &ws->scc_work, &ws->scc_comp, &ws->scc_flags, &ws->scc_misc, &ws->ty_off,
                    &ws->ty_vtx, &ws->ty_types, &ws->cg_cnt, &ws->cg_off, &ws->cg_src,
                    &ws->cg_dst, &ws->cx_qb, &ws->cx_cnt0, &ws->cx_cnt1, &ws->cx_node,
                    &ws->cx_len, &ws->cx_vfl, &ws->cx_orig, &ws->cx_off[0], &ws->cx_off[1],
                    &ws->cx_off[2], &ws->cx_vtx[0], &ws->cx_vtx[1], &ws->cx_vtx[2],
                    &ws->cm_kind, &ws->cm_orig, &ws->cm_cls, &ws->cm_len, &ws->cm_flag,
                    &ws->cm_lens, &ws->cm_pos, &ws->cm_voff, &ws->cm_off[0], &ws->cm_off[1],
                    &ws->cm_off[2], &ws->cm_vtx[0], &ws->cm_vtx[1], &ws->cm_vtx[2],
                    &ws->pv_rows0, &ws->pv_rows1, &ws->pv_voff0, &ws->pv_voff1, &ws->pv_ext,
                    &ws->pv_cnt, &ws->pv_flag, &ws->pv_pos,
                    &ws->b_pp_vtx, &ws->b_tp_off, &ws->b_tp_vtx, &ws->b_desc};
  for (DevBuf* b : bufs) ws_release(ws, *b);
  for (OutSet& o : ws->out) {
    ws_release(ws, o.pp_off);
    ws_release(ws, o.pp_vtx);
    ws_release(ws, o.tp_off);
    ws_release(ws, o.tp_vtx);
    ws_release(ws, o.ppg_off);
    ws_release(ws, o.ppg_vtx);
    ws_release(ws, o.comp_starts);
  }
  for (hipEvent_t e : ws->ev_pool) (void)hipEventDestroy(e);
  drop_level_graphs(ws);
  drop_seq_graph(ws->rank_up);
  drop_seq_graph(ws->rank_down);
  if (ws->h_ls) (void)hipHostFree(ws->h_ls);
  if (ws->h_scalars) (void)hipHostFree(ws->h_scalars);
  if (ws->own_stream) (void)hipStreamDestroy(ws->own_stream);
  if (ws->side_stream) (void)hipStreamDestroy(ws->side_stream);
  if (ws->ev_fork) (void)hipEventDestroy(ws->ev_fork);
  if (ws->ev_join) (void)hipEventDestroy(ws->ev_join);
  delete ws;
}

int64_t tpg_workspace_bytes(const tpg_workspace* ws) { return ws ? (int64_t)ws->bytes : 0; }

tpg_status tpg_prime_paths(const tpg_graph* g, const tpg_opts* opts, tpg_paths* out) {
  if (!out) return fail(TPG_ERR_INVALID_ARG, "out is NULL");
  memset(out, 0, sizeof *out);
  TPG_TRY(check_graph(g));
  CallCtx c;
  TPG_TRY(begin_call(opts, c));
  if ((c.flags & TPG_STREAM) && (c.flags & TPG_ORDER_BY_LAST))
    return fail(TPG_ERR_INVALID_ARG, "TPG_ORDER_BY_LAST cannot be streamed by first vertex");
  if (c.flags & TPG_STREAM) return prime_paths_stream(g, c, out);
  HostUnion U;
  add_component(U, g);
  Timer tm{c.ws, c.st, c.stats != nullptr && !(c.flags & TPG_NO_TIMING)};
  const bool timing = tm.on;
  std::vector<hipEvent_t> phase(2, nullptr);
  if (timing) {
    for (auto& e : phase) TPG_HIP(hipEventCreate(&e));
    TPG_HIP(hipEventRecord(phase[0], c.st));
  }
  TreeResult R;
  PPResult P;
  hipEvent_t ext_done = nullptr;
  OutSet& o = c.ws->out[0];
  tpg_status s = run_pp(U, c, tm, R, P, o, &ext_done);
  if (s == TPG_OK && (c.flags & TPG_ORDER_BY_LAST)) s = group_by_last(c.ws, U.n, c.st, o, P.n_pp, P.n_vtx);
  if (s == TPG_OK && timing) TPG_HIP(hipEventRecord(phase[1], c.st));
  const bool grouped = c.flags & TPG_ORDER_BY_LAST;
  if (s == TPG_OK)
    s = deliver_set(c.ws, grouped ? o.ppg_off : o.pp_off, grouped ? o.ppg_vtx : o.pp_vtx, P.n_pp,
                    P.n_vtx, c.flags, c.st, out);
  if (s == TPG_OK) {
    TPG_HIP(hipStreamSynchronize(c.st));
    if (c.stats) {
      memset(c.stats, 0, sizeof *c.stats);
      add_stats(c.stats, U, R, P, nullptr);
      c.stats->device_bytes = (int64_t)c.ws->bytes;
      if (timing) {
        c.stats->ms_extend = Timer::ms(phase[0], ext_done);
        c.stats->ms_rank = Timer::ms(ext_done, phase[1]);
        c.stats->ms_total = Timer::ms(phase[0], phase[1]);
      }
    }
    if (c.opts && c.opts->level_counts)
      for (int L = 0; L < c.opts->level_counts_len; ++L)
        c.opts->level_counts[L] = (L <= R.Lmax && L < (int)R.count.size()) ? R.count[L] : 0;
  }
  for (auto& e : phase)
    if (e) (void)hipEventDestroy(e);
  return s;
}

// Components of the uploaded graph (union) into the workspace's scc buffers.
tpg_status scc_device(tpg_workspace* ws, const HostUnion& U, hipStream_t st) {
  const int64_t n = std::max<int64_t>(ws->dg.n, 1);
  TPG_TRY(ws_reserve(ws, ws->scc_work, sizeof(int32_t) * 6 * n));
  TPG_TRY(ws_reserve(ws, ws->scc_comp, sizeof(int32_t) * n));
  TPG_TRY(ws_reserve(ws, ws->scc_flags, n));
  TPG_TRY(ws_reserve(ws, ws->scc_misc, 64 + sizeof(uint64_t) * kPpTypes));
  TPG_HIP(launch_scc(ws->dg, (int32_t)U.s.size(), ws->scc_work.as<int32_t>(),
                     ws->scc_comp.as<int32_t>(),
                     ws->scc_flags.as<uint8_t>(), ws->scc_misc.as<int32_t>(), st));
  return TPG_OK;
}

tpg_status tpg_scc(const tpg_graph* g, const tpg_opts* opts, int32_t* comp, uint8_t* flags,
                   int32_t* n_comp) {
  TPG_TRY(check_graph(g));
  CallCtx c;
  TPG_TRY(begin_call(opts, c));
  HostUnion U;
  add_component(U, g);
  TPG_TRY(upload_union(c.ws, U, c.st));
  TPG_TRY(scc_device(c.ws, U, c.st));
  if (comp)
    TPG_HIP(hipMemcpyAsync(comp, c.ws->scc_comp.p, sizeof(int32_t) * U.n, hipMemcpyDeviceToHost,
                           c.st));
  if (flags) TPG_HIP(hipMemcpyAsync(flags, c.ws->scc_flags.p, U.n, hipMemcpyDeviceToHost, c.st));
  int32_t nc = 0;
  TPG_HIP(hipMemcpyAsync(&nc, c.ws->scc_misc.p, sizeof nc, hipMemcpyDeviceToHost, c.st));
  TPG_HIP(hipStreamSynchronize(c.st));
  if (n_comp) *n_comp = nc;
  return TPG_OK;
}

tpg_status tpg_prime_path_types(const tpg_graph* g, const tpg_paths* pps, const tpg_opts* opts,
                                uint8_t* types, int64_t* counts) {
  TPG_TRY(check_graph(g));
  if (!pps) return fail(TPG_ERR_INVALID_ARG, "pps is NULL");
  const int64_t np = pps->n_paths, nv = pps->n_vertices;
  if (np < 0 || nv < 0 || (np > 0 && (!pps->offsets || !pps->vertices)))
    return fail(TPG_ERR_INVALID_ARG, "malformed path set");
  if (!pps->on_device && np > 0) {
    const int64_t* off = pps->offsets;
    if (off[0] != 0 || off[np] != nv) return fail(TPG_ERR_INVALID_ARG, "offsets do not span the set");
    for (int64_t i = 0; i < np; ++i)
      if (off[i + 1] <= off[i]) return fail(TPG_ERR_INVALID_ARG, "path %lld is empty", (long long)i);
    for (int64_t k = 0; k < nv; ++k)
      if (pps->vertices[k] < 0 || pps->vertices[k] >= g->n)
        return fail(TPG_ERR_INVALID_ARG, "vertex %d outside the graph", pps->vertices[k]);
  }
  CallCtx c;
  TPG_TRY(begin_call(opts, c));
  tpg_workspace* ws = c.ws;
  HostUnion U;
  add_component(U, g);
  TPG_TRY(upload_union(ws, U, c.st));
  TPG_TRY(scc_device(ws, U, c.st));
  const int64_t* d_off = pps->offsets;
  const int32_t* d_vtx = pps->vertices;
  if (!pps->on_device && np > 0) {
    TPG_TRY(ws_reserve(ws, ws->ty_off, sizeof(int64_t) * (np + 1)));
    TPG_TRY(ws_reserve(ws, ws->ty_vtx, sizeof(int32_t) * nv));
    TPG_HIP(hipMemcpyAsync(ws->ty_off.p, pps->offsets, sizeof(int64_t) * (np + 1),
                           hipMemcpyHostToDevice, c.st));
    TPG_HIP(hipMemcpyAsync(ws->ty_vtx.p, pps->vertices, sizeof(int32_t) * nv,
                           hipMemcpyHostToDevice, c.st));
    d_off = ws->ty_off.as<int64_t>();
    d_vtx = ws->ty_vtx.as<int32_t>();
  }
  uint8_t* d_types = nullptr;
  if (types && np > 0) {
    TPG_TRY(ws_reserve(ws, ws->ty_types, np));
    d_types = ws->ty_types.as<uint8_t>();
  }
  unsigned long long* d_cnt = (unsigned long long*)(ws->scc_misc.as<uint8_t>() + 64);
  TPG_HIP(launch_pp_types(ws->dg, ws->scc_comp.as<int32_t>(), ws->scc_flags.as<uint8_t>(), d_off,
                          d_vtx, np, d_types, d_cnt, c.st));
  if (d_types) TPG_HIP(hipMemcpyAsync(types, d_types, np, hipMemcpyDeviceToHost, c.st));
  uint64_t h_cnt[kPpTypes];
  TPG_HIP(hipMemcpyAsync(h_cnt, d_cnt, sizeof h_cnt, hipMemcpyDeviceToHost, c.st));
  TPG_HIP(hipStreamSynchronize(c.st));
  if (counts)
    for (int t = 0; t < kPpTypes; ++t) counts[t] = (int64_t)h_cnt[t];
  return TPG_OK;
}

// ---------------------------------------------------------------------------
// compositional method (Sec. 2.1): component graph, extraction, merge
// ---------------------------------------------------------------------------
namespace {

// Components of g on the device; labels and flags back on the host.
tpg_status components_host(CallCtx& c, const tpg_graph* g, std::vector<int32_t>& comp,
                           std::vector<uint8_t>& flags) {
  HostUnion U;
  add_component(U, g);
  TPG_TRY(upload_union(c.ws, U, c.st));
  TPG_TRY(scc_device(c.ws, U, c.st));
  comp.assign(g->n, 0);
  flags.assign(g->n, 0);
  TPG_HIP(hipMemcpyAsync(comp.data(), c.ws->scc_comp.p, sizeof(int32_t) * g->n,
                         hipMemcpyDeviceToHost, c.st));
  TPG_HIP(hipMemcpyAsync(flags.data(), c.ws->scc_flags.p, g->n, hipMemcpyDeviceToHost, c.st));
  TPG_HIP(hipStreamSynchronize(c.st));
  return TPG_OK;
}

// The components with a cycle, each taken alone (the arcs between its
// vertices; reversed with rev), as one disjoint union in ascending label
// order; inside a component the vertices keep g's order, so the path tree's
// order is the lexicographic order in g's ids.
struct ComponentUnion {
  std::vector<tpg_graph*> gs;
  std::vector<int32_t> orig;  // union vertex -> vertex of g
  std::vector<uint8_t> vfl;   // union vertex: bit 0 SccEntryVertex, bit 1 SccExitVertex
  ~ComponentUnion() {
    for (tpg_graph* h : gs) tpg_graph_free(h);
  }
};

tpg_status component_union(const tpg_graph* g, const std::vector<int32_t>& comp,
                           const std::vector<uint8_t>& fl, bool rev, ComponentUnion& S,
                           HostUnion& U) {
  std::map<int32_t, std::vector<int32_t>> members;
  for (int32_t v = 0; v < g->n; ++v)
    if (fl[v] & kSccCyclic) members[comp[v]].push_back(v);
  std::vector<int32_t> loc(g->n, -1);
  for (auto& kv : members) {
    const std::vector<int32_t>& vs = kv.second;
    const int32_t k = (int32_t)vs.size();
    for (int32_t i = 0; i < k; ++i) loc[vs[i]] = i;
    std::vector<std::vector<int32_t>> rows(k);
    for (int32_t i = 0; i < k; ++i)
      for (int32_t e = g->succ_ptr[vs[i]]; e < g->succ_ptr[vs[i] + 1]; ++e) {
        const int32_t w = g->succ[e];
        if (comp[w] != kv.first) continue;
        if (rev)
          rows[loc[w]].push_back(i);
        else
          rows[i].push_back(loc[w]);
      }
    std::vector<int64_t> rp(k + 1, 0);
    std::vector<int32_t> ci;
    for (int32_t i = 0; i < k; ++i) {
      ci.insert(ci.end(), rows[i].begin(), rows[i].end());
      rp[i + 1] = (int64_t)ci.size();
    }
    tpg_graph* h = nullptr;
    TPG_TRY(tpg_load_cfg_csr(k, rp.data(), ci.data(), 0, k - 1, TPG_LOAD_ANY_DIGRAPH, &h));
    S.gs.push_back(h);
    add_component(U, h);
    for (int32_t v : vs) {
      S.orig.push_back(v);
      S.vfl.push_back((uint8_t)(((fl[v] & kSccEntryVertex) ? 1 : 0) |
                                ((fl[v] & kSccExitVertex) ? 2 : 0)));
    }
  }
  return TPG_OK;
}

// Defs. 6-8 on the device (see kernels_compose.hip) into ws->cx_off / cx_vtx:
// slot 0 the SccEntryExitPaths, 1 the SccExitPaths, 2 the SccEntryPaths.
tpg_status extract_device(CallCtx& c, const tpg_graph* g, const std::vector<int32_t>& comp,
                          const std::vector<uint8_t>& fl, int64_t n_out[3], int64_t nv_out[3]) {
  tpg_workspace* ws = c.ws;
  hipStream_t st = c.st;
  for (int rev = 0; rev < 2; ++rev) {
    ComponentUnion S;
    HostUnion U;
    TPG_TRY(component_union(g, comp, fl, rev != 0, S, U));
    const int nsets = rev ? 1 : 2;
    const int slot[2] = {rev ? 1 : 0, 2};
    TPG_TRY(reserve_scan(ws, 16));
    int64_t* scal = ws->scalars.as<int64_t>();
    if (U.n == 0) {
      for (int s = 0; s < nsets; ++s) {
        TPG_TRY(ws_reserve(ws, ws->cx_off[slot[s]], sizeof(int64_t)));
        TPG_TRY(ws_reserve(ws, ws->cx_vtx[slot[s]], sizeof(int32_t)));
        TPG_HIP(launch_zero_u64(ws->cx_off[slot[s]].as<uint64_t>(), 1, st));
        n_out[slot[s]] = nv_out[slot[s]] = 0;
      }
      continue;
    }
    TPG_TRY(upload_union(ws, U, st));
    ws->seed_lo = 0;
    ws->seed_n = -1;
    TreeResult R;
    Timer tm{ws, st, false};
    if (c.flags & TPG_FORCE_TWO_PASS)
      TPG_TRY(build_tree_twopass(ws, U, st, tm, R));
    else
      TPG_TRY(build_tree_onepass(ws, U, st, tm, R, 0, 0));
    const int64_t N = R.n_nodes;
    TPG_TRY(ws_reserve(ws, ws->cx_qb, (size_t)N + 1));
    TPG_TRY(ws_reserve(ws, ws->cx_cnt0, sizeof(uint32_t) * (N + 1)));
    TPG_TRY(ws_reserve(ws, ws->cx_cnt1, sizeof(uint32_t) * (N + 1)));
    TPG_TRY(ws_reserve(ws, ws->cx_vfl, (size_t)U.n));
    TPG_TRY(ws_reserve(ws, ws->cx_orig, sizeof(int32_t) * U.n));
    TPG_HIP(hipMemcpyAsync(ws->cx_vfl.p, S.vfl.data(), U.n, hipMemcpyHostToDevice, st));
    TPG_HIP(hipMemcpyAsync(ws->cx_orig.p, S.orig.data(), sizeof(int32_t) * U.n,
                           hipMemcpyHostToDevice, st));
    const ExtArgs a = make_args(ws);
    uint8_t* qb = ws->cx_qb.as<uint8_t>();
    uint32_t* cnt[2] = {ws->cx_cnt0.as<uint32_t>(), ws->cx_cnt1.as<uint32_t>()};
    for (int L = R.Lmax; L >= 1; --L)
      TPG_HIP(launch_ex_up(a, R.off[L], R.count[L], ws->cx_vfl.as<uint8_t>(), rev, qb, cnt[0],
                           nsets > 1 ? cnt[1] : nullptr, st));
    for (int s = 0; s < nsets; ++s) {
      TPG_HIP(launch_ex_roots(cnt[s], R.count[1], scal, st));
      TPG_HIP(hipMemcpyAsync(ws->h_scalars, scal, sizeof(int64_t), hipMemcpyDeviceToHost, st));
      TPG_HIP(hipStreamSynchronize(st));
      const int64_t np = ws->h_scalars[0];
      TPG_TRY(ws_reserve(ws, ws->cx_node, sizeof(int64_t) * (np + 1)));
      TPG_TRY(ws_reserve(ws, ws->cx_len, sizeof(int32_t) * (np + 1)));
      for (int L = 1; L <= R.Lmax; ++L)
        TPG_HIP(launch_ex_down(a, L, R.off[L], R.count[L], qb, cnt[s], rev, s,
                               ws->cx_node.as<int64_t>(), ws->cx_len.as<int32_t>(), st));
      DevBuf& off = ws->cx_off[slot[s]];
      TPG_TRY(ws_reserve(ws, off, sizeof(int64_t) * (np + 1)));
      TPG_TRY(reserve_scan(ws, std::max<int64_t>(np, 16)));
      scal = ws->scalars.as<int64_t>();
      TPG_HIP(scan_i32_to_i64(ws->cx_len.as<int32_t>(), off.as<int64_t>(), np, 0, scal + 1,
                              ws->scan_status.as<uint64_t>(), ws->scan_ctr.as<uint32_t>(), st));
      TPG_HIP(launch_set_i64(off.as<int64_t>() + np, scal + 1, st));
      TPG_HIP(hipMemcpyAsync(ws->h_scalars + 1, scal + 1, sizeof(int64_t), hipMemcpyDeviceToHost,
                             st));
      TPG_HIP(hipStreamSynchronize(st));
      const int64_t nv = ws->h_scalars[1];
      DevBuf& vtx = ws->cx_vtx[slot[s]];
      TPG_TRY(ws_reserve(ws, vtx, sizeof(int32_t) * (nv + 1)));
      TPG_HIP(launch_ex_write(a, ws->cx_node.as<int64_t>(), off.as<int64_t>(), np, rev,
                              ws->cx_orig.as<int32_t>(), vtx.as<int32_t>(), st));
      n_out[slot[s]] = np;
      nv_out[slot[s]] = nv;
    }
  }
  TPG_HIP(hipStreamSynchronize(st));
  return TPG_OK;
}

struct HostSet {
  std::vector<int64_t> off;
  std::vector<int32_t> vtx;
  int64_t size() const { return (int64_t)off.size() - 1; }
};

tpg_status fetch_set(const DevBuf& off, const DevBuf& vtx, int64_t n, int64_t nv, hipStream_t st,
                     HostSet& h) {
  h.off.assign(n + 1, 0);
  h.vtx.assign(nv, 0);
  TPG_HIP(hipMemcpyAsync(h.off.data(), off.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, st));
  if (nv) TPG_HIP(hipMemcpyAsync(h.vtx.data(), vtx.p, sizeof(int32_t) * nv, hipMemcpyDeviceToHost, st));
  TPG_HIP(hipStreamSynchronize(st));
  return TPG_OK;
}

// A prefix trie of paths: node = a prefix; end bits mark the paths that end
// at a node (bit 0 SccEntryExitPath, 1 SccEntryPath, 2 SccExitPath).
struct PathTrie {
  std::vector<int32_t> v;
  std::vector<uint8_t> end;
  std::vector<std::vector<int32_t>> kids;
  std::map<std::pair<int32_t, int32_t>, int32_t> at;  // (parent or -1, vertex) -> node
  void add(const HostSet& h, uint8_t bit) {
    for (int64_t i = 0; i < h.size(); ++i) {
      int32_t x = -1;
      for (int64_t k = h.off[i]; k < h.off[i + 1]; ++k) {
        const auto key = std::make_pair(x, h.vtx[k]);
        auto it = at.find(key);
        if (it == at.end()) {
          const int32_t id = (int32_t)v.size();
          v.push_back(h.vtx[k]);
          end.push_back(0);
          kids.emplace_back();
          if (x >= 0) kids[x].push_back(id);
          it = at.emplace(key, id).first;
        }
        x = it->second;
      }
      if (x >= 0) end[x] |= bit;
    }
  }
  int32_t root(int32_t vertex) const {
    auto it = at.find(std::make_pair(-1, vertex));
    return it == at.end() ? -1 : it->second;
  }
};

}  // namespace

tpg_status tpg_ccfg(const tpg_graph* g, const tpg_opts* opts, int32_t* comp, int32_t* n_comp,
                    int64_t* n_arcs, int32_t* arc_src, int32_t* arc_dst, int64_t arc_cap) {
  TPG_TRY(check_graph(g));
  if (!n_arcs) return fail(TPG_ERR_INVALID_ARG, "n_arcs is NULL");
  CallCtx c;
  TPG_TRY(begin_call(opts, c));
  tpg_workspace* ws = c.ws;
  HostUnion U;
  add_component(U, g);
  TPG_TRY(upload_union(ws, U, c.st));
  TPG_TRY(scc_device(ws, U, c.st));
  const int n = g->n;
  TPG_TRY(ws_reserve(ws, ws->cg_cnt, sizeof(int32_t) * (n + 1)));
  TPG_TRY(ws_reserve(ws, ws->cg_off, sizeof(int64_t) * (n + 1)));
  TPG_TRY(reserve_scan(ws, std::max(n, 16)));
  int64_t* scal = ws->scalars.as<int64_t>();
  const int32_t* d_comp = ws->scc_comp.as<int32_t>();
  TPG_HIP(launch_ccfg_count(ws->dg, d_comp, ws->cg_cnt.as<int32_t>(), c.st));
  TPG_HIP(scan_i32_to_i64(ws->cg_cnt.as<int32_t>(), ws->cg_off.as<int64_t>(), n, 0, scal,
                          ws->scan_status.as<uint64_t>(), ws->scan_ctr.as<uint32_t>(), c.st));
  int32_t nc = 0;
  TPG_HIP(hipMemcpyAsync(ws->h_scalars, scal, sizeof(int64_t), hipMemcpyDeviceToHost, c.st));
  TPG_HIP(hipMemcpyAsync(&nc, ws->scc_misc.p, sizeof nc, hipMemcpyDeviceToHost, c.st));
  TPG_HIP(hipStreamSynchronize(c.st));
  const int64_t na = ws->h_scalars[0];
  *n_arcs = na;
  if (n_comp) *n_comp = nc;
  if (comp)
    TPG_HIP(hipMemcpyAsync(comp, d_comp, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c.st));
  if (arc_src || arc_dst) {
    if (!arc_src || !arc_dst) return fail(TPG_ERR_INVALID_ARG, "arc_src and arc_dst go together");
    if (na > arc_cap)
      return fail(TPG_ERR_CAPACITY, "%lld component-graph arcs, room for %lld", (long long)na,
                  (long long)arc_cap);
    TPG_TRY(ws_reserve(ws, ws->cg_src, sizeof(int32_t) * (na + 1)));
    TPG_TRY(ws_reserve(ws, ws->cg_dst, sizeof(int32_t) * (na + 1)));
    TPG_HIP(launch_ccfg_write(ws->dg, d_comp, ws->cg_off.as<int64_t>(), ws->cg_src.as<int32_t>(),
                              ws->cg_dst.as<int32_t>(), c.st));
    if (na) {
      TPG_HIP(hipMemcpyAsync(arc_src, ws->cg_src.p, sizeof(int32_t) * na, hipMemcpyDeviceToHost,
                             c.st));
      TPG_HIP(hipMemcpyAsync(arc_dst, ws->cg_dst.p, sizeof(int32_t) * na, hipMemcpyDeviceToHost,
                             c.st));
    }
  }
  TPG_HIP(hipStreamSynchronize(c.st));
  return TPG_OK;
}

tpg_status tpg_scc_paths(const tpg_graph* g, const tpg_opts* opts, tpg_paths* entry_exit,
                         tpg_paths* exit_paths, tpg_paths* entry_paths) {
  for (tpg_paths* p : {entry_exit, exit_paths, entry_paths})
    if (p) memset(p, 0, sizeof *p);
  TPG_TRY(check_graph(g));
  CallCtx c;
  TPG_TRY(begin_call(opts, c));
  std::vector<int32_t> comp;
  std::vector<uint8_t> fl;
  TPG_TRY(components_host(c, g, comp, fl));
  int64_t n[3], nv[3];
  TPG_TRY(extract_device(c, g, comp, fl, n, nv));
  tpg_paths* outs[3] = {entry_exit, exit_paths, entry_paths};
  for (int s = 0; s < 3; ++s)
    if (outs[s])
      TPG_TRY(export_paths(c.ws->cx_off[s], c.ws->cx_vtx[s], n[s], nv[s],
                           (c.flags & TPG_OUT_DEVICE) != 0, c.st, outs[s]));
  return TPG_OK;
}

tpg_status tpg_scc_internal_pps(const tpg_graph* g, const tpg_opts* opts, tpg_paths* out) {
  if (!out) return fail(TPG_ERR_INVALID_ARG, "out is NULL");
  memset(out, 0, sizeof *out);
  TPG_TRY(check_graph(g));
  CallCtx c;
  TPG_TRY(begin_call(opts, c));
  tpg_workspace* ws = c.ws;
  hipStream_t st = c.st;
  std::vector<int32_t> comp;
  std::vector<uint8_t> fl;
  TPG_TRY(components_host(c, g, comp, fl));
  ComponentUnion S;
  HostUnion U;
  TPG_TRY(component_union(g, comp, fl, false, S, U));
  DevBuf& ooff = ws->cm_off[0];
  DevBuf& ovtx = ws->cm_vtx[0];
  if (U.n == 0) {
    TPG_TRY(ws_reserve(ws, ooff, sizeof(int64_t)));
    TPG_TRY(ws_reserve(ws, ovtx, sizeof(int32_t)));
    TPG_HIP(launch_zero_u64(ooff.as<uint64_t>(), 1, st));
    return export_paths(ooff, ovtx, 0, 0, (c.flags & TPG_OUT_DEVICE) != 0, st, out);
  }
  // the extension on every component alone (one union), then Def. 9
  Timer tm{ws, st, false};
  TreeResult R;
  PPResult P;
  OutSet& o = ws->out[0];
  TPG_TRY(run_pp(U, c, tm, R, P, o, nullptr));
  const int64_t np = P.n_pp;
  TPG_TRY(ws_reserve(ws, ws->cx_vfl, (size_t)U.n));
  TPG_TRY(ws_reserve(ws, ws->cx_orig, sizeof(int32_t) * U.n));
  TPG_HIP(hipMemcpyAsync(ws->cx_vfl.p, S.vfl.data(), U.n, hipMemcpyHostToDevice, st));
  TPG_HIP(hipMemcpyAsync(ws->cx_orig.p, S.orig.data(), sizeof(int32_t) * U.n,
                         hipMemcpyHostToDevice, st));
  TPG_TRY(ws_reserve(ws, ws->cm_cls, (size_t)np + 1));
  TPG_TRY(ws_reserve(ws, ws->cm_len, sizeof(int32_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->cm_flag, sizeof(int32_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->cm_lens, sizeof(int32_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->cm_pos, sizeof(int64_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->cm_voff, sizeof(int64_t) * (np + 1)));
  TPG_HIP(launch_internal_class(o.pp_off.as<int64_t>(), o.pp_vtx.as<int32_t>(), np,
                                ws->cx_vfl.as<uint8_t>(), ws->cm_cls.as<uint8_t>(),
                                ws->cm_len.as<int32_t>(), st));
  TPG_TRY(reserve_scan(ws, std::max<int64_t>(np, 16)));
  int64_t* scal = ws->scalars.as<int64_t>();
  TPG_HIP(launch_merge_sel(ws->cm_cls.as<uint8_t>(), ws->cm_len.as<int32_t>(), np, 1,
                           ws->cm_flag.as<int32_t>(), ws->cm_lens.as<int32_t>(), st));
  TPG_HIP(scan_i32_to_i64(ws->cm_flag.as<int32_t>(), ws->cm_pos.as<int64_t>(), np, 0, scal + 2,
                          ws->scan_status.as<uint64_t>(), ws->scan_ctr.as<uint32_t>(), st));
  TPG_HIP(scan_i32_to_i64(ws->cm_lens.as<int32_t>(), ws->cm_voff.as<int64_t>(), np, 0, scal + 3,
                          ws->scan_status.as<uint64_t>(), ws->scan_ctr.as<uint32_t>(), st));
  TPG_HIP(hipMemcpyAsync(ws->h_scalars + 2, scal + 2, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  TPG_HIP(hipStreamSynchronize(st));
  const int64_t k = ws->h_scalars[2], kv = ws->h_scalars[3];
  TPG_TRY(ws_reserve(ws, ooff, sizeof(int64_t) * (k + 1)));
  TPG_TRY(ws_reserve(ws, ovtx, sizeof(int32_t) * (kv + 1)));
  TPG_HIP(launch_merge_emit(o.pp_off.as<int64_t>(), o.pp_vtx.as<int32_t>(), np,
                            ws->cm_cls.as<uint8_t>(), 1, ws->cm_pos.as<int64_t>(),
                            ws->cm_voff.as<int64_t>(), ws->cm_len.as<int32_t>(),
                            ws->cx_orig.as<int32_t>(), ooff.as<int64_t>(), ovtx.as<int32_t>(), st));
  TPG_HIP(launch_set_i64(ooff.as<int64_t>() + k, scal + 3, st));
  TPG_HIP(hipStreamSynchronize(st));
  return export_paths(ooff, ovtx, k, kv, (c.flags & TPG_OUT_DEVICE) != 0, st, out);
}

tpg_status tpg_merged_pps(const tpg_graph* g, const tpg_opts* opts, tpg_paths* complete,
                          tpg_paths* exit_pps, tpg_paths* entry_pps) {
  for (tpg_paths* p : {complete, exit_pps, entry_pps})
    if (p) memset(p, 0, sizeof *p);
  TPG_TRY(check_graph(g));
  if (g->load_flags & TPG_LOAD_ANY_DIGRAPH)
    return fail(TPG_ERR_UNREACHABLE, "the merge needs a CFG loaded with the entry/exit checks");
  CallCtx c;
  TPG_TRY(begin_call(opts, c));
  tpg_workspace* ws = c.ws;
  hipStream_t st = c.st;
  std::vector<int32_t> comp;
  std::vector<uint8_t> fl;
  TPG_TRY(components_host(c, g, comp, fl));
  int64_t n[3], nv[3];
  TPG_TRY(extract_device(c, g, comp, fl, n, nv));
  HostSet ee, ex, en;
  TPG_TRY(fetch_set(ws->cx_off[0], ws->cx_vtx[0], n[0], nv[0], st, ee));
  TPG_TRY(fetch_set(ws->cx_off[1], ws->cx_vtx[1], n[1], nv[1], st, ex));
  TPG_TRY(fetch_set(ws->cx_off[2], ws->cx_vtx[2], n[2], nv[2], st, en));

  // The macro graph H (graph preparation on the host): a vertex for every
  // vertex of g outside the components with a cycle; the trie of the
  // SccEntryExitPaths and SccEntryPaths (they start at SccEntryVertices); the
  // trie of the SccExitPaths; a terminal mark after every node where an
  // SccEntryPath ends.  Arcs: g's arcs out of the vertices outside the
  // components, trie arcs, and g's arcs that leave a component out of every
  // node where an SccEntryExitPath or an SccExitPath ends; an arc into a
  // component lands on the trie root of the vertex it enters.  H is acyclic
  // and its prime paths are the merged candidates: from the entry to the
  // exit (complete), from an exit-path trie root to the exit, from the entry
  // to a terminal mark.  H's ids follow g's vertex order (terminal marks
  // first), and the successors of an H vertex are distinct vertices of g, so
  // the lexicographic order of H's paths is that of the paths in g.
  PathTrie tin, tex;
  tin.add(ee, 1);
  tin.add(en, 2);
  tex.add(ex, 4);
  const int32_t n0 = g->n;
  const int32_t b_in = n0, b_ex = b_in + (int32_t)tin.v.size();
  const int32_t b_mk = b_ex + (int32_t)tex.v.size();
  std::vector<int32_t> mark_of(tin.v.size(), -1);
  int32_t nh = b_mk;
  for (size_t x = 0; x < tin.v.size(); ++x)
    if (tin.end[x] & 2) mark_of[x] = nh++;
  std::vector<uint8_t> kind(nh, 0);
  std::vector<int32_t> horig(nh, -1);
  for (int32_t v = 0; v < n0; ++v) horig[v] = v;  // ids of cyclic vertices stay unused
  for (size_t x = 0; x < tin.v.size(); ++x) {
    kind[b_in + x] = 1;
    horig[b_in + x] = tin.v[x];
  }
  for (size_t x = 0; x < tex.v.size(); ++x) {
    kind[b_ex + x] = 2;
    horig[b_ex + x] = tex.v[x];
  }
  for (int32_t h = b_mk; h < nh; ++h) kind[h] = 3;
  auto target = [&](int32_t w) -> int32_t {
    if (!(fl[w] & kSccCyclic)) return w;
    const int32_t r = tin.root(w);
    return r < 0 ? -1 : b_in + r;
  };
  std::vector<std::vector<int32_t>> adj(nh);
  std::vector<uint8_t> live(nh, 1);
  for (int32_t v = 0; v < n0; ++v) {
    if (fl[v] & kSccCyclic) {
      live[v] = 0;
      continue;
    }
    for (int32_t e = g->succ_ptr[v]; e < g->succ_ptr[v + 1]; ++e) {
      const int32_t t = target(g->succ[e]);
      if (t >= 0) adj[v].push_back(t);
    }
  }
  auto leave_arcs = [&](int32_t h, int32_t a) {
    for (int32_t e = g->succ_ptr[a]; e < g->succ_ptr[a + 1]; ++e) {
      const int32_t w = g->succ[e];
      if (comp[w] == comp[a]) continue;
      const int32_t t = target(w);
      if (t >= 0) adj[h].push_back(t);
    }
  };
  for (size_t x = 0; x < tin.v.size(); ++x) {
    const int32_t h = b_in + (int32_t)x;
    for (int32_t k : tin.kids[x]) adj[h].push_back(b_in + k);
    if (tin.end[x] & 1) leave_arcs(h, tin.v[x]);
    if (tin.end[x] & 2) adj[h].push_back(mark_of[x]);
  }
  for (size_t x = 0; x < tex.v.size(); ++x) {
    const int32_t h = b_ex + (int32_t)x;
    for (int32_t k : tex.kids[x]) adj[h].push_back(b_ex + k);
    if (tex.end[x] & 4) leave_arcs(h, tex.v[x]);
  }
  // renumber: live vertices by (vertex of g, kind, id); terminal marks first
  std::vector<int32_t> order;
  for (int32_t h = 0; h < nh; ++h)
    if (live[h]) order.push_back(h);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    if (horig[x] != horig[y]) return horig[x] < horig[y];
    return kind[x] < kind[y];
  });
  const int32_t nH = (int32_t)order.size();
  if (nH > TPG_MAX_VERTICES)
    return fail(TPG_ERR_UNSUPPORTED, "the merge graph has %d vertices (at most %d)", nH,
                TPG_MAX_VERTICES);
  std::vector<int32_t> nid(nh, -1);
  for (int32_t i = 0; i < nH; ++i) nid[order[i]] = i;
  std::vector<int64_t> rp(nH + 1, 0);
  std::vector<int32_t> ci;
  std::vector<uint8_t> hk(nH);
  std::vector<int32_t> ho(nH);
  for (int32_t i = 0; i < nH; ++i) {
    const int32_t h = order[i];
    for (int32_t t : adj[h]) ci.push_back(nid[t]);
    rp[i + 1] = (int64_t)ci.size();
    hk[i] = kind[h];
    ho[i] = horig[h];
  }
  if (ci.empty()) ci.push_back(0);
  tpg_graph* H = nullptr;
  TPG_TRY(tpg_load_cfg_csr(nH, rp.data(), ci.data(), nid[g->entry], nid[g->exit],
                           TPG_LOAD_ANY_DIGRAPH, &H));
  struct Free {
    tpg_graph* h;
    ~Free() { tpg_graph_free(h); }
  } free_h{H};
  // prime paths of H on the device
  HostUnion UH;
  add_component(UH, H);
  Timer tm{ws, st, false};
  TreeResult R;
  PPResult P;
  OutSet& o = ws->out[0];
  TPG_TRY(run_pp(UH, c, tm, R, P, o, nullptr));
  // classify them in g (its CSR back on the device), keep the prime ones
  HostUnion UG;
  add_component(UG, g);
  TPG_TRY(upload_union(ws, UG, st));
  const int64_t np = P.n_pp;
  TPG_TRY(ws_reserve(ws, ws->cm_kind, (size_t)nH));
  TPG_TRY(ws_reserve(ws, ws->cm_orig, sizeof(int32_t) * nH));
  TPG_TRY(ws_reserve(ws, ws->cm_cls, (size_t)np + 1));
  TPG_TRY(ws_reserve(ws, ws->cm_len, sizeof(int32_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->cm_flag, sizeof(int32_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->cm_lens, sizeof(int32_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->cm_pos, sizeof(int64_t) * (np + 1)));
  TPG_TRY(ws_reserve(ws, ws->cm_voff, sizeof(int64_t) * (np + 1)));
  TPG_HIP(hipMemcpyAsync(ws->cm_kind.p, hk.data(), nH, hipMemcpyHostToDevice, st));
  TPG_HIP(hipMemcpyAsync(ws->cm_orig.p, ho.data(), sizeof(int32_t) * nH, hipMemcpyHostToDevice, st));
  TPG_HIP(launch_merge_class(o.pp_off.as<int64_t>(), o.pp_vtx.as<int32_t>(), np,
                             ws->cm_kind.as<uint8_t>(), ws->cm_orig.as<int32_t>(), ws->dg,
                             nid[g->entry], nid[g->exit], ws->cm_cls.as<uint8_t>(),
                             ws->cm_len.as<int32_t>(), st));
  TPG_TRY(reserve_scan(ws, std::max<int64_t>(np, 16)));
  int64_t* scal = ws->scalars.as<int64_t>();
  const int cls_of[3] = {1, 3, 4};
  tpg_paths* outs[3] = {complete, exit_pps, entry_pps};
  for (int s = 0; s < 3; ++s) {
    TPG_HIP(launch_merge_sel(ws->cm_cls.as<uint8_t>(), ws->cm_len.as<int32_t>(), np, cls_of[s],
                             ws->cm_flag.as<int32_t>(), ws->cm_lens.as<int32_t>(), st));
    TPG_HIP(scan_i32_to_i64(ws->cm_flag.as<int32_t>(), ws->cm_pos.as<int64_t>(), np, 0, scal + 2,
                            ws->scan_status.as<uint64_t>(), ws->scan_ctr.as<uint32_t>(), st));
    TPG_HIP(scan_i32_to_i64(ws->cm_lens.as<int32_t>(), ws->cm_voff.as<int64_t>(), np, 0, scal + 3,
                            ws->scan_status.as<uint64_t>(), ws->scan_ctr.as<uint32_t>(), st));
    TPG_HIP(hipMemcpyAsync(ws->h_scalars + 2, scal + 2, 2 * sizeof(int64_t), hipMemcpyDeviceToHost,
                           st));
    TPG_HIP(hipStreamSynchronize(st));
    const int64_t k = ws->h_scalars[2], kv = ws->h_scalars[3];
    TPG_TRY(ws_reserve(ws, ws->cm_off[s], sizeof(int64_t) * (k + 1)));
    TPG_TRY(ws_reserve(ws, ws->cm_vtx[s], sizeof(int32_t) * (kv + 1)));
    TPG_HIP(launch_merge_emit(o.pp_off.as<int64_t>(), o.pp_vtx.as<int32_t>(), np,
                              ws->cm_cls.as<uint8_t>(), cls_of[s], ws->cm_pos.as<int64_t>(),
                              ws->cm_voff.as<int64_t>(), ws->cm_len.as<int32_t>(),
                              ws->cm_orig.as<int32_t>(), ws->cm_off[s].as<int64_t>(),
                              ws->cm_vtx[s].as<int32_t>(), st));
    TPG_HIP(launch_set_i64(ws->cm_off[s].as<int64_t>() + k, scal + 3, st));
    if (outs[s])
      TPG_TRY(export_paths(ws->cm_off[s], ws->cm_vtx[s], k, kv, (c.flags & TPG_OUT_DEVICE) != 0, st,
                           outs[s]));
  }
  TPG_HIP(hipStreamSynchronize(st));
  return TPG_OK;
}

tpg_status tpg_prime_paths_vertex_lists(const tpg_graph* g, const tpg_opts* opts,
                                        tpg_paths* out) {
  if (!out) return fail(TPG_ERR_INVALID_ARG, "out is NULL");
  memset(out, 0, sizeof *out);
  TPG_TRY(check_graph(g));
  CallCtx c;
  TPG_TRY(begin_call(opts, c));
  if (c.flags & (TPG_STREAM | TPG_TP_GREEDY))
    return fail(TPG_ERR_INVALID_ARG, "the per-vertex schedule is not streamed");
  tpg_workspace* ws = c.ws;
  hipStream_t st = c.st;
  HostUnion U;
  add_component(U, g);
  TPG_TRY(upload_union(ws, U, st));
  const int n = U.n;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool timing = c.stats && !(c.flags & TPG_NO_TIMING);
  if (timing) {
    TPG_HIP(hipEventCreate(&e0));
    TPG_HIP(hipEventCreate(&e1));
    TPG_HIP(hipEventRecord(e0, st));
  }
  OutSet& o = ws->out[0];
  DevBuf* rows = &ws->pv_rows0;
  DevBuf* nrows = &ws->pv_rows1;
  DevBuf* voff = &ws->pv_voff0;
  DevBuf* nvoff = &ws->pv_voff1;
  TPG_TRY(ws_reserve(ws, *voff, sizeof(int64_t) * (n + 1)));
  TPG_TRY(ws_reserve(ws, *nvoff, sizeof(int64_t) * (n + 1)));
  TPG_TRY(ws_reserve(ws, *rows, sizeof(int32_t) * n));
  TPG_TRY(ws_reserve(ws, ws->pv_cnt, sizeof(int32_t) * (n + 1)));
  TPG_TRY(ws_reserve(ws, o.pp_off, sizeof(int64_t) * 1024));
  TPG_TRY(ws_reserve(ws, o.pp_vtx, sizeof(int32_t) * 1024));
  TPG_TRY(reserve_scan(ws, n));
  TPG_HIP(launch_pv_init(n, voff->as<int64_t>(), rows->as<int32_t>(), st));
  int64_t* sc = ws->scalars.as<int64_t>();
  int64_t n_rows = n, n_pp = 0, n_vtx = 0, n_ext = 0, levels = 0;
  for (int L = 1; n_rows > 0; ++L) {
    if (L >= kMaxLevels) return fail(TPG_ERR_UNSUPPORTED, "more levels than supported");
    levels = L;
    // round L + 1: counts, offsets, rows; round L's rows get their marks
    TPG_TRY(ws_reserve(ws, ws->pv_ext, (n_rows + 8) & ~(int64_t)7));
    TPG_HIP(launch_zero_u64(ws->pv_ext.as<uint64_t>(), (n_rows + 7) / 8, st));
    TPG_HIP(launch_pv_count(ws->dg, L, voff->as<int64_t>(), rows->as<int32_t>(),
                            ws->pv_cnt.as<int32_t>(), st));
    TPG_HIP(scan_i32_to_i64(ws->pv_cnt.as<int32_t>(), nvoff->as<int64_t>(), n, 0, sc,
                            ws->scan_status.as<uint64_t>(), ws->scan_ctr.as<uint32_t>(), st));
    TPG_HIP(launch_set_i64(nvoff->as<int64_t>() + n, sc, st));
    TPG_HIP(hipMemcpyAsync(ws->h_scalars, sc, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    TPG_HIP(hipStreamSynchronize(st));
    const int64_t n_next = ws->h_scalars[0];
    if (n_next > 0) {
      TPG_TRY(ws_reserve(ws, *nrows, sizeof(int32_t) * n_next * (L + 1)));
      TPG_HIP(launch_pv_fill(ws->dg, L, voff->as<int64_t>(), rows->as<int32_t>(),
                             ws->pv_ext.as<uint8_t>(), nvoff->as<int64_t>(),
                             nrows->as<int32_t>(), st));
    }
    // round L is final: append its prime rows
    TPG_TRY(ws_reserve(ws, ws->pv_flag, sizeof(int32_t) * (n_rows + 1)));
    TPG_TRY(ws_reserve(ws, ws->pv_pos, sizeof(int64_t) * (n_rows + 1)));
    TPG_TRY(reserve_scan(ws, n_rows));
    TPG_HIP(launch_pv_prime(ws->dg, L, rows->as<int32_t>(), ws->pv_ext.as<uint8_t>(), n_rows,
                            ws->pv_flag.as<int32_t>(), st));
    TPG_HIP(scan_i32_to_i64(ws->pv_flag.as<int32_t>(), ws->pv_pos.as<int64_t>(), n_rows, 0, sc + 1,
                            ws->scan_status.as<uint64_t>(), ws->scan_ctr.as<uint32_t>(), st));
    TPG_HIP(hipMemcpyAsync(ws->h_scalars + 1, sc + 1, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    TPG_HIP(hipStreamSynchronize(st));
    const int64_t np_round = ws->h_scalars[1];
    if (np_round > 0) {
      TPG_TRY(ws_reserve(ws, o.pp_off, sizeof(int64_t) * (n_pp + np_round + 1), true, st,
                         sizeof(int64_t) * n_pp));
      TPG_TRY(ws_reserve(ws, o.pp_vtx, sizeof(int32_t) * (n_vtx + np_round * L + 1), true, st,
                         sizeof(int32_t) * n_vtx));
      TPG_HIP(launch_pv_emit(L, rows->as<int32_t>(), ws->pv_flag.as<int32_t>(),
                             ws->pv_pos.as<int64_t>(), n_rows, n_pp, n_vtx,
                             o.pp_off.as<int64_t>(), o.pp_vtx.as<int32_t>(), st));
      n_pp += np_round;
      n_vtx += np_round * L;
    }
    n_ext += n_next;
    n_rows = n_next;
    std::swap(rows, nrows);
    std::swap(voff, nvoff);
  }
  ws->h_scalars[2] = n_vtx;
  TPG_HIP(hipMemcpyAsync(o.pp_off.as<int64_t>() + n_pp, ws->h_scalars + 2, sizeof(int64_t),
                         hipMemcpyHostToDevice, st));
  // the paper's output: the prime paths ending at each vertex
  TPG_TRY(group_by_last(ws, n, st, o, n_pp, n_vtx));
  if (timing) TPG_HIP(hipEventRecord(e1, st));
  TPG_TRY(deliver_set(ws, o.ppg_off, o.ppg_vtx, n_pp, n_vtx, c.flags, st, out));
  TPG_HIP(hipStreamSynchronize(st));
  if (c.stats) {
    memset(c.stats, 0, sizeof *c.stats);
    c.stats->n_levels = levels;
    c.stats->n_nodes = n + n_ext;
    c.stats->n_extensions = n_ext;
    c.stats->n_pp = n_pp;
    c.stats->n_pp_vertices = n_vtx;
    c.stats->device_bytes = (int64_t)ws->bytes;
    if (timing) c.stats->ms_total = Timer::ms(e0, e1);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  o.n_pp = n_pp;
  o.n_ppv = n_vtx;
  return TPG_OK;
}

tpg_status tpg_test_paths(const tpg_graph* g, const tpg_opts* opts, tpg_paths* pp_out,
                          tpg_paths* tp_out) {
  if (!tp_out) return fail(TPG_ERR_INVALID_ARG, "tp_out is NULL");
  memset(tp_out, 0, sizeof *tp_out);
  if (pp_out) memset(pp_out, 0, sizeof *pp_out);
  TPG_TRY(check_graph(g));
  if (g->load_flags & TPG_LOAD_ANY_DIGRAPH)
    return fail(TPG_ERR_UNREACHABLE, "test paths need a graph loaded with the entry/exit checks");
  CallCtx c;
  TPG_TRY(begin_call(opts, c));
  if ((c.flags & TPG_STREAM) && (!c.opts || !c.opts->on_chunk))
    return fail(TPG_ERR_INVALID_ARG, "TPG_STREAM needs opts.on_chunk");
  HostUnion U;
  add_component(U, g);
  Timer tm{c.ws, c.st, c.stats != nullptr && !(c.flags & TPG_NO_TIMING)};
  const bool timing = tm.on;
  std::vector<hipEvent_t> phase(3, nullptr);
  if (timing) {
    for (auto& e : phase) TPG_HIP(hipEventCreate(&e));
    TPG_HIP(hipEventRecord(phase[0], c.st));
  }
  TreeResult R;
  PPResult P;
  TPResult T;
  hipEvent_t ext_done = nullptr;
  OutSet& o = c.ws->out[0];
  tpg_status s = run_pp(U, c, tm, R, P, o, &ext_done, 0, 0, true);
  if (s == TPG_OK && timing) TPG_HIP(hipEventRecord(phase[1], c.st));
  if (s == TPG_OK) s = test_paths_device(c.ws, U, c.st, P, T, o, c.flags & TPG_TP_GREEDY);
  if (s == TPG_OK && timing) TPG_HIP(hipEventRecord(phase[2], c.st));
  // with TPG_STREAM the sets come back as counts and digests and the test
  // paths go through on_chunk
  const uint32_t fl = (c.flags & TPG_STREAM) ? (c.flags | TPG_DIGEST_ONLY) : c.flags;
  const bool grouped = pp_out && (c.flags & TPG_ORDER_BY_LAST);
  if (s == TPG_OK && grouped) s = group_by_last(c.ws, U.n, c.st, o, P.n_pp, P.n_vtx);
  if (s == TPG_OK && pp_out)
    s = deliver_set(c.ws, grouped ? o.ppg_off : o.pp_off, grouped ? o.ppg_vtx : o.pp_vtx, P.n_pp,
                    P.n_vtx, fl, c.st, pp_out);
  if (s == TPG_OK) s = deliver_set(c.ws, o.tp_off, o.tp_vtx, T.n_tp, T.n_vtx, fl, c.st, tp_out);
  if (s == TPG_OK && (c.flags & TPG_STREAM)) s = test_paths_stream_out(c, o, T.n_tp);
  if (s == TPG_OK) {
    TPG_HIP(hipStreamSynchronize(c.st));
    if (c.stats) {
      memset(c.stats, 0, sizeof *c.stats);
      add_stats(c.stats, U, R, P, &T);
      c.stats->device_bytes = (int64_t)c.ws->bytes;
      if (timing) {
        c.stats->ms_extend = Timer::ms(phase[0], ext_done);
        c.stats->ms_rank = Timer::ms(ext_done, phase[1]);
        c.stats->ms_tp = Timer::ms(phase[1], phase[2]);
        c.stats->ms_total = Timer::ms(phase[0], phase[2]);
      }
    }
  }
  if (s != TPG_OK) {
    if (pp_out) tpg_paths_free(pp_out);
    tpg_paths_free(tp_out);
  }
  for (auto& e : phase)
    if (e) (void)hipEventDestroy(e);
  return s;
}

// ---------------------------------------------------------------------------
// batched form
// ---------------------------------------------------------------------------

// The device work of a batched call (everything between the call's set-up
// and the export of its results): unions by visited-set width, each one's
// prime and test paths, and the packing graph by graph.  pp_first /
// tp_first / ppv / tpv: the packed results' index arrays and sizes.
static tpg_status batch_body(CallCtx& c, const tpg_graph* const* graphs, int32_t n_graphs,
                      const float* predicted, bool want_levels, Timer& tm,
                      std::vector<int64_t>& pp_first, std::vector<int64_t>& tp_first,
                      int64_t& ppv, int64_t& tpv) {
  tpg_workspace* ws = c.ws;
  // unions: one per visited-set width class, split at 2^17 vertices and, with
  // predictions and a pool cap, at half the cap of predicted footprint
  std::vector<std::vector<int32_t>> unions;
  {
    std::vector<std::vector<int32_t>> cls(8);
    for (int32_t i = 0; i < n_graphs; ++i) {
      const int w = pow2_words(graphs[i]->n);
      int k = 0;
      while ((1 << k) < w) ++k;
      cls[k].push_back(i);
    }
    for (int k = 0; k < 8; ++k) {
      std::vector<int32_t> cur;
      int64_t nv = 0;
      double mem = 0;
      for (int32_t i : cls[k]) {
        double gm = 0;
        if (predicted && ws->cap) {
          for (int L = 0; L < 64; ++L) gm += predicted_paths(predicted, i, L);
          gm *= 24.0 + 2.0 * 8.0 * (1 << k);
        }
        if (!cur.empty() && (nv + graphs[i]->n > kMaxUnionVertices ||
                             (ws->cap && mem + gm > 0.5 * (double)ws->cap))) {
          unions.push_back(cur);
          cur.clear();
          nv = 0;
          mem = 0;
        }
        cur.push_back(i);
        nv += graphs[i]->n;
        mem += gm;
      }
      if (!cur.empty()) unions.push_back(cur);
    }
  }
  if (ws->out.size() < unions.size() + 1) ws->out.resize(unions.size() + 1);

  std::vector<int32_t> g_union(n_graphs), g_comp(n_graphs);
  std::vector<std::vector<int64_t>> starts(unions.size());
  for (size_t u = 0; u < unions.size(); ++u) {
    HostUnion U;
    for (size_t k = 0; k < unions[u].size(); ++k) {
      const int32_t i = unions[u][k];
      add_component(U, graphs[i]);
      g_union[i] = (int32_t)u;
      g_comp[i] = (int32_t)k;
    }
    int64_t rec0 = 0, msk0 = 0;
    const bool use_pred =
        predicted &&
        std::find(ws->pred_failed.begin(), ws->pred_failed.end(), U.uids) == ws->pred_failed.end();
    if (use_pred) {
      // capacities from the predicted per-level path counts, 25% margin;
      // index 63 pools every deeper level, so it sizes the total but not the
      // largest single level
      std::vector<double> lv(64, 0.0);
      for (int32_t i : unions[u])
        for (int L = 0; L < 64; ++L) lv[L] += predicted_paths(predicted, i, L);
      double tot = 0, peak = 0;
      for (int L = 0; L < 64; ++L) {
        tot += lv[L];
        if (L < 63) peak = std::max(peak, lv[L]);
      }
      // never more than the record limit, the pool cap or half the free
      // device memory: an over-prediction costs capacity, not the call
      double rec_lim = (double)INT32_MAX - 2, msk_lim = (double)INT32_MAX - 2;
      const double node_b = 13.0, set_b = 2.0 * 8.0 * U.Wu;
      size_t free_b = 0, total_b = 0;
      if (ws->io_mode != 2 && hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0) {
        rec_lim = std::min(rec_lim, 0.5 * (double)free_b / node_b);
        msk_lim = std::min(msk_lim, 0.25 * (double)free_b / set_b);
      } else {
        (void)hipGetLastError();
      }
      if (ws->cap) {
        rec_lim = std::min(rec_lim, 0.5 * (double)ws->cap / node_b);
        msk_lim = std::min(msk_lim, 0.25 * (double)ws->cap / set_b);
      }
      rec0 = (int64_t)std::min(1.25 * tot + U.n + 1024, rec_lim);
      msk0 = (int64_t)std::min(1.25 * peak + 1024, msk_lim);
      io_value(ws, rec0);  // free device memory may differ between calls
      io_value(ws, msk0);
      if (c.stats) {
        c.stats->pred_nodes += (int64_t)std::min(tot, 9.0e18);
        c.stats->pred_peak_level_nodes =
            std::max<int64_t>(c.stats->pred_peak_level_nodes, (int64_t)std::min(peak, 9.0e18));
      }
    }
    OutSet& o = ws->out[u + 1];
    TreeResult R;
    PPResult P;
    TPResult T;
    tpg_status s_pp = run_pp(U, c, tm, R, P, o, nullptr, rec0, msk0, true);
    if (s_pp != TPG_OK && (rec0 || msk0) &&
        (s_pp == TPG_ERR_CAPACITY || s_pp == TPG_ERR_OOM_DEVICE || s_pp == TPG_ERR_UNSUPPORTED)) {
      // the predicted capacities did not fit: size this union exactly, by
      // growth and replay from the smallest buffers, and from what the
      // workspace holds on later calls
      if (ws->pred_failed.size() >= 64) ws->pred_failed.erase(ws->pred_failed.begin());
      ws->pred_failed.push_back(U.uids);
      release_tree(ws);
      R = TreeResult{};
      P = PPResult{};
      s_pp = run_pp(U, c, tm, R, P, o, nullptr, 0, 0, true);
    }
    TPG_TRY(s_pp);
    TPG_TRY(test_paths_device(ws, U, c.st, P, T, o));
    const int nc = U.n_comp;
    if (want_levels) {
      // per-graph path counts of levels 1..64 (deeper levels pooled into 64)
      TPG_TRY(ws_reserve(ws, ws->lvl_comp, sizeof(int64_t) * 64 * (size_t)nc));
      TPG_HIP(launch_zero_u64(ws->lvl_comp.as<uint64_t>(), 64 * (int64_t)nc, c.st));
      ExtArgs a = make_args(ws);
      for (int L = 1; L <= R.Lmax; ++L)
        TPG_HIP(launch_level_comp_counts(a, L, R.off[L], R.count[L], ws->lvl_comp.as<int64_t>(),
                                         c.st));
      std::vector<int64_t> h((size_t)64 * nc);
      TPG_HIP(hipMemcpyAsync(h.data(), ws->lvl_comp.p, sizeof(int64_t) * h.size(),
                             hipMemcpyDeviceToHost, c.st));
      TPG_HIP(hipStreamSynchronize(c.st));
      for (size_t k = 0; k < unions[u].size(); ++k)
        memcpy(c.opts->level_counts + (size_t)64 * unions[u][k], h.data() + 64 * k,
               sizeof(int64_t) * 64);
    }
    // graph-wide ids -> ids of each graph; per-graph output starts
    TPG_HIP(launch_localize(ws->dg.loc, o.pp_vtx.as<int32_t>(), o.n_ppv, c.st));
    TPG_HIP(launch_localize(ws->dg.loc, o.tp_vtx.as<int32_t>(), o.n_tpv, c.st));
    starts[u].assign((size_t)4 * (nc + 1), 0);
    if (nc == 1) {
      starts[u] = {0, o.n_pp, 0, o.n_ppv, 0, o.n_tp, 0, o.n_tpv};
    } else {
      TPG_TRY(io_read(ws, c.st, starts[u].data(), o.comp_starts.p,
                      sizeof(int64_t) * starts[u].size()));
      starts[u][2 * (nc + 1) + nc] = o.n_tp;
      starts[u][3 * (nc + 1) + nc] = o.n_tpv;
    }
    if (c.stats) add_stats(c.stats, U, R, P, &T);
  }

  // pack the unions' outputs graph by graph in caller order: per union and
  // set one launch over its graphs' segments, cut into fixed-size chunks
  const size_t nu = unions.size();
  std::vector<PackDesc> desc(2 * (size_t)n_graphs);
  std::vector<size_t> at(2 * nu + 1, 0);  // descriptors of (union, set) from at[2u + set]
  for (size_t u = 0; u < nu; ++u) {
    at[2 * u + 1] = at[2 * u] + unions[u].size();
    at[2 * u + 2] = at[2 * u + 1] + unions[u].size();
  }
  std::vector<int64_t> n_chunks(2 * nu, 0);
  pp_first.assign(n_graphs + 1, 0);
  tp_first.assign(n_graphs + 1, 0);
  ppv = 0;
  tpv = 0;
  for (int32_t i = 0; i < n_graphs; ++i) {
    const int u = g_union[i];
    const auto& S = starts[u];
    const int nc = (int)unions[u].size();
    const int k = g_comp[i];
    const int64_t p0 = S[k], p1 = S[k + 1], v0 = S[(nc + 1) + k], v1 = S[(nc + 1) + k + 1];
    const int64_t q0 = S[2 * (nc + 1) + k], q1 = S[2 * (nc + 1) + k + 1];
    const int64_t w0 = S[3 * (nc + 1) + k], w1 = S[3 * (nc + 1) + k + 1];
    // graphs of a union are in caller order, so segment k of the union is graph i
    PackDesc& dp = desc[at[2 * u] + k];
    PackDesc& dt = desc[at[2 * u + 1] + k];
    dp = PackDesc{p0, p1 - p0, v0, v1 - v0, pp_first[i], ppv, 0, 0};
    dt = PackDesc{q0, q1 - q0, w0, w1 - w0, tp_first[i], tpv, 0, 0};
    pp_first[i + 1] = pp_first[i] + (p1 - p0);
    tp_first[i + 1] = tp_first[i] + (q1 - q0);
    ppv += v1 - v0;
    tpv += w1 - w0;
  }
  for (size_t r = 0; r < 2 * nu; ++r)
    for (size_t j = at[r]; j < at[r + 1]; ++j) {
      desc[j].chunk0 = n_chunks[r];
      n_chunks[r] += pack_chunks(desc[j]);
    }
  TPG_TRY(ws_reserve(ws, ws->b_pp_off, sizeof(int64_t) * (pp_first[n_graphs] + 1)));
  TPG_TRY(ws_reserve(ws, ws->b_pp_vtx, sizeof(int32_t) * (ppv + 1)));
  TPG_TRY(ws_reserve(ws, ws->b_tp_off, sizeof(int64_t) * (tp_first[n_graphs] + 1)));
  TPG_TRY(ws_reserve(ws, ws->b_tp_vtx, sizeof(int32_t) * (tpv + 1)));
  TPG_TRY(ws_reserve(ws, ws->b_desc, sizeof(PackDesc) * desc.size()));
  PackDesc* dd = ws->b_desc.as<PackDesc>();
  TPG_HIP(hipMemcpyAsync(dd, io_src(ws, desc.data(), sizeof(PackDesc) * desc.size()),
                         sizeof(PackDesc) * desc.size(), hipMemcpyHostToDevice, c.st));
  // an ordinary call waits so the host vector can go (under capture the
  // graph reads its staged copy)
  if (ws->io_mode != 2) TPG_HIP(hipStreamSynchronize(c.st));
  for (size_t u = 0; u < nu; ++u) {
    OutSet& o = ws->out[u + 1];
    const int32_t nd = (int32_t)unions[u].size();
    TPG_HIP(launch_pack(o.pp_off.as<int64_t>(), o.pp_vtx.as<int32_t>(), dd + at[2 * u], nd,
                        n_chunks[2 * u], ws->b_pp_off.as<int64_t>(), ws->b_pp_vtx.as<int32_t>(),
                        c.st));
    TPG_HIP(launch_pack(o.tp_off.as<int64_t>(), o.tp_vtx.as<int32_t>(), dd + at[2 * u + 1], nd,
                        n_chunks[2 * u + 1], ws->b_tp_off.as<int64_t>(),
                        ws->b_tp_vtx.as<int32_t>(), c.st));
  }
  TPG_HIP(launch_set_value_i64(ws->b_pp_off.as<int64_t>() + pp_first[n_graphs], ppv, c.st));
  TPG_HIP(launch_set_value_i64(ws->b_tp_off.as<int64_t>() + tp_first[n_graphs], tpv, c.st));
  return TPG_OK;
}

tpg_status tpg_batch_test_paths(const tpg_graph* const* graphs, int32_t n_graphs,
                                const tpg_opts* opts, const float* predicted,
                                tpg_batch_result* out) {
  if (!out) return fail(TPG_ERR_INVALID_ARG, "out is NULL");
  memset(out, 0, sizeof *out);
  if (!graphs || n_graphs < 1) return fail(TPG_ERR_INVALID_ARG, "no graphs");
  for (int32_t i = 0; i < n_graphs; ++i) {
    TPG_TRY(check_graph(graphs[i]));
    if (graphs[i]->load_flags & TPG_LOAD_ANY_DIGRAPH)
      return fail(TPG_ERR_UNREACHABLE, "graph %d was loaded without the entry/exit checks", i);
  }
  CallCtx c;
  TPG_TRY(begin_call(opts, c));
  tpg_workspace* ws = c.ws;
  const bool want_levels = c.opts && c.opts->level_counts &&
                           (int64_t)c.opts->level_counts_len >= (int64_t)64 * n_graphs;
  Timer tm{ws, c.st, c.stats != nullptr && !(c.flags & TPG_NO_TIMING)};
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (tm.on) {
    TPG_HIP(hipEventCreate(&t0));
    TPG_HIP(hipEventCreate(&t1));
    TPG_HIP(hipEventRecord(t0, c.st));
  }
  if (c.stats) memset(c.stats, 0, sizeof *c.stats);

  std::vector<int64_t> pp_first, tp_first;
  int64_t ppv = 0, tpv = 0;
  // A call that repeats the previous one exactly (same graphs, flags,
  // predictions, stream and launch shapes, and no buffer changed since) runs
  // as one captured HIP graph: the call after a recorded one is captured and
  // from then on replayed with one launch and one wait.  The record holds
  // every value the host read from the device; the graph copies the
  // device's values beside them and a replay whose values differ is
  // discarded and the call run again the ordinary way.
  CallGraph& cg = ws->cg;
  const bool graphable = !tm.on && !want_levels &&
                         !(c.flags & (TPG_FORCE_TWO_PASS | TPG_STREAM | TPG_TP_GREEDY |
                                      TPG_DIGEST | TPG_DIGEST_ONLY | TPG_NO_CALL_GRAPH)) &&
                         c.opts && c.opts->ws;
  std::vector<uint8_t> key;
  if (graphable) {
    key_add(key, n_graphs);
    for (int32_t i = 0; i < n_graphs; ++i) key_add(key, graphs[i]->uid);
    key_add(key, c.flags);
    key_add(key, c.st);
    key_add(key, ws->cap);
    key_add(key, predicted != nullptr);
    if (predicted) {
      const uint8_t* pb = reinterpret_cast<const uint8_t*>(predicted);
      key.insert(key.end(), pb, pb + sizeof(float) * 65 * (size_t)n_graphs);
    }
    for (int k = 0; k < 7; ++k) {
      key_add(key, ws->tune_items[k]);
      key_add(key, ws->tune_wgs[k]);
      key_add(key, ws->tune_variant[k]);
    }
  }
  const bool same = graphable && cg.recorded && cg.key == key && cg.gen == ws->alloc_gen;
  int32_t graph_state = 0;  // 0 ordinary, 1 captured by this call, 2 replayed
  bool done = false;
  if (same && !cg.failed) {
    if (!cg.exec) {
      // capture the call into one graph
      ws->io_mode = 2;
      ws->io_rec = &cg.vals;
      ws->io_pos = 0;
      ws->io_check_used = 0;
      ws->io_stage_used = 0;
      ws->io_diverged = false;
      hipGraph_t graph = nullptr;
      tpg_status bs = TPG_OK;
      if (hipStreamBeginCapture(c.st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        std::vector<int64_t> pf, tf;
        int64_t a = 0, b = 0;
        tpg_stats saved{};
        if (c.stats) saved = *c.stats;
        bs = batch_body(c, graphs, n_graphs, predicted, want_levels, tm, pf, tf, a, b);
        if (c.stats) *c.stats = saved;
        const hipError_t ee = hipStreamEndCapture(c.st, &graph);
        hipError_t ei = hipSuccess;
        if (bs == TPG_OK && ee == hipSuccess && !ws->io_diverged && ws->io_pos == cg.vals.size() &&
            graph && (ei = hipGraphInstantiate(&cg.exec, graph, nullptr, nullptr, 0)) == hipSuccess) {
          graph_state = 1;
        } else {
          // the reason stays in the error text; the call runs the ordinary way
          if (bs == TPG_OK)
            (void)fail(TPG_ERR_UNSUPPORTED,
                       "call graph not used: end of capture %s, instantiation %s, %s, %zu of %zu "
                       "recorded values read",
                       hipGetErrorString(ee), hipGetErrorString(ei),
                       ws->io_diverged ? "diverged" : "on the recorded path", ws->io_pos,
                       cg.vals.size());
          cg.exec = nullptr;
          cg.failed = true;
        }
      } else {
        (void)fail(TPG_ERR_UNSUPPORTED, "call graph not used: the stream could not be captured");
        (void)hipGetLastError();
        cg.failed = true;
      }
      if (graph) (void)hipGraphDestroy(graph);
      ws->io_mode = 0;
      ws->io_rec = nullptr;
      (void)hipGetLastError();
    }
    if (cg.exec) {
      TPG_HIP(hipGraphLaunch(cg.exec, c.st));
      TPG_HIP(hipStreamSynchronize(c.st));
      if (ws->io_check_used == cg.vals.size() &&
          memcmp(ws->io_check, cg.vals.data(), cg.vals.size()) == 0) {
        pp_first = cg.pp_first;
        tp_first = cg.tp_first;
        ppv = cg.ppv;
        tpv = cg.tpv;
        if (c.stats) *c.stats = cg.stats;
        if (graph_state == 0) graph_state = 2;
        done = true;
      } else {
        // the device took another path than the recorded call: run it again
        (void)hipGraphExecDestroy(cg.exec);
        cg.exec = nullptr;
        cg.recorded = false;
        if (c.stats) memset(c.stats, 0, sizeof *c.stats);
        graph_state = 0;
      }
    }
  }
  if (!done) {
    // an ordinary call, recorded when it may be captured next time
    if (cg.exec && !same) {
      (void)hipGraphExecDestroy(cg.exec);
      cg.exec = nullptr;
    }
    ws->io_mode = graphable ? 1 : 0;
    ws->io_vals.clear();
    ws->io_stage_used = 0;
    const uint64_t gen0 = ws->alloc_gen;
    const tpg_status bs = batch_body(c, graphs, n_graphs, predicted, want_levels, tm, pp_first,
                                     tp_first, ppv, tpv);
    ws->io_mode = 0;
    TPG_TRY(bs);
    if (c.stats) c.stats->n_allocs = (int64_t)(ws->alloc_gen - gen0);
    if (same && cg.failed) graph_state = 3;
    if (graphable) {
      // worth recording only when nothing grew: a replay must not allocate
      const bool stable = ws->alloc_gen == gen0;
      const bool new_key = !(cg.key == key);
      cg.key = key;
      cg.recorded = stable;
      if (new_key) cg.failed = false;
      cg.vals.swap(ws->io_vals);
      cg.stage_bytes = ws->io_stage_used;
      cg.gen = ws->alloc_gen;
      cg.pp_first = pp_first;
      cg.tp_first = tp_first;
      cg.ppv = ppv;
      cg.tpv = tpv;
      if (c.stats) cg.stats = *c.stats;
      // pinned room for the next call's capture (allocated now, outside it)
      if (stable && cg.vals.size() > ws->io_check_cap) {
        if (ws->io_check) (void)hipHostFree(ws->io_check);
        ws->io_check = nullptr;
        ws->io_check_cap = 0;
        TPG_HIP(hipHostMalloc((void**)&ws->io_check, cg.vals.size() + 64));
        ws->io_check_cap = cg.vals.size() + 64;
      }
      if (stable && cg.stage_bytes > ws->io_stage_cap) {
        if (ws->io_stage) (void)hipHostFree(ws->io_stage);
        ws->io_stage = nullptr;
        ws->io_stage_cap = 0;
        TPG_HIP(hipHostMalloc((void**)&ws->io_stage, cg.stage_bytes + 256));
        ws->io_stage_cap = cg.stage_bytes + 256;
      }
    }
  }
  if (c.stats) c.stats->call_graph = graph_state;
  const bool dev = c.flags & TPG_OUT_DEVICE;
  if (tm.on) TPG_HIP(hipEventRecord(t1, c.st));

  tpg_status s = export_paths(ws->b_pp_off, ws->b_pp_vtx, pp_first[n_graphs], ppv, dev, c.st, &out->pp);
  if (s == TPG_OK)
    s = export_paths(ws->b_tp_off, ws->b_tp_vtx, tp_first[n_graphs], tpv, dev, c.st, &out->tp);
  if (s == TPG_OK) {
    out->n_graphs = n_graphs;
    out->pp_first = (int64_t*)malloc(sizeof(int64_t) * (n_graphs + 1));
    out->tp_first = (int64_t*)malloc(sizeof(int64_t) * (n_graphs + 1));
    if (!out->pp_first || !out->tp_first) {
      s = fail(TPG_ERR_OOM_HOST, "batch index arrays");
    } else {
      memcpy(out->pp_first, pp_first.data(), sizeof(int64_t) * (n_graphs + 1));
      memcpy(out->tp_first, tp_first.data(), sizeof(int64_t) * (n_graphs + 1));
    }
  }
  if (s == TPG_OK) {
    TPG_HIP(hipStreamSynchronize(c.st));
    if (c.stats) {
      c.stats->device_bytes = (int64_t)ws->bytes;
      if (tm.on) c.stats->ms_total = Timer::ms(t0, t1);
    }
  } else {
    tpg_batch_result_free(out);
  }
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  return s;
}

tpg_status tpg_workspace_set_tuning(tpg_workspace* ws, const tpg_tuning* t) {
  if (!ws || !t) return fail(TPG_ERR_INVALID_ARG, "NULL argument");
  for (int i = 0; i < 7; ++i) {
    const int it = t->items[i], wg = t->wgs_per_cu[i];
    const int va = t->variant[i];
    if ((it != 1 && it != 2 && it != 4 && it != 8) || wg < 1 || wg > 32 || va < 0 || va > 2)
      return fail(TPG_ERR_INVALID_ARG, "tuning entry %d: items %d, workgroups per CU %d, variant %d",
                  i, it, wg, va);
  }
  for (int i = 0; i < 7; ++i) {
    ws->tune_items[i] = t->items[i];
    ws->tune_wgs[i] = t->wgs_per_cu[i];
    ws->tune_variant[i] = t->variant[i];
    ws->tune_ms[i] = t->best_ms[i];
  }
  return TPG_OK;
}

tpg_status tpg_workspace_get_tuning(const tpg_workspace* ws, tpg_tuning* t) {
  if (!ws || !t) return fail(TPG_ERR_INVALID_ARG, "NULL argument");
  for (int i = 0; i < 7; ++i) {
    t->items[i] = ws->tune_items[i];
    t->wgs_per_cu[i] = ws->tune_wgs[i];
    t->variant[i] = ws->tune_variant[i];
    t->best_ms[i] = ws->tune_ms[i];
  }
  return TPG_OK;
}

tpg_status tpg_autotune(const tpg_graph* const* graphs, int32_t n_graphs, const tpg_opts* opts,
                        tpg_tuning* out) {
  if (!graphs || n_graphs < 1 || !out) return fail(TPG_ERR_INVALID_ARG, "bad argument");
  for (int32_t i = 0; i < n_graphs; ++i) TPG_TRY(check_graph(graphs[i]));
  CallCtx c;
  TPG_TRY(begin_call(opts, c));
  tpg_workspace* ws = c.ws;
  // one union per visited-set width (first 2^17 vertices of each width)
  std::vector<HostUnion> unions(7);
  for (int32_t i = 0; i < n_graphs; ++i) {
    const int w = pow2_words(graphs[i]->n);
    int k = 0;
    while ((1 << k) < w) ++k;
    if (unions[k].n + graphs[i]->n <= kMaxUnionVertices) add_component(unions[k], graphs[i]);
  }
  const int items_c[4] = {1, 2, 4, 8};
  const int wgs_c[4] = {1, 2, 4, 8};
  Timer tm{ws, c.st, true};
  for (int k = 0; k < 7; ++k) {
    const HostUnion& U = unions[k];
    if (U.n_comp == 0) continue;
    TPG_TRY(upload_union(ws, U, c.st));
    TreeResult warm;
    TPG_TRY(build_tree_onepass(ws, U, c.st, tm, warm, 0, 0));
    double best = 1e30;
    int bi = ws->tune_items[k], bw = ws->tune_wgs[k], bv = ws->tune_variant[k];
    for (int va = 0; va < 3; ++va)
    for (int it : items_c)
      for (int wg : wgs_c) {
        if (va == 2 && wg > 2) continue;  // 1024-thread workgroups: at most 2 per CU
        if (va != 0 && it * (1 << k) > 32) continue;  // register-resident visited sets
        ws->tune_items[k] = it;
        ws->tune_wgs[k] = wg;
        ws->tune_variant[k] = va;
        double t_min = 1e30;
        for (int rep = 0; rep < 2; ++rep) {
          TreeResult R;
          TPG_TRY(build_tree_onepass(ws, U, c.st, tm, R, 0, 0));
          t_min = std::min(t_min, R.ms_kernel);
        }
        if (t_min < best) {
          best = t_min;
          bi = it;
          bw = wg;
          bv = va;
        }
      }
    ws->tune_items[k] = bi;
    ws->tune_wgs[k] = bw;
    ws->tune_variant[k] = bv;
    ws->tune_ms[k] = best;
  }
  return tpg_workspace_get_tuning(ws, out);
}

void tpg_batch_result_free(tpg_batch_result* r) {
  if (!r) return;
  tpg_paths_free(&r->pp);
  tpg_paths_free(&r->tp);
  free(r->pp_first);
  free(r->tp_first);
  memset(r, 0, sizeof *r);
}

}  // extern "C"
