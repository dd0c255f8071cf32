// Host-visible declarations of the device structures and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"

namespace tpg {

constexpr int kMaxLevels = 4096 + 4;  // path entries <= n + 1

// Level bookkeeping kept in device memory so that levels can follow each
// other without the host learning their sizes.  The 32-byte header is what
// the host polls.
struct LevelState {
  int32_t batch_start;     // level extended by launch 0 of the running batch
  int32_t overflow;        // non-zero: the children of overflow_level did not fit
  int32_t overflow_level;
  int32_t pad;
  int64_t pad2[2];
  // nodes (paths) per level, cycle closures included; while level L is
  // extended, count[L + 1] is the running claim counter of its tiles
  int64_t count[kMaxLevels];
  int64_t off[kMaxLevels];    // global index of the first node of each level
};

// Buffers of the path tree and of the frontier.
struct TreeBufs {
  int32_t* par;       // [rec_cap]
  uint32_t* info;     // [rec_cap]
  int32_t* cstart;    // [rec_cap + 1] global index of the first child
  uint8_t* nch;       // [rec_cap] number of children (<= 64) or leaf kind (nch_code)
  uint64_t* mask[2];  // visited sets of the odd levels, alternating [mask_cap * mask_words]
  int64_t rec_cap;
  int64_t mask_cap;
  int32_t mask_words;  // words stored per visited set (<= the kernel width W)
  int32_t pad;
};

struct ExtArgs {
  DGraph g;
  TreeBufs t;
  LevelState* ls;
  int64_t tiles_target;  // one-pass tiles per level aimed at (tile size grows above it)
  // level 1: paths <v> for the first vertices v = seed_lo .. seed_lo + seed_n - 1
  // (node k holds vertex seed_lo + k; all vertices unless a call streams by
  // first-vertex range)
  int32_t seed_lo, seed_n;
};

// --- path tree -------------------------------------------------------------
hipError_t launch_seed(const ExtArgs& a, hipStream_t st);
// items: most parents per thread (tile <= threads * items); variant: 0
// load-balanced tiles of 256 threads, 1 / 2 thread-per-parent with 256 /
// 1024 threads; grid: persistent workgroups; li: index of the launch in its
// batch (it extends level batch_start + li)
// e0 / e1 (optional): events recorded at the kernel's own start and end
hipError_t launch_extend(int W, int items, int variant, const ExtArgs& a, int grid, int li,
                         hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_resume_fix(const ExtArgs& a, int level, hipStream_t st);
// two-pass (plain) form
// prev: first node of level L - 1 (an even level's visited sets are rebuilt
// from its parents' stored sets)
hipError_t launch_count(int W, const ExtArgs& a, int L, int64_t prev, int64_t base, int64_t F,
                        hipStream_t st);
hipError_t launch_fill(int W, const ExtArgs& a, int L, int64_t prev, int64_t base, int64_t F,
                       hipStream_t st);

// --- ranking / materialization ---------------------------------------------
// sub_cnt: PP leaves per subtree (k_up), then rewritten top-down into the
// rank of the subtree's first PP (or 0xFFFFFFFF when it has none).
// n_cycles: kCycleSlots counters, zeroed before the sweep; a workgroup adds
// its closed cycles to slot blockIdx.x % kCycleSlots (one address for all
// would serialize the adds of a large level)
constexpr int kCycleSlots = 64;
hipError_t launch_up(const ExtArgs& a, int L, int64_t base, int64_t F, uint32_t* sub_cnt,
                     unsigned long long* n_cycles, hipStream_t st);
// mode 0: totals[0] = #PP (no change to the arrays) and, with n_cycles given,
// n_cycles[kCycleSlots] = the sum of its slots; mode 1: level-1 ranks, root
// leaves recorded (leaf_by_rank, pp_len = 1), and with rb given (roots =
// every vertex, in id order) rb[v] = rank of the first prime path whose
// first vertex is >= v (v = 0 .. n_roots).
hipError_t launch_roots(const ExtArgs& a, int64_t n_roots, uint32_t* sub_cnt, int64_t* leaf_by_rank,
                        int32_t* pp_len, int64_t* totals, int mode, int64_t* rb,
                        unsigned long long* n_cycles, hipStream_t st);
// parents of level L: ranks to the children; PP leaves record node and length
hipError_t launch_down(const ExtArgs& a, int L, int64_t base, int64_t F, uint32_t* sub_cnt,
                       int64_t* leaf_by_rank, int32_t* pp_len, hipStream_t st);
// the same for depth + 1 levels in one launch (depth 1 or 2; base, F: the
// run's top level L): counts of levels L .. L + depth, and ranks handed down
// by the parents of levels L .. L + depth
hipError_t launch_up_run(const ExtArgs& a, int depth, int64_t base, int64_t F, uint32_t* sub_cnt,
                         unsigned long long* n_cycles, hipStream_t st);
hipError_t launch_down_run(const ExtArgs& a, int depth, int L, int64_t base, int64_t F,
                           uint32_t* sub_cnt, int64_t* leaf_by_rank, int32_t* pp_len,
                           hipStream_t st);
// What the prime-path writer also records for the test paths when the BFS
// tables are ready (tp_len null: nothing): per prime path i, the length of
// its test path, and lead[i] = the first index t >= 1 whose entry's BFS
// parent is not entry t - 1 (the path's length when there is none).
struct PPWriteTp {
  const int32_t* parent;   // BFS parent of each vertex
  const int64_t* pfx_off;  // prefix / suffix table offsets (their lengths)
  const int64_t* sfx_off;
  int64_t* tp_len;
  // per prime path: (lead, w, e, v1): the first entry index t >= 1 whose BFS
  // parent is not entry t - 1 (the length if none), the entries w at lead - 1
  // and e at lead (-1 if none), and the first vertex
  int4* lead;
};
hipError_t launch_pp_write(const ExtArgs& a, const int64_t* leaf_by_rank, const int64_t* pp_off,
                           int64_t n_pp, int32_t* pp_vtx, const PPWriteTp& tp, hipStream_t st);

// --- scans -------------------------------------------------------------------
// out[i] = add + sum(in[0..i)), *total = add + sum(in); n may be 0.
hipError_t scan_i32_to_i32(const int32_t* in, int32_t* out, int64_t n, int64_t add,
                           int64_t* total, uint64_t* status, uint32_t* ctr, hipStream_t st);
hipError_t scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, int64_t add,
                           int64_t* total, uint64_t* status, uint32_t* ctr, hipStream_t st);
hipError_t scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t add, int64_t* total,
                    uint64_t* status, uint32_t* ctr, hipStream_t st);
int64_t scan_tiles(int64_t n);  // status slots needed by the scans for n items

hipError_t launch_zero_u64(uint64_t* p, int64_t n, hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);

// --- strongly connected components and prime-path types (Sec. 2) ----------
// per-vertex flags (Defs. 4-5) and path types (Defs. 2, 9, 10, 11); the values
// are the ones the C API exports
constexpr uint8_t kSccCyclic = 1, kSccEntryVertex = 2, kSccExitVertex = 4;
constexpr uint8_t kPpComplete = 1, kPpSccInternal = 2, kPpSccExit = 3, kPpSccEntry = 4,
                  kPpOther = 5;
constexpr int kPpTypes = 6;  // counts are indexed by type (index 0 unused)
// comp[v] = smallest vertex of v's component, flags[v], n_comp[0] = number of
// components; m: arcs of the union; work: 6 n int32 of scratch
hipError_t launch_scc(const DGraph& g, int32_t m, int32_t* work, int32_t* comp, uint8_t* flags,
                      int32_t* n_comp, hipStream_t st);
// --- the paper's per-vertex schedule (comparison variant) ------------------
hipError_t launch_pv_init(int n, int64_t* voff, int32_t* rows, hipStream_t st);
hipError_t launch_pv_count(const DGraph& g, int L, const int64_t* voff, const int32_t* rows,
                           int32_t* cnt, hipStream_t st);
hipError_t launch_pv_fill(const DGraph& g, int L, const int64_t* voff, const int32_t* rows,
                          uint8_t* extended, const int64_t* nvoff, int32_t* nrows,
                          hipStream_t st);
hipError_t launch_pv_prime(const DGraph& g, int L, const int32_t* rows, const uint8_t* extended,
                           int64_t n_rows, int32_t* flag, hipStream_t st);
hipError_t launch_pv_emit(int L, const int32_t* rows, const int32_t* flag, const int64_t* pos,
                          int64_t n_rows, int64_t base, int64_t voff0, int64_t* out_off,
                          int32_t* out_vtx, hipStream_t st);
// types[i] (may be null) and counts[0 .. kPpTypes) of a prime-path set
// --- compositional method (Sec. 2.1): component graph, extraction, merge ---
hipError_t launch_ccfg_count(const DGraph& g, const int32_t* comp, int32_t* cnt, hipStream_t st);
hipError_t launch_ccfg_write(const DGraph& g, const int32_t* comp, const int64_t* off, int32_t* src,
                             int32_t* dst, hipStream_t st);
// mode 0: forward tree of the components (set 0 entry-exit paths, set 1 entry
// paths); mode 1: tree of the reversed components (set 0 exit paths)
hipError_t launch_ex_up(const ExtArgs& a, int64_t base, int64_t F, const uint8_t* vfl, int mode,
                        uint8_t* qb, uint32_t* cnt0, uint32_t* cnt1, hipStream_t st);
hipError_t launch_ex_roots(uint32_t* cnt, int64_t n_roots, int64_t* total, hipStream_t st);
hipError_t launch_ex_down(const ExtArgs& a, int L, int64_t base, int64_t F, const uint8_t* qb,
                          uint32_t* cnt, int mode, int set, int64_t* out_node, int32_t* out_len,
                          hipStream_t st);
hipError_t launch_ex_write(const ExtArgs& a, const int64_t* out_node, const int64_t* off,
                           int64_t n, int reversed, const int32_t* orig, int32_t* vtx,
                           hipStream_t st);
hipError_t launch_merge_class(const int64_t* off, const int32_t* vtx, int64_t n,
                              const uint8_t* hkind, const int32_t* horig, const DGraph& g,
                              int h_entry, int h_exit, uint8_t* cls, int32_t* len, hipStream_t st);
hipError_t launch_internal_class(const int64_t* off, const int32_t* vtx, int64_t n,
                                 const uint8_t* vfl, uint8_t* cls, int32_t* len, hipStream_t st);
hipError_t launch_merge_sel(const uint8_t* cls, const int32_t* len, int64_t n, int c, int32_t* flag,
                            int32_t* lens, hipStream_t st);
hipError_t launch_merge_emit(const int64_t* off, const int32_t* vtx, int64_t n, const uint8_t* cls,
                             int c, const int64_t* pos, const int64_t* voff, const int32_t* len,
                             const int32_t* horig, int64_t* out_off, int32_t* out_vtx,
                             hipStream_t st);
hipError_t launch_pp_types(const DGraph& g, const int32_t* comp, const uint8_t* flags,
                           const int64_t* off, const int32_t* vtx, int64_t n_pp, uint8_t* types,
                           unsigned long long* counts, hipStream_t st);
// --- stable counting sorts by a small integer key (tiles of kGroupTile) -------
constexpr int kGroupTile = 1024;
// --- prime paths grouped by last vertex (stable counting sort) ---------------
// key[i] = last vertex of path i; hist[key * ntiles + tile] counts (hist must
// be zero, nkeys * ntiles entries, tile = group_tiles granularity)
int64_t group_tiles(int64_t n);
hipError_t launch_last_hist(const int64_t* off, const int32_t* vtx, int64_t n, int64_t ntiles,
                            int32_t* key, uint64_t* hist, hipStream_t st);
// perm[slot] = path index, slot = base[key * ntiles + tile] + rank among the
// tile's earlier paths with the same key (base: exclusive scan of hist)
hipError_t launch_last_place(const int32_t* key, int64_t n, int64_t ntiles, const int64_t* base,
                             int32_t* perm, hipStream_t st);
// len[k] = length of path perm[k], pos[k] = k (the gather's inputs)
hipError_t launch_perm_lens(const int64_t* off, const int32_t* perm, int64_t n, int64_t* len,
                            int64_t* pos, hipStream_t st);

// --- test paths by longest-first covering (kernels_cover.hip) ----------------
// Hash table of the prime paths (keys / vals of mask + 1 slots, keys zeroed);
// dups counts hashes shared by two prime paths (then retry with another mul).
uint64_t cover_hash_mul(int attempt);
hipError_t launch_pp_hash_insert(const int64_t* off, const int32_t* vtx, int64_t n, uint64_t mul,
                                 uint64_t* keys, int32_t* vals, int64_t mask, uint64_t* dups,
                                 hipStream_t st);
// Prime paths contained in each spliced test path p: pass 0 writes cnt[p],
// pass 1 the pairs (p, q) at at[p] (exclusive scan of cnt); missing counts
// accepted windows absent from the table (never, unless the input is bad).
hipError_t launch_cover(int W, const DGraph& g, const int64_t* tp_off, const int32_t* tp_vtx,
                        int64_t n, uint64_t mul, const uint64_t* keys, const int32_t* vals,
                        int64_t mask, int64_t* cnt, const int64_t* at, int32_t* pair_p,
                        int32_t* pair_q, int pass, uint64_t* missing, hipStream_t st);
// key[i] = max_len - length of path i (decreasing length first)
hipError_t launch_len_key(const int64_t* off, int64_t n, int64_t max_len, int32_t* key,
                          hipStream_t st);
hipError_t launch_key_hist(const int32_t* key, int64_t n, int64_t ntiles, uint64_t* hist,
                           hipStream_t st);
hipError_t launch_invert(const int32_t* perm, int64_t n, int32_t* pos, hipStream_t st);
// A round of the covering decision: pass over the pairs (drop / block
// flags, state read only), then decide every undecided path (state 0 ->
// 1 chosen, 2 dropped) and count the ones left (undecided must be zeroed).
hipError_t launch_round_pairs(const int32_t* pair_p, const int32_t* pair_q, int64_t np,
                              const int32_t* pos, const uint8_t* state, uint8_t* drop,
                              uint8_t* block, hipStream_t st);
hipError_t launch_round_decide(int64_t n, uint8_t* state, uint8_t* drop, uint8_t* block,
                               uint64_t* undecided, hipStream_t st);
hipError_t launch_chosen_flags(const uint8_t* state, int64_t n, int32_t* flag, hipStream_t st);
// list[at[q]] = q for the chosen paths; then their runs by first vertex
hipError_t launch_chosen_list(const uint8_t* state, const int64_t* at, int64_t n, int32_t* list,
                              hipStream_t st);
hipError_t launch_chosen_runs(const int32_t* list, int64_t m, const int64_t* pp_off,
                              const int32_t* pp_vtx, int nv, int64_t* rb, hipStream_t st);
// Set digest of paths [0, n) (offsets off, entries vtx): out[0] = sum and
// out[1] = xor of the per-path FNV-1a 64 hashes of (k, v_1 .. v_k) as int32
// little-endian bytes; out is cleared first.
hipError_t launch_digest(const int64_t* off, const int32_t* vtx, int64_t n, uint64_t* out,
                         hipStream_t st);
hipError_t launch_zero_u32(uint32_t* p, int64_t n, hipStream_t st);

// --- test paths --------------------------------------------------------------
struct BfsOut {
  int32_t* dist_f;   // [n] arcs from entry
  int32_t* parent;   // [n] lexicographically smallest shortest-path parent
  int32_t* dist_b;   // [n] arcs to exit
  int32_t* next;     // [n] first step of the smallest shortest path to exit
  int64_t* pfx_off;  // [n+1] prefix table offsets (entries before v)
  int32_t* pfx;      // [pfx_off[n]]
  int64_t* sfx_off;  // [n+1] suffix table offsets (entries after v)
  int32_t* sfx;      // [sfx_off[n]]
  int32_t* pre;      // [n] graph-wide preorder rank in the BFS tree (children ascending)
  int32_t* pend;     // [n] end of v's subtree rank range
  int32_t* cfirst;   // [n] v's tree children: bq[cfirst[v] .. cfirst[v] + ccnt[v]), ascending
  int32_t* ccnt;     // [n]
  int32_t* bq;       // [n] the search queue (graph-wide ids)
  uint64_t* pfx_pk;  // prefix rows packed like the test paths (see k_pack_tables)
  uint64_t* sfx_pk;  // suffix rows packed likewise
};
// What the test-path comparison reads: per test path kTpKeyWords 64-bit keys
// (see k_tp_keys: two words of tree position, then kTpKeyTail words of the
// entries after the tree prefix) and, for the ties the keys leave, the
// packed entries.
constexpr int kTpKeyTail = 4;
constexpr int kTpKeyWords = 2 + kTpKeyTail;
struct TpOrder {
  const int64_t* off;   // [n + 1] test-path offsets
  const uint64_t* key;  // [kTpKeyWords n], 16-byte aligned
  const uint64_t* pk;   // the entries packed (see k_tp_write)
  int eb;               // bits per packed entry (entry + 1; 0 = past the end)
  int pe;               // packed entries per 64-bit word, 64 / eb
};
// one workgroup per component: dist_f, parent, pre, pend, tree children, dist_b, next
hipError_t launch_bfs_dist(const DGraph& g, const BfsOut& b, hipStream_t st);
// after pfx_off / sfx_off are scans of dist_f / dist_b: fill pfx / sfx
hipError_t launch_bfs_tables(const DGraph& g, const BfsOut& b, hipStream_t st);
hipError_t launch_localize(const int32_t* loc, int32_t* v, int64_t n, hipStream_t st);
// per-component output starts: pp_start[c] = rank of the first PP of c and
// ppv_start[c] = offset of its first entry (after the PP offsets exist)
hipError_t launch_comp_pp_starts(const DGraph& g, const uint32_t* sub_cnt, const int64_t* pp_off,
                                 const int64_t* totals, int64_t* pp_start, int64_t* ppv_start,
                                 hipStream_t st);

// test-path lengths, and rb[v] = first prime path with first vertex >= v
// (v = 0..n); either output may be null (not computed)
hipError_t launch_tp_len(const int64_t* pp_off, const int32_t* pp_vtx, int64_t n_pp, int n,
                         const BfsOut& b, int64_t* tp_len, int64_t* rb, hipStream_t st);
// writes the test paths packed (pk: (n_entries + pe - 1) / pe + 2 n_pp + 4
// words, pe = 64 / eb), their comparison keys, idx[i] = i and, when tp_vtx
// is not null, their plain entries
// Packed prefix / suffix rows of every vertex (after the tables exist).
hipError_t launch_pack_tables(int n, const BfsOut& b, int eb, hipStream_t st);
// lead: what the prime-path writer recorded (null: found here by a scan)
hipError_t launch_tp_write(const int64_t* pp_off, const int32_t* pp_vtx, int64_t n_pp,
                           const BfsOut& b, const int64_t* tp_off, int32_t* tp_vtx,
                           uint64_t* key, uint64_t* pk, int eb, int32_t* idx,
                           const int4* lead, hipStream_t st);
// one round of pairwise merging of sorted runs [rb[r], rb[r+1]) of idx;
// split: device scratch of merge_split_slots(n) int64 (the tiles' splits and pairs)
hipError_t launch_merge_round(const TpOrder& K, const int32_t* idx_in, int32_t* idx_out,
                              const int64_t* rb, int64_t n_runs, int64_t n, int64_t* split,
                              hipStream_t st);
int64_t merge_split_slots(int64_t n);
hipError_t launch_next_runs(const int64_t* rb, int64_t n_runs, int64_t* rb_out, hipStream_t st);
// the per-vertex runs rb[0..n] of a union, each graph's padded to 2^R runs:
// out[0..n_out], n_out = n_comp * 2^R
hipError_t launch_pad_runs(const DGraph& g, const int64_t* rb, int R, int64_t n_out, int64_t* out,
                           hipStream_t st);
hipError_t launch_dedup_flags(const TpOrder& K, const int32_t* idx, int64_t n, int64_t* keep_cnt,
                              int64_t* keep_len, hipStream_t st);
// copies the kept paths (keep_len[k] > 0) of idx to out_off / out_vtx
hipError_t launch_gather(const int64_t* tp_off, const int32_t* tp_vtx, const int32_t* idx,
                         int64_t n, const int64_t* keep_pos, const int64_t* keep_voff,
                         const int64_t* keep_len, int64_t* out_off, int32_t* out_vtx,
                         hipStream_t st);
// the same for test paths held packed (tp_off: their entry offsets, pk: the
// words k_tp_write built with eb bits per entry; the words that hold only
// prefix entries come from the packed prefix rows in b, test path a having
// been spliced from prime path a of pp_off / pp_vtx)
hipError_t launch_unpack_gather(const int64_t* tp_off, const uint64_t* pk, const int64_t* pp_off,
                                const int32_t* pp_vtx, const BfsOut& b, int eb,
                                const int32_t* idx, int64_t n, const int64_t* keep_pos,
                                const int64_t* keep_voff, const int64_t* keep_len,
                                int64_t* out_off, int32_t* out_vtx, hipStream_t st);
// start[c] / vstart[c] (c = 0..n_comp) of a sorted path list; off[n] = total
hipError_t launch_comp_bounds(const int64_t* off, const int32_t* vtx, int64_t n,
                              const int32_t* comp, int n_comp, int64_t* start, int64_t* vstart,
                              hipStream_t st);
hipError_t launch_set_i64(int64_t* p, const int64_t* src, hipStream_t st);
hipError_t launch_set_value_i64(int64_t* p, int64_t value, hipStream_t st);

// --- batched form --------------------------------------------------------------
// One graph's segment of a union's output, where it goes in the packed
// output (caller order), and the first of its copy chunks in the launch
// (its offsets in chunks of kPackPaths, then its entries in chunks of
// kPackVtx).
constexpr int kPackPaths = 1024;
constexpr int kPackVtx = 4096;
struct PackDesc {
  int64_t src_path, n_paths, src_v0, n_v;
  int64_t dst_path, dst_v;
  int64_t chunk0;
  int64_t pad;
};
inline int64_t pack_chunks(const PackDesc& e) {
  return (e.n_paths + kPackPaths - 1) / kPackPaths + (e.n_v + kPackVtx - 1) / kPackVtx;
}
// copies the segments d[0 .. n_desc) of one union (chunk0 ascending from 0;
// n_chunks in all): one workgroup per chunk
hipError_t launch_pack(const int64_t* src_off, const int32_t* src_vtx, const PackDesc* d,
                       int32_t n_desc, int64_t n_chunks, int64_t* dst_off, int32_t* dst_vtx,
                       hipStream_t st);
// lvl_comp[c * 64 + min(L, 64) - 1] += paths of level L in component c
hipError_t launch_level_comp_counts(const ExtArgs& a, int L, int64_t base, int64_t F,
                                    int64_t* lvl_comp, hipStream_t st);

}  // namespace tpg
