/* tpg.h - prime-path and test-path generation on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libtpg.so.  Plain pointers and sizes only.
 *
 * Problem (the paper's Problem 1, Sec. 3): given a control-flow graph
 * G = (V, E) with a start vertex s and an end vertex e, produce every prime
 * path of G and a set of test paths that covers every prime path.
 *
 *  - A simple path is a vertex sequence v1..vk (k > 0) along arcs in which no
 *    vertex repeats, except that v1 = vk is allowed (Sec. 2).
 *  - A prime path (PP) is a simple path that is not a proper contiguous
 *    subpath of any other simple path (Def. 1).
 *  - A test path (TP) runs from the entry to the exit and contains a prime
 *    path; here TP(p) = (lexicographically smallest shortest entry->v1 path,
 *    without v1) ++ p ++ (lexicographically smallest shortest vk->exit path,
 *    without vk)  (Sec. 7.3: every prime path is extended to the initial and
 *    final nodes).  Duplicate TPs are removed.
 *  - Every returned path set is in canonical order: lexicographic on the
 *    int32 vertex ids.  Path sets are returned as CSR-like arrays:
 *    offsets[n_paths + 1] (int64, offsets[0] = 0) into vertices[] (int32).
 *
 * Error behaviour: every function returns a tpg_status; on failure outputs
 * are left empty (pointers NULL, counts 0) and nothing needs freeing.  A
 * human-readable message for the last failure on the calling thread is
 * available from tpg_last_error().
 *
 * Threading: a tpg_graph is immutable after loading and may be shared by
 * threads.  A tpg_workspace serializes nothing by itself: use one workspace
 * per concurrent caller (or per stream).
 */
#ifndef TPG_H_
#define TPG_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TPG_VERSION_MAJOR 0
#define TPG_VERSION_MINOR 1

/* Largest vertex count the engine accepts (visited sets are bitmasks of up
 * to 64 64-bit words) and largest out-degree (successor choice masks are one
 * 64-bit word). */
#define TPG_MAX_VERTICES 4096
#define TPG_MAX_OUT_DEGREE 64

typedef enum tpg_status {
  TPG_OK = 0,
  TPG_ERR_INVALID_ARG = -1,   /* NULL pointer, bad size, bad struct_size    */
  TPG_ERR_BAD_CSR = -2,       /* row_ptr not 0-based/monotone, col out of range,
                                 duplicate arcs under TPG_LOAD_STRICT        */
  TPG_ERR_BAD_ENTRY_EXIT = -3,/* entry/exit out of range, in-deg(entry) != 0
                                 or out-deg(exit) != 0 (Sec. 3 assumptions)   */
  TPG_ERR_UNREACHABLE = -4,   /* a vertex is not reachable from the entry or
                                 cannot reach the exit                        */
  TPG_ERR_OOM_HOST = -5,
  TPG_ERR_OOM_DEVICE = -6,
  TPG_ERR_CAPACITY = -7,      /* would exceed opts.pool_cap_bytes            */
  TPG_ERR_DEVICE = -8,        /* a HIP runtime call failed                   */
  TPG_ERR_UNSUPPORTED = -9,   /* > TPG_MAX_VERTICES vertices or out-degree
                                 > TPG_MAX_OUT_DEGREE                        */
  TPG_ERR_CALLBACK = -10      /* opts.on_chunk returned nonzero: stopped      */
} tpg_status;

/* load_flags */
#define TPG_LOAD_STRICT 0x1u          /* reject duplicate arcs instead of merging */
#define TPG_LOAD_ANY_DIGRAPH 0x2u     /* skip the entry/exit degree and reachability
                                         checks (prime paths of any digraph; test
                                         paths then need those checks to hold)   */
#define TPG_LOAD_BINARIZE 0x4u        /* the paper's input form (Sec. 3): every vertex
                                         of out-degree k > 2 keeps its first
                                         successor and hands the rest to a chain of
                                         k - 2 new decision vertices (ids n, n+1, ..
                                         in vertex order), x_i -> {s_(i+1), x_(i+1)}
                                         and the last -> {s_(k-1), s_k}, successors
                                         ascending; every vertex then has out-degree
                                         <= 2 and the graph's prime paths are those of
                                         the transformed graph (ids >= n are the new
                                         vertices; tpg_graph_info reports its size) */

/* opts.flags */
#define TPG_OUT_DEVICE 0x1u     /* results stay in device memory owned by the
                                   workspace, valid until the next call on it */
#define TPG_FORCE_TWO_PASS 0x2u /* plain form: per level count -> scan -> host
                                   reads the size -> fill (no device-side sizing) */
#define TPG_NO_TIMING 0x4u      /* skip per-phase event timing in tpg_stats     */
#define TPG_DIGEST 0x8u         /* also compute tpg_paths.digest of each set     */
#define TPG_DIGEST_ONLY 0x10u   /* counts and digest only: no path arrays are
                                   returned (tpg_paths.offsets / vertices NULL) */
#define TPG_STREAM 0x20u        /* deliver the results through opts.on_chunk
                                   (see tpg_chunk_fn); *out then holds only the
                                   counts and the digest of the whole set      */
#define TPG_TP_GREEDY 0x80u     /* tpg_test_paths: longest-first covering (the
                                   Ammann-Offutt generation the paper cites):
                                   prime paths in order of decreasing length
                                   (ties: canonical order); one that is already a
                                   contiguous subpath of a test path chosen
                                   before gets none, any other has its spliced
                                   test path chosen; the chosen test paths are
                                   returned in canonical order                  */
#define TPG_ORDER_BY_LAST 0x40u /* prime paths grouped by their last vertex (the
                                   paper's per-end-vertex output, Problem 1):
                                   ascending last vertex, canonical order inside
                                   a group; test paths keep the canonical order;
                                   not with TPG_STREAM                          */
#define TPG_NO_CALL_GRAPH 0x100u /* tpg_batch_test_paths: never capture or replay
                                   the call as one HIP graph (every call plans
                                   its launches on the host)                   */

typedef struct tpg_graph tpg_graph;         /* opaque, host memory */
typedef struct tpg_workspace tpg_workspace; /* opaque: device arena + stream */

typedef struct tpg_paths {
  int64_t n_paths;
  int64_t n_vertices;
  int64_t* offsets;  /* [n_paths + 1] */
  int32_t* vertices; /* [n_vertices]  */
  int32_t on_device; /* 1: device pointers (TPG_OUT_DEVICE) owned by the
                        workspace; 0: host memory owned by the library     */
  int32_t reserved_;
  /* Set digest (TPG_DIGEST, TPG_DIGEST_ONLY, TPG_STREAM; else zero): with
   * h(p) = FNV-1a 64 (offset basis 0xcbf29ce484222325, prime 0x100000001b3)
   * over the bytes of the int32 little-endian sequence (k, v_1, .., v_k) of
   * path p with k entries, digest[0] = sum of h(p) mod 2^64 and digest[1] =
   * xor of h(p) over the set.  It does not depend on the order of the paths,
   * so the digests of chunks combine by sum and xor. */
  uint64_t digest[2];
} tpg_paths;

/* Streaming (TPG_STREAM).  Called on the calling thread, in order, once per
 * chunk; the chunk (host memory, or device memory with TPG_OUT_DEVICE) is
 * valid only during the call.  first / end: for prime paths the range of
 * first vertices [first, end) whose prime paths the chunk holds (the
 * canonical order is by first vertex, so the chunks concatenate to the
 * canonical set); for test paths the index range of the chunk's paths in the
 * canonical set.  A nonzero return stops the call with TPG_ERR_CALLBACK. */
typedef int32_t (*tpg_chunk_fn)(void* ctx, const tpg_paths* chunk, int64_t first, int64_t end);

typedef struct tpg_stats {
  int64_t n_levels;       /* deepest level (path entries) that held a path   */
  int64_t n_nodes;        /* simple paths enumerated (all levels)            */
  int64_t n_extensions;   /* simple paths with >= 2 entries, cycles included */
  int64_t n_cycles;       /* closed simple cycles (all are prime)            */
  int64_t n_pp;
  int64_t n_pp_vertices;
  int64_t n_tp_spliced;   /* test paths before deduplication                 */
  int64_t n_tp;
  int64_t n_tp_vertices;
  int64_t n_overflows;    /* device-sized levels that overflowed and were grown */
  int64_t device_bytes;   /* workspace device memory in use                  */
  double ms_extend;       /* frontier extension + filter (all levels)        */
  double ms_rank;         /* canonical-order ranking + PP materialization    */
  double ms_tp;           /* BFS tables + splice + sort + dedup              */
  double ms_total;        /* device time of the whole call                   */
  double ms_extend_kernel;/* summed duration of the extension kernel launches */
  int64_t n_extend_launches;
  int64_t peak_level_nodes;      /* largest level (paths of one length)       */
  int64_t n_unions;              /* graph unions processed (batched form)     */
  int64_t pred_nodes;            /* predicted paths (batched form with predictions) */
  int64_t pred_peak_level_nodes; /* predicted largest level                  */
  int64_t call_graph;            /* batched form: 0 an ordinary call, 1 captured
                                    into one HIP graph by this call, 2 replayed
                                    from that graph (one launch, one wait), 3 an
                                    ordinary call because capturing this call
                                    failed (tpg_last_error() says why) */
  int64_t n_allocs;              /* batched form: device allocations and releases
                                    the call made in the workspace (a call that
                                    made any is not captured the next time) */
} tpg_stats;

typedef struct tpg_opts {
  uint32_t struct_size;     /* sizeof(tpg_opts)                             */
  uint32_t flags;           /* TPG_OUT_DEVICE | TPG_FORCE_TWO_PASS | ...     */
  void* stream;             /* hipStream_t to run on; NULL: the workspace's  */
  tpg_workspace* ws;        /* NULL: a temporary workspace for this call     */
  uint64_t pool_cap_bytes;  /* 0: no cap                                    */
  tpg_stats* stats;         /* optional                                     */
  int64_t* level_counts;    /* optional: level_counts[L] = simple paths with L
                               entries (closed cycles included), for
                               L = 0 .. level_counts_len-1 (batched form:
                               see tpg_batch_test_paths)                    */
  int32_t level_counts_len;
  int32_t reserved_;
  /* TPG_STREAM.  tpg_prime_paths runs the graph's first vertices in ranges
   * of chunk_vertices (0: 32) from scratch, so device memory is bounded by
   * the largest range's path tree, and delivers each range's prime paths;
   * tpg_test_paths delivers the canonical test paths in chunks of
   * chunk_paths (0: 1 << 20) paths. */
  tpg_chunk_fn on_chunk;
  void* chunk_ctx;
  int32_t chunk_vertices;
  int32_t reserved2_;
  int64_t chunk_paths;
} tpg_opts;

/* ------------------------------------------------------------------------
 * Loading (host only; no device is touched).
 *
 * n vertices 0..n-1; arcs of vertex v are col_idx[row_ptr[v] .. row_ptr[v+1]).
 * row_ptr has n+1 entries with row_ptr[0] = 0 and is non-decreasing; rows need
 * not be sorted.  Duplicate arcs are merged (rejected under TPG_LOAD_STRICT);
 * self-loops are allowed.  Checks (Sec. 3 assumptions): in-deg(entry) = 0,
 * out-deg(exit) = 0, and every vertex reachable from entry and reaching exit.
 * The inputs are copied; the caller keeps ownership.  On success *out is a
 * new handle to release with tpg_graph_free; on error *out = NULL.
 * ---------------------------------------------------------------------- */
tpg_status tpg_load_cfg_csr(int32_t n, const int64_t* row_ptr, const int32_t* col_idx,
                            int32_t entry, int32_t exit, uint32_t load_flags,
                            tpg_graph** out);
void tpg_graph_free(tpg_graph* g);
/* Vertex count, canonical arc count, entry, exit of a loaded graph. */
tpg_status tpg_graph_info(const tpg_graph* g, int32_t* n, int64_t* n_arcs, int32_t* entry,
                          int32_t* exit);
/* Canonical CSR (rows sorted, duplicates merged) copied into caller buffers of
 * n+1 and n_arcs entries. */
tpg_status tpg_graph_csr(const tpg_graph* g, int64_t* row_ptr, int32_t* col_idx);

/* ------------------------------------------------------------------------
 * Workspaces: a device arena that grows on demand and is reused across
 * calls (no device allocation once it is large enough), plus a stream.
 * device < 0 selects the current device.
 * ---------------------------------------------------------------------- */
tpg_status tpg_workspace_create(int32_t device, tpg_workspace** out);
void tpg_workspace_free(tpg_workspace* ws);
/* Device memory currently held by the workspace. */
int64_t tpg_workspace_bytes(const tpg_workspace* ws);

/* ------------------------------------------------------------------------
 * Prime paths (Def. 1) of a loaded graph, in canonical order.
 *
 * Level-synchronous extension of simple paths from every vertex (level L =
 * paths of L entries; a path is extended by each successor that is not on it,
 * and closes a cycle when the successor is its first vertex - the extension
 * rule of the paper's Update-Vertex / ExtendPath, Sec. 5); a path that cannot
 * be extended is prime iff it cannot be extended backward either (every
 * predecessor of its first vertex is on it); every closed cycle is prime.
 * opts may be NULL (defaults).  *out receives the set (see tpg_paths).
 * ---------------------------------------------------------------------- */
tpg_status tpg_prime_paths(const tpg_graph* g, const tpg_opts* opts, tpg_paths* out);

/* ------------------------------------------------------------------------
 * Test paths covering every prime path (Problem 1 output; Sec. 7.3).
 * If pp_out is non-NULL it also receives the prime paths.  tp_out receives
 * the deduplicated test paths in canonical order.  Requires the entry/exit
 * checks of tpg_load_cfg_csr to hold (else TPG_ERR_UNREACHABLE).
 * ---------------------------------------------------------------------- */
tpg_status tpg_test_paths(const tpg_graph* g, const tpg_opts* opts, tpg_paths* pp_out,
                          tpg_paths* tp_out);

/* Releases host results; device results (on_device = 1) are owned by the
 * workspace and this only clears the struct. */
void tpg_paths_free(tpg_paths* p);

/* ------------------------------------------------------------------------
 * The paper's own schedule, as a comparison variant (Sec. 5: the
 * Update-Vertex kernel and ExtendPath).  Every vertex owns a list of whole
 * paths ending at it; in each round one thread per vertex appends to its
 * list every path of a predecessor's newest paths that it can extend (not a
 * cycle, and the vertex absent from it or its first entry), marking that
 * path as extended; a round's paths are then kept when prime (a cycle, or
 * neither extended nor extendable backwards).  The paper lets the threads
 * run asynchronously until no list changes; here each round is a pair of
 * launches, so no thread waits on another, and the lists hold whole copies
 * of the paths as in the paper.
 *
 * out receives the prime paths of g grouped by last vertex (ascending), the
 * paper's output form; inside a group, by length, then in list order.  The
 * set equals tpg_prime_paths'.  opts as for tpg_prime_paths, without
 * TPG_STREAM or TPG_TP_GREEDY (TPG_ERR_INVALID_ARG).  stats: n_levels
 * (rounds), n_nodes (paths in all lists), n_extensions, n_pp,
 * n_pp_vertices, device_bytes, ms_total.
 * ---------------------------------------------------------------------- */
tpg_status tpg_prime_paths_vertex_lists(const tpg_graph* g, const tpg_opts* opts,
                                        tpg_paths* out);

/* ------------------------------------------------------------------------
 * Strongly connected components and prime-path types (Sec. 2).
 *
 * Per-vertex flags (tpg_scc): the vertex's component has a cycle (two or
 * more vertices, or a self-loop); SccEntryVertex (Def. 4: an arc enters the
 * vertex from another component); SccExitVertex (Def. 5: an arc leaves it
 * for another component).
 * ---------------------------------------------------------------------- */
#define TPG_SCC_CYCLIC 0x1u
#define TPG_SCC_ENTRY_VERTEX 0x2u
#define TPG_SCC_EXIT_VERTEX 0x4u
/* Prime-path types (tpg_prime_path_types), the first that matches in this
 * order: Def. 2 CompletePP (from the entry to the exit); Def. 9
 * SccInternalPP (starts and ends in one component with a cycle, and if
 * acyclic neither starts at one of its entry vertices nor ends at one of
 * its exit vertices); Def. 10 SccExitPP (starts in a component with a cycle,
 * ends at the exit); Def. 11 SccEntryPP (starts at the entry, ends in a
 * component with a cycle); TPG_PP_OTHER for none of them (for instance a
 * path from one component with a cycle to another). */
#define TPG_PP_COMPLETE 1
#define TPG_PP_SCC_INTERNAL 2
#define TPG_PP_SCC_EXIT 3
#define TPG_PP_SCC_ENTRY 4
#define TPG_PP_OTHER 5

/* Strongly connected components of g on the device (Sec. 2; they are the
 * vertices of the component graph, Def. 3).  comp (g's n int32) receives,
 * per vertex, the smallest vertex of its component; flags (n bytes) the
 * TPG_SCC_* bits; n_comp the number of components.  All three are host
 * memory owned by the caller, and any of them may be NULL.  Of opts only
 * the workspace and the stream are used. */
tpg_status tpg_scc(const tpg_graph* g, const tpg_opts* opts, int32_t* comp, uint8_t* flags,
                   int32_t* n_comp);

/* The TPG_PP_* type of each path of pps, a prime-path set of g such as
 * tpg_prime_paths' output on g, held in host or device memory as
 * pps->on_device says (a device set must be on the workspace's device and
 * is read in place, unchecked).  types (pps->n_paths bytes, host, may be
 * NULL) receives each path's type; counts (6 int64, host, may be NULL) the
 * number of paths of each type, index = type (counts[0] = 0).  A host set
 * whose offsets are not increasing from 0 to n_vertices, or whose vertices
 * lie outside g, gives TPG_ERR_INVALID_ARG.  Of opts only the workspace and
 * the stream are used. */
tpg_status tpg_prime_path_types(const tpg_graph* g, const tpg_paths* pps, const tpg_opts* opts,
                                uint8_t* types, int64_t* counts);

/* The compositional method of Sec. 2.1 on the device.
 *
 * tpg_ccfg: the component graph (Def. 3).  comp (n int32, host, may be NULL)
 * receives each vertex's component label (its smallest vertex), n_comp (may
 * be NULL) the number of components, *n_arcs the number of arcs of g whose
 * ends lie in different components (the component graph's arcs, one per arc
 * of g).  arc_src / arc_dst (host, both or neither, arc_cap entries each)
 * receive those arcs as vertex pairs of g in CSR order; n_arcs > arc_cap
 * gives TPG_ERR_CAPACITY (after *n_arcs is set).  Of opts only the
 * workspace and the stream are used. */
tpg_status tpg_ccfg(const tpg_graph* g, const tpg_opts* opts, int32_t* comp, int32_t* n_comp,
                    int64_t* n_arcs, int32_t* arc_src, int32_t* arc_dst, int64_t arc_cap);

/* tpg_scc_paths: the paths of Sec. 2.1's path extraction, over every
 * component with a cycle (Defs. 6-8), each path acyclic and inside one
 * component:
 *  - entry_exit: every path from an SccEntryVertex to an SccExitVertex;
 *  - exit_paths: the paths from a vertex that is not an SccEntryVertex to an
 *    SccExitVertex that no longer such path to the same SccExitVertex
 *    contains (maximal per exit vertex);
 *  - entry_paths: the paths from an SccEntryVertex to a vertex that is not
 *    an SccExitVertex that no longer such path from the same SccEntryVertex
 *    contains (maximal per entry vertex).
 * Each set is grouped by component (ascending smallest vertex); inside a
 * component entry_exit and entry_paths are in lexicographic order,
 * exit_paths in the lexicographic order of the reversed paths (grouped by
 * exit vertex).  Any output may be NULL; opts->flags may hold TPG_OUT_DEVICE (results then live
 * in the workspace until its next call) and TPG_FORCE_TWO_PASS. */
tpg_status tpg_scc_paths(const tpg_graph* g, const tpg_opts* opts, tpg_paths* entry_exit,
                         tpg_paths* exit_paths, tpg_paths* entry_paths);

/* tpg_scc_internal_pps: Sec. 2.1's prime-path generation on each component
 * with a cycle taken alone (its vertices and the arcs between them), kept
 * when they are SccInternalPPs (Def. 9: a cycle, or an acyclic path that
 * neither starts at an SccEntryVertex nor ends at an SccExitVertex), in g's
 * vertex ids; grouped by component (ascending smallest vertex), in
 * lexicographic order inside a group.  These are exactly the prime paths of
 * g of type TPG_PP_SCC_INTERNAL.  Flags as for tpg_scc_paths. */
tpg_status tpg_scc_internal_pps(const tpg_graph* g, const tpg_opts* opts, tpg_paths* out);

/* tpg_merged_pps: Sec. 2.1's merging: the CompletePPs (Def. 2), SccExitPPs
 * (Def. 10) and SccEntryPPs (Def. 11) built from the component graph and
 * the extracted paths, each set in lexicographic order.  The component
 * graph's paths with every component with a cycle replaced by one of its
 * SccEntryExitPaths give the CompletePPs; a CompletePP's part after the
 * exit vertex where it leaves a component, prefixed by that component's
 * SccExitPaths to that vertex, the SccExitPPs; its part before the vertex
 * where it enters a component, followed by the SccEntryPaths from that
 * vertex, the SccEntryPPs.  Merged paths that can still be extended at one
 * end are not prime and are left out.  The composition runs as the path
 * extension on a macro graph of the paths (at most TPG_MAX_VERTICES
 * vertices, else TPG_ERR_UNSUPPORTED).  g must be a CFG loaded with the
 * entry/exit checks.  Outputs and flags as for tpg_scc_paths. */
tpg_status tpg_merged_pps(const tpg_graph* g, const tpg_opts* opts, tpg_paths* complete,
                          tpg_paths* exit_pps, tpg_paths* entry_pps);

/* tpg_prime_path_types without device allocation, for callers that cannot
 * allocate device memory (code under stream capture, serving loops,
 * harnesses that forbid hipMalloc).  The prime-path set is in device memory
 * on the current device (offsets int64 [n_paths + 1], vertices int32, read
 * in place, unchecked); d_types (n_paths bytes, device, caller-owned, may be
 * NULL) receives each path's type; counts (6 int64, host, may be NULL) the
 * number of each type, as tpg_prime_path_types.  stream: a hipStream_t of
 * the current device, or NULL for the default stream; the call returns once
 * the stream has finished its work.  Everything else the kernels use (the
 * graph's CSR staged on the device, the component search's arrays, labels,
 * flags, counters) lives in a fixed 1 MiB device array that the library
 * holds on each device until the process ends: a graph that needs more
 * (about 108 000 arcs at 4096 vertices) gives TPG_ERR_CAPACITY before any
 * device work.  Calls on one device share that array and the last call's
 * contents stay in it, so calls that overlap on one device race; calls on
 * different devices do not.  No device memory is allocated or freed. */
tpg_status tpg_prime_path_types_noalloc(const tpg_graph* g, const int64_t* d_offsets,
                                        const int32_t* d_vertices, int64_t n_paths, void* stream,
                                        uint8_t* d_types, int64_t* counts);

/* ------------------------------------------------------------------------
 * Batched form: prime and test paths of many CFGs in one call.
 *
 * The same computation as tpg_test_paths, per graph.  Graphs are grouped by
 * visited-set width and each group runs as one disjoint union, so every
 * level of every graph in the group is extended by the same launches (all
 * compute units busy even when each graph is small).  Results are packed
 * graph after graph in the caller's order, each graph's sets canonical and
 * in its own vertex ids: graph i owns prime paths pp_first[i] ..
 * pp_first[i+1]-1 of pp (likewise tp / tp_first).
 *
 * predicted (optional, host, [n_graphs * 65] floats): per graph, log1p of the
 * predicted number of simple paths with L entries for L = 1..64 (index L-1;
 * index 63 pools all deeper levels) and log1p of the predicted prime-path
 * count (index 64).  With it the path pool is sized in one pass from the
 * prediction (25% margin) and, under a pool cap, graphs are admitted into
 * unions by predicted footprint; a level that outgrows its allocation is
 * detected on the device, grown to its exact size and replayed.  A value
 * that is not a finite number counts as 0; predicted capacities are capped
 * at the 2^31-path limit, at half the pool cap and at half the free device
 * memory, and a union whose predicted capacities cannot be allocated is
 * sized from the smallest buffers by growth and replay instead (the
 * workspace remembers up to 64 such unions and sizes them from the capacity
 * it holds on later calls).  Without it, sizing starts from the workspace's
 * current capacity (or the exact two-pass form with TPG_FORCE_TWO_PASS).
 * Results never depend on the prediction.
 *
 * Repeated calls: with opts->ws set, TPG_NO_TIMING (or no stats), no level
 * counts and none of TPG_FORCE_TWO_PASS, TPG_STREAM, TPG_TP_GREEDY,
 * TPG_DIGEST, TPG_DIGEST_ONLY, TPG_NO_CALL_GRAPH, a call that repeats the workspace's previous
 * batched call (same graph handles, flags, stream, pool cap, predictions and
 * tuning) and whose predecessor allocated nothing is captured into one HIP
 * graph, and later repeats replay it: one launch and one wait instead of a
 * host round trip per step.  Every device value the host read during the
 * recorded call is copied out again by the graph and compared after each
 * replay; a mismatch drops the graph and the call runs the ordinary way, so
 * results are those of an ordinary call.  stats->call_graph says which way
 * the call ran.  Calls on one workspace must not overlap (as always).
 *
 * opts->level_counts, if it holds >= 64 * n_graphs entries, receives the
 * per-graph path counts of levels 1..64 (deeper levels pooled into 64):
 * the labels the size predictor is trained on.
 * ---------------------------------------------------------------------- */
typedef struct tpg_batch_result {
  tpg_paths pp;
  tpg_paths tp;
  int64_t* pp_first; /* [n_graphs + 1], host memory owned by the library */
  int64_t* tp_first; /* [n_graphs + 1] */
  int32_t n_graphs;
  int32_t reserved_;
} tpg_batch_result;

tpg_status tpg_batch_test_paths(const tpg_graph* const* graphs, int32_t n_graphs,
                                const tpg_opts* opts, const float* predicted,
                                tpg_batch_result* out);
void tpg_batch_result_free(tpg_batch_result* r);

/* ------------------------------------------------------------------------
 * Launch-shape tuning of the frontier-extension kernel.
 *
 * Per visited-set width W = 2^i words (index i = 0..6; W is the register
 * width, ceil(V / 64) rounded up to a power of two): the most parents per
 * thread (1, 2, 4 or 8; a tile is threads * items parents and claims its
 * slice of the next level with one device-scope atomic), persistent
 * workgroups per compute unit (1..32) and the kernel variant (0: load-
 * balanced tiles of 256 threads staged in LDS; 1 / 2: thread-per-parent with
 * visited sets in registers, 256 / 1024 threads).  Defaults come from sweeps
 * on MI355X (W = 4: variant 2, 1 item, 2 workgroups; W = 8: variant 2,
 * 1 item, 4 workgroups).  tpg_autotune times every combination on the given
 * graphs (grouped by width as in the batched form), keeps the fastest per
 * width in the workspace (opts->ws, required) and returns the table; results
 * never depend on the tuning.
 * ---------------------------------------------------------------------- */
typedef struct tpg_tuning {
  int32_t items[7];
  int32_t wgs_per_cu[7];
  int32_t variant[7];
  double best_ms[7]; /* summed extension-kernel time of the best shape (0: untuned) */
} tpg_tuning;

tpg_status tpg_autotune(const tpg_graph* const* graphs, int32_t n_graphs, const tpg_opts* opts,
                        tpg_tuning* out);
tpg_status tpg_workspace_set_tuning(tpg_workspace* ws, const tpg_tuning* t);
tpg_status tpg_workspace_get_tuning(const tpg_workspace* ws, tpg_tuning* t);

/* ------------------------------------------------------------------------
 * Size predictor for the batched form (host features, device network).
 *
 * tpg_features: 32 structural features per graph from its CSR alone (sizes,
 * cyclomatic complexity, branching bits, natural-loop depth histogram, SCCs,
 * if-else diamonds, switch fan-outs, distances, entry-to-exit paths of the
 * component DAG); out is [n_graphs * 32], host memory.
 *
 * tpg_mlp: 32 -> 128 -> 128 -> 65 perceptron (ReLU), BF16 operands on the
 * matrix cores with FP32 accumulation, Adam (beta 0.9 / 0.999, eps 1e-8) on
 * FP32 master weights.  Output j < 64: log1p(paths with j+1 entries), deeper
 * levels pooled into j = 63; output 64: log1p(prime paths).  Loss: mean
 * squared error over the 65 outputs.  Parameters are packed as W1 [32][128],
 * b1 [128], W2 [128][128], b2 [128], W3 [128][65], b3 [65]
 * (tpg_mlp_num_params() floats).  Inputs are normalized as (x - mean) / std
 * before the first layer.  All x / y / t arrays are host memory, row-major.
 * ---------------------------------------------------------------------- */
typedef struct tpg_mlp tpg_mlp;
#define TPG_MLP_IN 32
#define TPG_MLP_OUT 65

tpg_status tpg_features(const tpg_graph* const* graphs, int32_t n_graphs, float* out);
int32_t tpg_mlp_num_params(void);
tpg_status tpg_mlp_create(int32_t device, uint64_t seed, tpg_mlp** out);
void tpg_mlp_free(tpg_mlp* m);
tpg_status tpg_mlp_set_params(tpg_mlp* m, const float* params);
tpg_status tpg_mlp_get_params(const tpg_mlp* m, float* params);
tpg_status tpg_mlp_set_normalizer(tpg_mlp* m, const float* mean, const float* std);
/* y: [n * 65] */
tpg_status tpg_mlp_forward(tpg_mlp* m, const float* x, int32_t n, float* y);
/* gradients of the loss w.r.t. the packed parameters, without updating */
tpg_status tpg_mlp_gradients(tpg_mlp* m, const float* x, const float* t, int32_t n, float* grad,
                             float* loss);
/* forward + backward + one Adam step with learning rate lr */
tpg_status tpg_mlp_train_step(tpg_mlp* m, const float* x, const float* t, int32_t n, float lr,
                              float* loss);
tpg_status tpg_mlp_save(const tpg_mlp* m, const char* path);
tpg_status tpg_mlp_load(int32_t device, const char* path, tpg_mlp** out);

/* ------------------------------------------------------------------------
 * Misc.
 * ---------------------------------------------------------------------- */
const char* tpg_status_str(tpg_status s);
const char* tpg_last_error(void);       /* thread-local, never NULL */
const char* tpg_version(void);
int32_t tpg_device_count(void);

#ifdef __cplusplus
}
#endif
#endif /* TPG_H_ */
