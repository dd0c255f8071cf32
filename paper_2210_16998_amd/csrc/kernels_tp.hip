// Test-path kernels: BFS tables, splice, canonical sort and deduplication.
//
// A test path extends a prime path to the initial and final nodes (paper
// Sec. 7.3, the Ammann-Offutt construction; Problem 1 asks for test paths
// covering every prime path).  The shortest connection is taken, and among
// shortest ones the lexicographically smallest, so the result is unique:
//  * prefix(v): smallest shortest entry -> v path.  A FIFO breadth-first
//    search that scans successors in ascending order discovers it (each
//    layer's queue order is the lexicographic order of those paths); the
//    level-synchronous search here reproduces FIFO discovery order by giving
//    every vertex the discoverer with the smallest (queue position, successor
//    slot) key.
//  * suffix(v): smallest shortest v -> exit path: distances to the exit by a
//    reverse search, then the smallest successor one step closer.
//  * TP(p) = prefix(v1) without v1 ++ p ++ suffix(vk) without vk.
//
// Sorting: prime paths arrive in lexicographic order, hence grouped by first
// vertex; within a group all test paths share the prefix and keep the order
// of their prime paths, and no two are equal.  The groups are therefore
// already sorted runs, merged pairwise (merge path partitioning, each thread
// merges a fixed-size chunk), after which duplicates are adjacent.  Almost
// every comparison is decided by two 64-bit keys per path derived from the
// BFS tree (see tp_cmp).

#include <climits>

#include "kernels.h"

namespace tpg {

constexpr int kBfsThreads = 256;
constexpr int kMaxComp = 4096;  // vertices per component

// Exclusive scan of data[0..m) in place (m <= kMaxComp), in chunks of
// 4 * kBfsThreads; returns the total.
__device__ int lds_excl_scan(int16_t* data, int m, int32_t* s_w) {
  int carry = 0;
  for (int c0 = 0; c0 < m; c0 += 4 * kBfsThreads) {
    const int b = c0 + (int)threadIdx.x * 4;
    int v[4];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = (b + k < m) ? (int)data[b + k] : 0;
      sum += v[k];
    }
    int tot;
    int pre = block_excl_scan<kBfsThreads, int>(sum, tot, s_w) + carry;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (b + k < m) data[b + k] = (int16_t)pre;
      pre += v[k];
    }
    carry += tot;
    __syncthreads();
  }
  return carry;
}

// One workgroup per component: distances from the entry with the FIFO
// (smallest discoverer) parent, the BFS tree's preorder (children in
// ascending order) as rank ranges, distances to the exit, and next[].
//
// The forward search keeps one queue in LDS whose layers are contiguous;
// the children of a vertex form a contiguous ascending block of the next
// layer, which gives subtree sizes bottom-up and preorder ranks top-down.
__global__ __launch_bounds__(kBfsThreads) void k_bfs_dist(DGraph g, BfsOut b) {
  __shared__ int16_t s_df[kMaxComp];
  __shared__ int16_t s_db[kMaxComp];
  __shared__ int32_t s_key[kMaxComp];   // smallest discoverer key, then the parent (local id)
  __shared__ int16_t s_q[kMaxComp];     // forward queue (layers contiguous), then reverse queue
  __shared__ int16_t s_lb[kMaxComp + 2];  // layer d of the forward queue: [s_lb[d], s_lb[d + 1])
  __shared__ int16_t s_cnt[kMaxComp];   // per-layer child counts, then preorder ranks
  __shared__ int32_t s_sz[kMaxComp];    // subtree sizes, then reverse-search marks
  __shared__ int32_t s_w[kBfsThreads / 64];
  __shared__ int32_t s_m;
  const int c = (int)blockIdx.x;
  const int base = g.cbase[c];
  const int nc = g.cbase[c + 1] - base;
  const int tid = (int)threadIdx.x;
  for (int v = tid; v < nc; v += kBfsThreads) {
    s_df[v] = -1;
    s_db[v] = -1;
    s_key[v] = INT_MAX;
    s_sz[v] = 1;
    b.parent[base + v] = -1;
    b.next[base + v] = -1;
    b.ccnt[base + v] = 0;
    b.cfirst[base + v] = base;
  }
  const int el = g.centry[c] - base;
  if (tid == 0) {
    s_df[el] = 0;
    s_key[el] = -1;
    s_q[0] = (int16_t)el;
    s_lb[0] = 0;
    s_lb[1] = 1;
  }
  __syncthreads();
  int qb = 0, qe = 1, d = 0;
  while (qe > qb) {
    const int m = qe - qb;
    for (int q = tid; q < m; q += kBfsThreads) {
      const int u = base + s_q[qb + q];
      for (int k = g.sp[u]; k < g.sp[u + 1]; ++k) {
        const int wl = g.s[k] - base;
        if (s_df[wl] == -1) atomicMin(&s_key[wl], q * 64 + (k - g.sp[u]));
      }
    }
    __syncthreads();
    for (int q = tid; q < m; q += kBfsThreads) {
      const int u = base + s_q[qb + q];
      int cnt = 0;
      for (int k = g.sp[u]; k < g.sp[u + 1]; ++k) {
        const int wl = g.s[k] - base;
        if (s_df[wl] == -1 && s_key[wl] == q * 64 + (k - g.sp[u])) ++cnt;
      }
      s_cnt[q] = (int16_t)cnt;
    }
    __syncthreads();
    const int m2 = lds_excl_scan(s_cnt, m, s_w);
    for (int q = tid; q < m; q += kBfsThreads) {
      const int u = base + s_q[qb + q];
      int pos = qe + s_cnt[q];
      b.cfirst[u] = base + pos;
      b.ccnt[u] = (q + 1 < m ? (int)s_cnt[q + 1] : m2) - (int)s_cnt[q];
      for (int k = g.sp[u]; k < g.sp[u + 1]; ++k) {
        const int wl = g.s[k] - base;
        if (s_df[wl] == -1 && s_key[wl] == q * 64 + (k - g.sp[u])) {
          s_q[pos++] = (int16_t)wl;
          b.parent[base + wl] = u;
        }
      }
    }
    __syncthreads();
    for (int i = tid; i < m2; i += kBfsThreads) {
      const int wl = s_q[qe + i];
      s_df[wl] = (int16_t)(d + 1);
      s_key[wl] = s_q[qb + s_key[wl] / 64];
    }
    qb = qe;
    qe += m2;
    ++d;
    if (tid == 0) s_lb[d + 1] = (int16_t)qe;
    __syncthreads();
  }
  const int nlayers = d;  // layers 0 .. nlayers - 1
  for (int i = tid; i < qe; i += kBfsThreads) b.bq[base + i] = base + s_q[i];
  // subtree sizes, deepest layer first
  for (int l = nlayers - 1; l >= 1; --l) {
    for (int i = s_lb[l] + tid; i < s_lb[l + 1]; i += kBfsThreads) {
      const int v = s_q[i];
      atomicAdd(&s_sz[s_key[v]], s_sz[v]);
    }
    __syncthreads();
  }
  // preorder ranks, top layer first: a vertex follows its parent and the
  // subtrees of its smaller siblings
  if (tid == 0) s_cnt[el] = 0;
  __syncthreads();
  for (int l = 1; l < nlayers; ++l) {
    const int lo = s_lb[l];
    for (int i = lo + tid; i < s_lb[l + 1]; i += kBfsThreads) {
      const int v = s_q[i];
      const int p = s_key[v];
      int acc = 0;
      for (int j = i - 1; j >= lo && s_key[s_q[j]] == p; --j) acc += s_sz[s_q[j]];
      s_cnt[v] = (int16_t)(s_cnt[p] + 1 + acc);
    }
    __syncthreads();
  }
  for (int v = tid; v < nc; v += kBfsThreads) {
    const bool r = s_df[v] >= 0;
    b.pre[base + v] = r ? base + s_cnt[v] : -1;
    b.pend[base + v] = r ? base + s_cnt[v] + s_sz[v] : -1;
  }
  __syncthreads();
  // distances to the exit (reverse search; order does not matter)
  for (int v = tid; v < nc; v += kBfsThreads) s_sz[v] = 0;
  __syncthreads();
  const int xl = g.cexit[c] - base;
  if (tid == 0) {
    s_db[xl] = 0;
    s_q[0] = (int16_t)xl;
    s_sz[xl] = 1;
  }
  __syncthreads();
  qb = 0;
  qe = 1;
  d = 0;
  while (qe > qb) {
    if (tid == 0) s_m = 0;
    __syncthreads();
    for (int q = qb + tid; q < qe; q += kBfsThreads) {
      const int u = base + s_q[q];
      for (int k = g.pp[u]; k < g.pp[u + 1]; ++k) {
        const int wl = g.p[k] - base;
        if (atomicExch(&s_sz[wl], 1) == 0) s_q[qe + atomicAdd(&s_m, 1)] = (int16_t)wl;
      }
    }
    __syncthreads();
    const int m2 = s_m;
    for (int i = tid; i < m2; i += kBfsThreads) s_db[s_q[qe + i]] = (int16_t)(d + 1);
    qb = qe;
    qe += m2;
    ++d;
    __syncthreads();
  }
  for (int v = tid; v < nc; v += kBfsThreads) {
    b.dist_f[base + v] = s_df[v];
    b.dist_b[base + v] = s_db[v];
    if (v != xl && s_db[v] > 0) {
      const int u = base + v;
      for (int k = g.sp[u]; k < g.sp[u + 1]; ++k)
        if (s_db[g.s[k] - base] == s_db[v] - 1) {
          b.next[u] = g.s[k];
          break;
        }
    }
  }
}

hipError_t launch_bfs_dist(const DGraph& g, const BfsOut& b, hipStream_t st) {
  k_bfs_dist<<<(unsigned)g.n_comp, kBfsThreads, 0, st>>>(g, b);
  return hipGetLastError();
}

// Prefix / suffix tables (graph-wide ids): entries before v on its
// smallest shortest path from the entry, entries after v to the exit.
__global__ void k_bfs_tables(DGraph g, BfsOut b) {
  const int v = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (v >= g.n) return;
  const int df = b.dist_f[v], db = b.dist_b[v];
  if (df > 0) {
    const int64_t lo = b.pfx_off[v];
    int64_t pos = lo + df - 1;
    int x = b.parent[v];
    while (x >= 0 && pos >= lo) {
      b.pfx[pos--] = x;
      x = b.parent[x];
    }
  }
  if (db > 0) {
    int64_t pos = b.sfx_off[v];
    const int64_t hi = pos + db;
    int x = b.next[v];
    while (x >= 0 && pos < hi) {
      b.sfx[pos++] = x;
      x = b.next[x];
    }
  }
}

hipError_t launch_bfs_tables(const DGraph& g, const BfsOut& b, hipStream_t st) {
  k_bfs_tables<<<(unsigned)((g.n + kBlock - 1) / kBlock), kBlock, 0, st>>>(g, b);
  return hipGetLastError();
}

// Graph-wide ids -> ids local to each component (batched output).
__global__ void k_localize(const int32_t* loc, int32_t* v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = loc[v[i]];
}

hipError_t launch_localize(const int32_t* loc, int32_t* v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_localize<<<(unsigned)std::min<int64_t>(4096, (n + kBlock - 1) / kBlock), kBlock, 0, st>>>(loc, v, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// splice
// ---------------------------------------------------------------------------
__global__ void k_tp_len(const int64_t* pp_off, const int32_t* pp_vtx, int64_t n_pp, BfsOut b,
                         int64_t* tp_len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pp) return;
  const int64_t o0 = pp_off[i], o1 = pp_off[i + 1];
  const int v1 = pp_vtx[o0], vk = pp_vtx[o1 - 1];
  tp_len[i] = (b.pfx_off[v1 + 1] - b.pfx_off[v1]) + (o1 - o0) + (b.sfx_off[vk + 1] - b.sfx_off[vk]);
}

// Prime paths are sorted, hence grouped by first vertex: rb[v] = index of the
// first prime path whose first vertex is >= v (v = 0..n), from the points
// where the first vertex changes.
__global__ void k_run_bounds(const int64_t* pp_off, const int32_t* pp_vtx, int64_t n_pp, int n,
                             int64_t* rb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pp) return;
  const int cur = pp_vtx[pp_off[i]];
  const int prev = i == 0 ? -1 : pp_vtx[pp_off[i - 1]];
  for (int u = prev + 1; u <= cur; ++u) rb[u] = i;
  if (i == n_pp - 1)
    for (int u = cur + 1; u <= n; ++u) rb[u] = n_pp;
}

hipError_t launch_tp_len(const int64_t* pp_off, const int32_t* pp_vtx, int64_t n_pp, int n,
                         const BfsOut& b, int64_t* tp_len, int64_t* rb, hipStream_t st) {
  if (n_pp == 0) return hipSuccess;
  const unsigned grid = (unsigned)((n_pp + kBlock - 1) / kBlock);
  if (tp_len) k_tp_len<<<grid, kBlock, 0, st>>>(pp_off, pp_vtx, n_pp, b, tp_len);
  if (rb) k_run_bounds<<<grid, kBlock, 0, st>>>(pp_off, pp_vtx, n_pp, n, rb);
  return hipGetLastError();
}

// Comparison key of a test path t (graph-wide ids; ranks fit 18 bits):
//  * w = last vertex of the longest prefix of t that is a BFS-tree path
//    (the tree path to the prime path's first vertex u, extended while each
//    next entry is the tree child of the one before), D = its depth;
//  * e = the entry after that prefix (none when t ends there);
//  * split = preorder rank of w's first tree child larger than e (pend(w)
//    when none; pre(w) + 1 when there is no e).
// k1 = pre(w) | pend(w) << 18 | D << 36 | (e exists) << 49
// k2 = e | split << 17 | pre(u) << 35
// k3 .. = kTpKeyTail words of the entries after e, P = 64 / eb to a word,
//      each as entry + 1 in eb bits (0 past the end), the first one highest:
//      comparing them word by word compares those entries lexicographically,
//      a path that ends first being the smaller
constexpr uint64_t kM17 = (1ull << 17) - 1, kM18 = (1ull << 18) - 1, kM13 = (1ull << 13) - 1;

// Packed copy of test path x (entry offset off): its entries, each as
// entry + 1 in eb bits, pe = 64 / eb to a 64-bit word with the first one
// highest and 0 past the end, so that comparing words in order compares the
// entries lexicographically (a path that ends first being the smaller).  The
// words start at tp_pk_base(off, x), which is even (16-byte aligned) and
// leaves each path at least its ceil(len / pe) words, so an aligned pair of
// words that starts inside a path's words stays inside its slot.
__device__ __forceinline__ int64_t tp_pk_base(int64_t off, int64_t x, int pe) {
  return ((off + pe - 1) / pe + 2 * x + 1) & ~(int64_t)1;
}

// Packed prefix and suffix tables: row v holds v's prefix (suffix) entries
// packed like the test paths' words (entry + 1 in eb bits, pe per word, first
// one highest, 0 past the end), followed by one zero word.  Row v starts at
// word pfx_off[v] / pe + 2 v (sfx_off for the suffix rows), which leaves
// every row its ceil(len / pe) + 1 words without a scan.
__device__ __forceinline__ int64_t tbl_pk_base(int64_t off, int v, int pe) {
  return off / pe + 2 * (int64_t)v;
}

__global__ void k_pack_tables(int n, BfsOut b, int eb) {
  const int v = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (v >= n) return;
  const int pe = 64 / eb;
#pragma unroll 1
  for (int side = 0; side < 2; ++side) {
    const int64_t* off = side ? b.sfx_off : b.pfx_off;
    const int32_t* tbl = side ? b.sfx : b.pfx;
    uint64_t* pk = side ? b.sfx_pk : b.pfx_pk;
    const int64_t o = off[v];
    const int len = (int)(off[v + 1] - o);
    const int64_t base = tbl_pk_base(o, v, pe);
    const int nw = (len + pe - 1) / pe + 1;
    for (int q = 0; q < nw; ++q) {
      uint64_t w = 0;
      for (int j = 0; j < pe; ++j) {
        const int k = q * pe + j;
        w = (w << eb) | (k < len ? (uint64_t)(tbl[o + k] + 1) : 0ull);
      }
      pk[base + q] = w;
    }
  }
}

hipError_t launch_pack_tables(int n, const BfsOut& b, int eb, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (eb < 1 || eb > 32) return hipErrorInvalidValue;
  k_pack_tables<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(n, b, eb);
  return hipGetLastError();
}

// A workgroup splices kSplicePaths consecutive test paths.  Their layout
// (where each one's prefix, prime-path and suffix entries are, and the word
// offset of its packed suffix row) goes to LDS with a map of the words it
// builds to their paths, then each thread builds one packed word at a time
// (pe consecutive entries; the built words of the paths are one flat range).
// A word that lies wholly in the prefix is neither written nor visited: it is
// the same word of the first vertex's packed prefix row, from which the
// unpack takes it, and no comparison reads it (they start past the prime
// path's first vertex).  A word that lies wholly in the suffix is cut from two
// consecutive words of the last vertex's packed suffix row; one that lies
// wholly in the prime path packs pe consecutive prime-path entries; only the
// words across two of these parts are built entry by entry.  The entry width
// is a compile-time constant, so the shifts and the divisions by pe are
// constants: the kernel is bound by its work per word.  The words the key's
// entry windows start in are kept in LDS, and after a barrier the windows
// (k_tp_keys has stored where they start) are cut from them.  The plain
// entries are written only when asked for (tp_vtx not null, every word then
// built entry by entry): the comparisons read the packed words and the kept
// paths are unpacked from them when gathered.
constexpr int kSplicePaths = 64;
constexpr int kSpliceMap = 8192;  // built words a workgroup maps to paths in LDS
constexpr int kSpliceMixed = 512;  // words across two parts listed per workgroup

struct SpliceRow {
  int64_t o0, p0, s0;  // prime-path entries, prefix table, suffix table
  int32_t lp, lq, ls;  // prefix, prime-path and suffix lengths
  int32_t v1, vk;      // first and last vertex of the prime path
};

// Layout of test path i: where its prefix, prime-path and suffix entries are.
__device__ __forceinline__ SpliceRow splice_row(const int64_t* pp_off, const int32_t* pp_vtx,
                                                const BfsOut& b, int64_t i) {
  const int64_t o0 = pp_off[i], o1 = pp_off[i + 1];
  const int v1 = pp_vtx[o0], vk = pp_vtx[o1 - 1];
  SpliceRow r;
  r.o0 = o0;
  r.p0 = b.pfx_off[v1];
  r.lp = (int32_t)(b.pfx_off[v1 + 1] - r.p0);
  r.lq = (int32_t)(o1 - o0);
  r.s0 = b.sfx_off[vk];
  r.ls = (int32_t)(b.sfx_off[vk + 1] - r.s0);
  r.v1 = v1;
  r.vk = vk;
  return r;
}

__device__ __forceinline__ int splice_entry(const SpliceRow& r, const int32_t* pp_vtx,
                                            const BfsOut& b, int64_t k) {
  if (k < r.lp) return b.pfx[r.p0 + k];
  if (k < r.lp + r.lq) return pp_vtx[r.o0 + (k - r.lp)];
  return b.sfx[r.s0 + (k - r.lp - r.lq)];
}

// Entries k .. k + pe - 1 of a packed test path (words p, len entries) in
// the packed word format, entries past the end 0: cut from two consecutive
// words, the second read only when the window reaches into it.
__device__ __forceinline__ uint64_t packed_window(const uint64_t* p, int64_t len, int64_t k, int pe,
                                                  int eb) {
  if (k >= len) return 0;
  const int64_t q = k / pe;
  const int r = (int)(k - q * pe);
  uint64_t w = p[q];
  if (r != 0) {
    const int hb = (pe - r) * eb;  // bits of the first word's entries r .. pe-1
    w = (w & ((1ull << hb) - 1)) << (r * eb);
    if (k + (pe - r) < len) w |= p[q + 1] >> hb;
  }
  const int64_t nv = len - k;
  if (nv < pe) w &= ~((1ull << ((pe - nv) * eb)) - 1);
  return w;
}

template <int EB>
__global__ __launch_bounds__(kBlock) void k_tp_write(const int64_t* pp_off, const int32_t* pp_vtx,
                                                     int64_t n_pp, BfsOut b, const int64_t* tp_off,
                                                     int32_t* tp_vtx, uint64_t* pk, uint64_t* key,
                                                     int32_t* idx) {
  constexpr int pe = 64 / EB;
  // the words each key's entry windows are cut from (k_tp_keys has stored
  // where the window starts), kept as they are built
  __shared__ uint64_t s_kw[kSplicePaths][kTpKeyTail + 1];
  __shared__ int32_t s_kf[kSplicePaths];  // first entry of the windows
  __shared__ int32_t s_kq[kSplicePaths];  // its word
  // words across two parts, built after the others (see below)
  __shared__ int32_t s_mix[kSpliceMixed];
  __shared__ int32_t s_nmix;
  __shared__ SpliceRow s_row[kSplicePaths];
  __shared__ int64_t s_w[kSplicePaths + 1];   // entry offsets
  __shared__ int32_t s_a[kSplicePaths + 1];   // packed-word offsets from the first path's
  __shared__ int64_t s_sb[kSplicePaths];      // first word of the packed suffix row
  __shared__ int32_t s_c[kSplicePaths + 1];   // built words before each path
  __shared__ int32_t s_q0[kSplicePaths];      // a path's first built word
  __shared__ uint8_t s_map[kSpliceMap];       // built word -> path
  __shared__ int64_t s_a0;
  const int tid = (int)threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * kSplicePaths;
  const int cnt = (int)(n_pp - i0 < kSplicePaths ? n_pp - i0 : kSplicePaths);
  int64_t a_mine = 0;
  if (tid < cnt) {
    const int64_t i = i0 + tid;
    const SpliceRow r = splice_row(pp_off, pp_vtx, b, i);
    s_row[tid] = r;
    const int64_t o = tp_off[i];
    s_w[tid] = o;
    a_mine = tp_pk_base(o, i, pe);
    s_sb[tid] = tbl_pk_base(r.s0, r.vk, pe);
    idx[i] = (int32_t)i;
    // the entries after e start two past the tree prefix's last entry
    const int32_t f = (int32_t)((key[(int64_t)kTpKeyWords * i] >> 36) & kM13) + 2;
    s_kf[tid] = f;
    s_kq[tid] = f / pe;
#pragma unroll
    for (int j = 0; j <= kTpKeyTail; ++j) s_kw[tid][j] = 0;
  }
  if (tid == cnt) {
    const int64_t o = tp_off[i0 + cnt];
    s_w[cnt] = o;
    a_mine = tp_pk_base(o, i0 + cnt, pe);
  }
  if (tid == 0) {
    s_a0 = a_mine;
    s_nmix = 0;
  }
  __syncthreads();
  const int64_t a0 = s_a0;
  if (tid <= cnt) s_a[tid] = (int32_t)(a_mine - a0);
  // The words built here: from the first one holding an entry past the tree
  // prefix (the prefix-only words are the packed prefix row's, left alone)
  // to the last one holding an entry; the slack after it is not touched.
  // Without plain entries to write, the loop below runs over these words
  // only, counted from 0 across the workgroup's paths.
  int32_t nb = 0;
  if (tid < cnt) {
    const SpliceRow& r = s_row[tid];
    const int len = r.lp + r.lq + r.ls;
    const int q0 = tp_vtx ? 0 : r.lp / pe;
    s_q0[tid] = q0;
    nb = (len + pe - 1) / pe - q0;
  }
  const int32_t nb_inc = wave_incl_scan(nb);  // the paths fit in the first wave
  if (tid < cnt) s_c[tid + 1] = nb_inc;
  if (tid == 0) s_c[0] = 0;
  __syncthreads();
  const int32_t nc = s_c[cnt];
  const bool mapped = nc <= kSpliceMap;
  if (mapped && tid < cnt)
    for (int32_t c = s_c[tid]; c < s_c[tid + 1]; ++c) s_map[c] = (uint8_t)tid;
  __syncthreads();
  // the path of built word c
  auto path_of = [&](int32_t c) -> int {
    if (mapped) return s_map[c];
    int lo = 0, hi = cnt - 1;  // the last path whose built words start at or before c
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_c[mid] <= c) lo = mid; else hi = mid - 1;
    }
    return lo;
  };
  // stores word w of path t and keeps it when a key window starts in it
  auto store = [&](int32_t w, int t, int q, uint64_t word) {
    pk[a0 + w] = word;
    const int kq = q - s_kq[t];
    if (kq >= 0 && kq <= kTpKeyTail) s_kw[t][kq] = word;
  };
  // a word across two (or three) parts, entry by entry
  auto build_mixed = [&](int32_t w, int t) {
    const SpliceRow r = s_row[t];
    const int len = r.lp + r.lq + r.ls;
    const int q = w - s_a[t];
    const int k0 = q * pe;
    uint64_t word = 0;
    for (int q0 = 0; q0 < pe; q0 += 8) {  // eight entries at a time, loads in flight together
      int x[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = k0 + q0 + j;
        x[j] = q0 + j < pe && k < len ? splice_entry(r, pp_vtx, b, k) : -1;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = k0 + q0 + j;
        if (q0 + j < pe) {
          uint64_t code = 0;
          if (k < len) {
            if (tp_vtx) tp_vtx[s_w[t] + k] = x[j];
            code = (uint64_t)(x[j] + 1);
          }
          word = (word << EB) | code;
        }
      }
    }
    store(w, t, q, word);
  };
  // Words wholly inside one part take a short path of their own; the words
  // across two parts (about two per test path) would make every wave run
  // the entry-by-entry path as well, so they are listed and built after the
  // others, all lanes then taking that path together.
  for (int32_t c = tid; c < nc; c += kBlock) {
    const int t = path_of(c);
    const SpliceRow r = s_row[t];
    const int q = s_q0[t] + (c - s_c[t]);
    const int32_t w = s_a[t] + q;
    const int k0 = q * pe;
    if (tp_vtx) {
      build_mixed(w, t);  // plain entries asked for: every word entry by entry
      continue;
    }
    uint64_t word = 0;
    if (k0 >= r.lp + r.lq) {
      const int j0 = k0 - r.lp - r.lq;  // first suffix entry of the word
      const int sq = j0 / pe, sr = j0 - sq * pe;
      const uint64_t* row = b.sfx_pk + s_sb[t];
      const uint64_t A = row[sq];
      if (sr == 0) {
        word = A;
      } else {
        // entries sr .. pe-1 of A, then entries 0 .. sr-1 of the next word
        const int hb = (pe - sr) * EB;  // bits of A's entries sr .. pe-1
        const uint64_t B = row[sq + 1];
        word = ((A & ((1ull << hb) - 1)) << (sr * EB)) | (B >> hb);
      }
    } else if (pe <= 16 && k0 >= r.lp && k0 + pe <= r.lp + r.lq) {
      const int32_t* src = pp_vtx + r.o0 + (k0 - r.lp);
      int32_t x[pe <= 16 ? pe : 1];
#pragma unroll
      for (int j = 0; j < (pe <= 16 ? pe : 1); ++j) x[j] = src[j];
#pragma unroll
      for (int j = 0; j < (pe <= 16 ? pe : 1); ++j) word = (word << EB) | (uint64_t)(uint32_t)(x[j] + 1);
    } else {
      const int m = atomicAdd(&s_nmix, 1);
      if (m < kSpliceMixed) s_mix[m] = c;
      else build_mixed(w, t);  // the list is full: build it here
      continue;
    }
    store(w, t, q, word);
  }
  __syncthreads();
  const int nmix = s_nmix < kSpliceMixed ? s_nmix : kSpliceMixed;
  for (int m = tid; m < nmix; m += kBlock) {
    const int32_t c = s_mix[m];
    const int t = path_of(c);
    build_mixed(s_a[t] + s_q0[t] + (c - s_c[t]), t);
  }
  __syncthreads();
  // the key's entry words: windows of pe entries from the first entry after e
  for (int u = tid; u < cnt * kTpKeyTail; u += kBlock) {
    const int t = u / kTpKeyTail, j = u - t * kTpKeyTail;
    const SpliceRow& r = s_row[t];
    const int64_t len = (int64_t)r.lp + r.lq + r.ls - (int64_t)s_kq[t] * pe;  // from word s_kq
    const int64_t k = (int64_t)(s_kf[t] - s_kq[t] * pe) + (int64_t)j * pe;
    key[(int64_t)kTpKeyWords * (i0 + t) + 2 + j] = packed_window(s_kw[t], len, k, pe, EB);
  }
}

// The comparison keys of test path i (see above): where it leaves the BFS
// tree (the first entry after the prime path's first vertex whose tree
// parent is not the entry before it), that tree path's preorder range and
// depth, the entry after it and the split rank, and the next pe entries.
// One thread per test path.
__global__ __launch_bounds__(kBlock) void k_tp_keys(const int64_t* pp_off, const int32_t* pp_vtx,
                                                    int64_t n_pp, BfsOut b, const int4* lead,
                                                    uint64_t* key) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n_pp) {
    // a path that leaves the tree inside its prime path: the prime-path
    // writer has recorded where (entry lp + lead) and the entries w and e
    if (lead) {
      const int4 ld = lead[i];
      if (ld.x < pp_off[i + 1] - pp_off[i]) {
        const int lp = (int)(b.pfx_off[ld.w + 1] - b.pfx_off[ld.w]);
        tp_tree_key(b.pre, b.pend, b.cfirst, b.ccnt, b.bq, ld.y, lp + ld.x, true, ld.z, ld.w,
                    key + (int64_t)kTpKeyWords * i);
        return;
      }
    }
    const SpliceRow r = splice_row(pp_off, pp_vtx, b, i);
    const int len = r.lp + r.lq + r.ls;
    // where the path leaves the BFS tree: entries up to the prime path's
    // first vertex are its tree path; then the prime path's own entries, as
    // far as the prime-path writer found them following the tree (lead), and
    // past those the suffix, scanned eight entries at a time
    int first = len;
    int prev = r.v1;
    int kscan = r.lp + 1;
    if (lead) {  // the whole prime path follows the tree
      prev = r.vk;
      kscan = r.lp + r.lq;
    }
    for (int k0 = kscan; k0 < len && first == len; k0 += 8) {
      int x[8], px[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) x[j] = k0 + j < len ? splice_entry(r, pp_vtx, b, k0 + j) : -1;
#pragma unroll
      for (int j = 0; j < 8; ++j) px[j] = x[j] >= 0 ? b.parent[x[j]] : -1;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (k0 + j < len && first == len) {
          if (px[j] != prev) first = k0 + j;
          prev = x[j];
        }
      }
    }
    const bool has_e = first < len;
    const int w = splice_entry(r, pp_vtx, b, first - 1);
    const int ev = has_e ? splice_entry(r, pp_vtx, b, first) : 0;
    tp_tree_key(b.pre, b.pend, b.cfirst, b.ccnt, b.bq, w, first, has_e, ev, r.v1,
                key + (int64_t)kTpKeyWords * i);
    // the words of entries after e come from k_tp_write, which runs next
  }
}

hipError_t launch_tp_write(const int64_t* pp_off, const int32_t* pp_vtx, int64_t n_pp,
                           const BfsOut& b, const int64_t* tp_off, int32_t* tp_vtx,
                           uint64_t* key, uint64_t* pk, int eb, int32_t* idx,
                           const int4* lead, hipStream_t st) {
  if (n_pp == 0) return hipSuccess;
  if (eb < 1 || eb > 18) return hipErrorInvalidValue;  // more than 2^18 - 1 vertices in one union
  // the tree-position keys first: the splice cuts the entry words after e
  k_tp_keys<<<(unsigned)((n_pp + kBlock - 1) / kBlock), kBlock, 0, st>>>(pp_off, pp_vtx, n_pp, b,
                                                                        lead, key);
  const unsigned grid = (unsigned)((n_pp + kSplicePaths - 1) / kSplicePaths);
#define TPG_SPLICE_CASE(E)                                                                     \
  case E:                                                                                      \
    k_tp_write<E><<<grid, kBlock, 0, st>>>(pp_off, pp_vtx, n_pp, b, tp_off, tp_vtx, pk, key, idx); \
    break;
  switch (eb) {
    TPG_SPLICE_CASE(1) TPG_SPLICE_CASE(2) TPG_SPLICE_CASE(3) TPG_SPLICE_CASE(4)
    TPG_SPLICE_CASE(5) TPG_SPLICE_CASE(6) TPG_SPLICE_CASE(7) TPG_SPLICE_CASE(8)
    TPG_SPLICE_CASE(9) TPG_SPLICE_CASE(10) TPG_SPLICE_CASE(11) TPG_SPLICE_CASE(12)
    TPG_SPLICE_CASE(13) TPG_SPLICE_CASE(14) TPG_SPLICE_CASE(15) TPG_SPLICE_CASE(16)
    TPG_SPLICE_CASE(17) TPG_SPLICE_CASE(18)
    default:
      return hipErrorInvalidValue;
  }
#undef TPG_SPLICE_CASE
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// sort + dedup
// ---------------------------------------------------------------------------
// Entries k0.. of two test paths whose entries before k0 agree, compared
// lexicographically (then by length) on their packed copies: 2 P words per
// step, P aligned 16-byte loads per path.  P = 2 by default; the split
// search, which moves few bytes and waits on each step, takes 4.
template <int P = 2>
__device__ __forceinline__ int tp_cmp_tail(const TpOrder& K, int64_t x, int64_t y, int64_t k0) {
  const int64_t ox = K.off[x], oy = K.off[y];
  const int64_t lx = K.off[x + 1] - ox, ly = K.off[y + 1] - oy;
  const int pe = K.pe;
  const int64_t nw = ((lx < ly ? lx : ly) + pe - 1) / pe;  // words holding entries of both
  const uint64_t* px = K.pk + tp_pk_base(ox, x, pe);
  const uint64_t* py = K.pk + tp_pk_base(oy, y, pe);
  for (int64_t q = (k0 / pe) & ~(int64_t)1; q < nw; q += 2 * P) {
    uint64_t a[2 * P], c[2 * P];
#pragma unroll
    for (int i = 0; i < 2 * P; ++i) a[i] = c[i] = 0;
#pragma unroll
    for (int h = 0; h < P; ++h) {
      if (q + 2 * h < nw) {
        const ulonglong2 u = *reinterpret_cast<const ulonglong2*>(px + q + 2 * h);
        const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(py + q + 2 * h);
        a[2 * h] = u.x;
        c[2 * h] = v.x;
        if (q + 2 * h + 1 < nw) {
          a[2 * h + 1] = u.y;
          c[2 * h + 1] = v.y;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 2 * P; ++i)
      if (a[i] != c[i]) return a[i] < c[i] ? -1 : 1;
  }
  return lx < ly ? -1 : (lx > ly ? 1 : 0);
}

// Lexicographic comparison of test paths x and y from their keys (kx(i),
// ky(i): key word i; word 0 holds pre(w), pend(w) and the prefix depth, word
// 1 the entry e, split and the prime path's first vertex, words 2.. the
// entries after e):
//  * same prime-path first vertex: the order of the prime paths (indices);
//  * same tree prefix w: no e sorts first (equal when both end there), then
//    e decides, then the entries after e: the ones packed in the keys, then,
//    when those tie and neither path ended inside them, the rest read from
//    memory;
//  * w_x a proper ancestor of w_y: t_y continues with the tree child c of
//    w_x towards w_y, t_x with e_x (not a tree child), and e_x < c exactly
//    when pre(w_y) < split_x; symmetric the other way round;
//  * otherwise the tree prefixes differ first and preorder decides.
template <int P = 2, class KX, class KY>
__device__ __forceinline__ int tp_cmp_keys(const TpOrder& K, int64_t x, KX kx, int64_t y, KY ky) {
  if (x == y) return 0;
  const uint64_t ax = kx(0), ay = ky(0), bx = kx(1), by = ky(1);
  if ((bx >> 35) == (by >> 35)) return x < y ? -1 : 1;
  const uint32_t pwx = (uint32_t)(ax & kM18), pwy = (uint32_t)(ay & kM18);
  if (pwx == pwy) {
    const bool hx = (ax >> 49) & 1, hy = (ay >> 49) & 1;
    if (!hx || !hy) return hx == hy ? 0 : (hx ? 1 : -1);
    const uint32_t ex = (uint32_t)(bx & kM17), ey = (uint32_t)(by & kM17);
    if (ex != ey) return ex < ey ? -1 : 1;
#pragma unroll
    for (int t = 0; t < kTpKeyTail; ++t) {
      const uint64_t cx = kx(2 + t), cy = ky(2 + t);
      if (cx != cy) return cx < cy ? -1 : 1;
      if ((cx & ((1ull << K.eb) - 1)) == 0) return 0;  // both ended inside this word
    }
    return tp_cmp_tail<P>(K, x, y, (int64_t)((ax >> 36) & kM13) + 2 + (int64_t)kTpKeyTail * K.pe);
  }
  const uint32_t pex = (uint32_t)((ax >> 18) & kM18), pey = (uint32_t)((ay >> 18) & kM18);
  if (pwx < pwy && pwy < pex) return pwy >= (uint32_t)((bx >> 17) & kM18) ? -1 : 1;
  if (pwy < pwx && pwx < pey) return pwx >= (uint32_t)((by >> 17) & kM18) ? 1 : -1;
  return pwx < pwy ? -1 : 1;
}

// The same, reading the keys from memory (x, y: test-path indices).
template <int P = 2>
__device__ __forceinline__ int tp_cmp(const TpOrder& K, int64_t x, int64_t y) {
  if (x == y) return 0;
  const uint64_t* kx = K.key + (int64_t)kTpKeyWords * x;
  const uint64_t* ky = K.key + (int64_t)kTpKeyWords * y;
  return tp_cmp_keys<P>(K, x, [kx](int i) { return kx[i]; }, y, [ky](int i) { return ky[i]; });
}

// Merge path: number of elements taken from A among the first d outputs of
// merge(A, B) (stable: A first on ties).  A, B: test-path indices (global).
// Found by one whole wave: each step its 64 lanes test 64 evenly spaced
// candidates at once and the interval shrinks 64-fold, so a search costs
// ~log_64(n) comparison latencies instead of log_2(n).  This matters where
// the candidates share a long tree prefix and next entry, because then every
// comparison reads the paths' entries (dependent global loads).
__device__ __forceinline__ int64_t merge_split_wave(const TpOrder& K, const int32_t* A, int64_t na,
                                                    const int32_t* B, int64_t nb, int64_t d) {
  const int lane = lane_id();
  int64_t lo = d - nb > 0 ? d - nb : 0, hi = d < na ? d : na;  // answer in [lo, hi]
  while (lo < hi) {
    const int64_t span = hi - lo;
    const int64_t step = (span + 63) / 64;
    const int64_t c = lo + (int64_t)lane * step;  // candidate tested by this lane
    // P(c): the merge takes A[c] before B[d - 1 - c]; true then false along c
    const bool p = c < hi && tp_cmp<4>(K, B[d - 1 - c], A[c]) >= 0;
    const uint64_t t = __ballot(p);
    if (t == 0) {
      hi = lo;  // P(lo) is false: the split is lo
    } else {
      const int k = 63 - __builtin_clzll(t);  // last lane with P true
      const int64_t ck = lo + (int64_t)k * step;
      lo = ck + 1;
      const int64_t nxt = ck + step;
      hi = nxt < hi ? nxt : hi;
    }
  }
  return lo;
}

// One round of pairwise merges of the sorted runs [rb[r], rb[r + 1]): run
// 2p with run 2p + 1.  A workgroup produces kMergeTile consecutive outputs.
// Where its input slices start is found beforehand, by k_merge_splits (one
// merge-path search per tile, a whole wave each, at full occupancy: the
// searches are chains of dependent loads); the workgroup stages the slices'
// indices and keys in LDS and every thread then splits and merges its own
// kMergeItems outputs from LDS (the entries themselves are read only when
// two paths share their tree prefix, next entry and the entries the keys
// hold).  A thread's split costs a binary search over the tile, so several
// outputs per thread mean fewer comparisons per output.
constexpr int kMergeThreads = 256;
constexpr int kMergeItems = 4;
constexpr int kMergeTile = kMergeThreads * kMergeItems;
static_assert(kTpKeyWords % 2 == 0, "keys are loaded 16 bytes at a time");
constexpr int kSplitWaves = 4;  // splits found per workgroup of k_merge_splits

// Pair p of runs: [a0, a1) with [a1, b1).
__device__ __forceinline__ void merge_pair_bounds(const int64_t* rb, int64_t n_runs, int64_t p,
                                                  int64_t& a0, int64_t& a1, int64_t& b1) {
  a0 = rb[2 * p];
  a1 = rb[2 * p + 1 < n_runs ? 2 * p + 1 : n_runs];
  b1 = rb[2 * p + 2 < n_runs ? 2 * p + 2 : n_runs];
}
// The pair of runs holding output position pos, found by a whole wave: each
// step its lanes test 64 evenly spaced run starts at once.
__device__ __forceinline__ int64_t merge_pair_of_wave(const int64_t* rb, int64_t n_runs,
                                                      int64_t pos) {
  int64_t lo = 0, hi = n_runs - 1;  // the last run starting at or before pos is in [lo, hi]
  while (lo < hi) {
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t c = lo + 1 + (int64_t)lane_id() * step;  // candidates lo + 1 .. hi
    const uint64_t t = __ballot(c <= hi && rb[c] <= pos);
    if (t == 0) {
      hi = lo;
    } else {
      const int64_t ck = lo + 1 + (int64_t)(63 - __builtin_clzll(t)) * step;
      lo = ck;
      hi = ck + step - 1 < hi ? ck + step - 1 : hi;
    }
  }
  return lo >> 1;
}

// For tile b (its first output at b * kMergeTile): split[b], how many of the
// first (b * kMergeTile - a0) outputs of its pair's merge come from the
// pair's first run, and split[n_tiles + 1 + b], the pair's index times two,
// plus one when the pair is already in order (its first run's last path does
// not come after the second run's first, or a run is empty).  The merge of
// such a pair is its input as it stands, and the split needs no search.
__global__ __launch_bounds__(64 * kSplitWaves) void k_merge_splits(TpOrder K, const int32_t* in,
                                                                  const int64_t* rb, int64_t n_runs,
                                                                  int64_t n_tiles, int64_t* split) {
  const int64_t b = (int64_t)blockIdx.x * kSplitWaves + (threadIdx.x >> 6);
  if (b >= n_tiles) return;  // whole waves
  const int64_t pos = b * kMergeTile;
  const int64_t p = merge_pair_of_wave(rb, n_runs, pos);
  int64_t a0, a1, b1;
  merge_pair_bounds(rb, n_runs, p, a0, a1, b1);
  const bool ordered = a1 == a0 || b1 == a1 || tp_cmp<4>(K, in[a1 - 1], in[a1]) <= 0;
  const int64_t d = pos - a0;
  const int64_t r = ordered ? (d < a1 - a0 ? d : a1 - a0)
                            : merge_split_wave(K, in + a0, a1 - a0, in + a1, b1 - a1, d);
  if (lane_id() == 0) {
    split[b] = r;
    split[n_tiles + 1 + b] = 2 * p + (ordered ? 1 : 0);
  }
}

__global__ __launch_bounds__(kMergeThreads) void k_merge_round(TpOrder K, const int32_t* in,
                                                               int32_t* out, const int64_t* rb,
                                                               int64_t n_runs, int64_t n,
                                                               const int64_t* split) {
  __shared__ int32_t s_idx[kMergeTile];
  __shared__ uint64_t s_key[kTpKeyWords][kMergeTile];
  const int tid = (int)threadIdx.x;
  const int64_t t0 = (int64_t)blockIdx.x * kMergeTile;
  const int64_t t1 = t0 + kMergeTile < n ? t0 + kMergeTile : n;
  int64_t pos = t0;
  // the tile's first pair as k_merge_splits found it; each later segment
  // starts the next pair (an empty pair ends where it starts and is stepped
  // over)
  const int64_t n_tiles = (n + kMergeTile - 1) / kMergeTile;
  const int64_t pv = split[n_tiles + 1 + blockIdx.x];
  int64_t p = pv >> 1;
  while (pos < t1) {
    int64_t a0, a1, b1;
    merge_pair_bounds(rb, n_runs, p, a0, a1, b1);
    ++p;
    if (b1 <= pos) continue;
    const int32_t* A = in + a0;
    const int32_t* B = in + a1;
    const int64_t na = a1 - a0;
    const int64_t stop = t1 < b1 ? t1 : b1;
    if (pos == t0 && (pv & 1)) {
      // the first pair (it holds t0) is in order: output q is input q
      for (int64_t q = pos + tid; q < stop; q += kMergeThreads) out[q] = in[q];
      pos = stop;
      continue;
    }
    // input slices of this segment: the tile's first segment starts at its
    // split, a later one at the start of its pair; a segment ends at the end
    // of its pair or at the next tile's split
    const int64_t ia = pos == t0 ? split[blockIdx.x] : 0, ja = (pos - a0) - ia;
    const int64_t ib = stop == b1 ? na : split[blockIdx.x + 1], jb = (stop - a0) - ib;
    const int la = (int)(ib - ia), lb = (int)(jb - ja);
    // A segment has at most kMergeTile inputs: kMergeItems per thread.  All
    // of a thread's index loads go out together, then all its key loads (a
    // key is kTpKeyWords words at a 16-byte aligned address), so the staging
    // waits for two load latencies, not two per input.
    {
      int32_t xs[kMergeItems];
#pragma unroll
      for (int u = 0; u < kMergeItems; ++u) {
        const int q = tid + u * kMergeThreads;
        xs[u] = q < la ? A[ia + q] : (q < la + lb ? B[ja + (q - la)] : -1);
      }
      ulonglong2 kv[kMergeItems][kTpKeyWords / 2];
#pragma unroll
      for (int u = 0; u < kMergeItems; ++u) {
        if (xs[u] < 0) continue;
        const ulonglong2* kx =
            reinterpret_cast<const ulonglong2*>(K.key + (int64_t)kTpKeyWords * xs[u]);
#pragma unroll
        for (int h = 0; h < kTpKeyWords / 2; ++h) kv[u][h] = kx[h];
      }
#pragma unroll
      for (int u = 0; u < kMergeItems; ++u) {
        if (xs[u] < 0) continue;
        const int q = tid + u * kMergeThreads;
        s_idx[q] = xs[u];
#pragma unroll
        for (int h = 0; h < kTpKeyWords / 2; ++h) {
          s_key[2 * h][q] = kv[u][h].x;
          s_key[2 * h + 1][q] = kv[u][h].y;
        }
      }
    }
    __syncthreads();
    // this thread's outputs within the segment, merged from LDS
    const int m = la + lb;
    const int d0 = tid * kMergeItems < m ? tid * kMergeItems : m;
    const int d1 = d0 + kMergeItems < m ? d0 + kMergeItems : m;
    if (d0 < d1) {
      int l2 = d0 - lb > 0 ? d0 - lb : 0, h2 = d0 < la ? d0 : la;
      while (l2 < h2) {
        const int mid = (l2 + h2) >> 1;
        const int qb = la + (d0 - 1 - mid);
        if (tp_cmp_keys(K, s_idx[qb], [&](int t) { return s_key[t][qb]; }, s_idx[mid],
                        [&](int t) { return s_key[t][mid]; }) >= 0)
          l2 = mid + 1;
        else
          h2 = mid;
      }
      int i = l2, j = d0 - l2;
      for (int o = d0; o < d1; ++o) {
        bool take_a;
        if (j >= lb) take_a = true;
        else if (i >= la) take_a = false;
        else {
          const int qb = la + j;
          take_a = tp_cmp_keys(K, s_idx[qb], [&](int t) { return s_key[t][qb]; }, s_idx[i],
                               [&](int t) { return s_key[t][i]; }) >= 0;
        }
        out[pos + o] = take_a ? s_idx[i++] : s_idx[la + j++];
      }
    }
    __syncthreads();
    pos = stop;
  }
}

int64_t merge_split_slots(int64_t n) { return 2 * ((n + kMergeTile - 1) / kMergeTile + 1); }

hipError_t launch_merge_round(const TpOrder& K, const int32_t* idx_in, int32_t* idx_out,
                              const int64_t* rb, int64_t n_runs, int64_t n, int64_t* split,
                              hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t n_tiles = (n + kMergeTile - 1) / kMergeTile;
  k_merge_splits<<<(unsigned)((n_tiles + kSplitWaves - 1) / kSplitWaves), 64 * kSplitWaves, 0,
                   st>>>(K, idx_in, rb, n_runs, n_tiles, split);
  k_merge_round<<<(unsigned)n_tiles, kMergeThreads, 0, st>>>(K, idx_in, idx_out, rb, n_runs, n,
                                                             split);
  return hipGetLastError();
}

// Runs of a union of graphs, each graph's runs padded to 2^R with empty
// ones: out[s] for s = c * 2^R + j (j < 2^R) is the start of graph c's j-th
// run (its end once j reaches its run count), out[n_comp * 2^R] the end.
// Pairing runs 2p, 2p + 1 then never crosses two graphs, so R rounds sort
// every graph's test paths, and the graphs already follow each other in
// order (their ids are disjoint ranges).
__global__ void k_pad_runs(DGraph g, const int64_t* rb, int R, int64_t n_out, int64_t* out) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s > n_out) return;
  const int64_t c = s >> R;
  if (c >= g.n_comp) {
    out[s] = rb[g.n];
    return;
  }
  const int64_t j = s & ((1ll << R) - 1);
  const int64_t nc = g.cbase[c + 1] - g.cbase[c];
  out[s] = rb[g.cbase[c] + (j < nc ? j : nc)];
}

hipError_t launch_pad_runs(const DGraph& g, const int64_t* rb, int R, int64_t n_out, int64_t* out,
                           hipStream_t st) {
  k_pad_runs<<<(unsigned)((n_out + 1 + kBlock - 1) / kBlock), kBlock, 0, st>>>(g, rb, R, n_out, out);
  return hipGetLastError();
}

__global__ void k_next_runs(const int64_t* rb, int64_t n_runs, int64_t* rb_out) {
  const int64_t h = (n_runs + 1) / 2;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < h) rb_out[p] = rb[2 * p];
  if (p == h) rb_out[h] = rb[n_runs];
}

hipError_t launch_next_runs(const int64_t* rb, int64_t n_runs, int64_t* rb_out, hipStream_t st) {
  const int64_t h = (n_runs + 1) / 2;
  k_next_runs<<<(unsigned)((h + 1 + kBlock - 1) / kBlock), kBlock, 0, st>>>(rb, n_runs, rb_out);
  return hipGetLastError();
}

// keep_cnt[k] = 1 unless sorted position k holds the same test path as k - 1;
// keep_len[k] = its length when kept, else 0.  A workgroup stages the keys
// of positions k0 - 1 .. k0 + kBlock - 1 in LDS, each key loaded once and
// whole (16 bytes at a time), then each thread compares its position with
// the one before.
__global__ __launch_bounds__(kBlock) void k_dedup_flags(TpOrder K, const int32_t* idx, int64_t n,
                                                        int64_t* keep_cnt, int64_t* keep_len) {
  __shared__ uint64_t s_key[kTpKeyWords][kBlock + 1];
  __shared__ int32_t s_idx[kBlock + 1];
  const int tid = (int)threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.x * kBlock;
  for (int q = tid; q <= kBlock; q += kBlock) {  // slot q: position k0 - 1 + q
    const int64_t k = k0 - 1 + q;
    if (k >= 0 && k < n) {
      const int32_t x = idx[k];
      s_idx[q] = x;
      const ulonglong2* kx = reinterpret_cast<const ulonglong2*>(K.key + (int64_t)kTpKeyWords * x);
      ulonglong2 w[kTpKeyWords / 2];
#pragma unroll
      for (int h = 0; h < kTpKeyWords / 2; ++h) w[h] = kx[h];
#pragma unroll
      for (int h = 0; h < kTpKeyWords / 2; ++h) {
        s_key[2 * h][q] = w[h].x;
        s_key[2 * h + 1][q] = w[h].y;
      }
    }
  }
  __syncthreads();
  const int64_t k = k0 + tid;
  if (k >= n) return;
  const int q = tid + 1;
  const int64_t a = s_idx[q];
  const bool keep = k == 0 || tp_cmp_keys(K, (int64_t)s_idx[q - 1],
                                          [&](int t) { return s_key[t][q - 1]; }, a,
                                          [&](int t) { return s_key[t][q]; }) != 0;
  keep_cnt[k] = keep ? 1 : 0;
  keep_len[k] = keep ? K.off[a + 1] - K.off[a] : 0;
}

hipError_t launch_dedup_flags(const TpOrder& K, const int32_t* idx, int64_t n, int64_t* keep_cnt,
                              int64_t* keep_len, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_dedup_flags<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(K, idx, n, keep_cnt,
                                                                          keep_len);
  return hipGetLastError();
}

// A workgroup copies the kept paths among kSplicePaths consecutive sorted
// positions: their sources, destinations and lengths go to LDS, then the
// threads copy the entries as one flat range (kept paths are contiguous in
// the output).
__global__ __launch_bounds__(kBlock) void k_gather(const int64_t* off, const int32_t* vtx,
                                                   const int32_t* idx, int64_t n,
                                                   const int64_t* keep_pos,
                                                   const int64_t* keep_voff,
                                                   const int64_t* keep_len, int64_t* out_off,
                                                   int32_t* out_vtx) {
  __shared__ int64_t s_src[kSplicePaths];
  __shared__ int64_t s_cum[kSplicePaths + 1];
  __shared__ int64_t s_dst0;
  __shared__ int32_t s_w[kBlock / 64];
  const int tid = (int)threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.x * kSplicePaths;
  const int cnt = (int)(n - k0 < kSplicePaths ? n - k0 : kSplicePaths);
  int64_t len = 0;
  if (tid < cnt) {
    const int64_t k = k0 + tid;
    len = keep_len[k];  // 0 for a duplicate (every kept path has >= 1 entry)
    if (len) {
      const int64_t a = idx[k];
      s_src[tid] = off[a];
      out_off[keep_pos[k]] = keep_voff[k];
    }
  }
  if (tid == 0) s_dst0 = keep_voff[k0];
  int32_t tot;
  const int32_t ex = block_excl_scan<kBlock, int32_t>((int32_t)len, tot, s_w);
  if (tid < cnt) s_cum[tid] = ex;
  if (tid == 0) s_cum[cnt] = tot;
  __syncthreads();
  const int64_t d0 = s_dst0;
  for (int64_t e = tid; e < tot; e += kBlock) {
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_cum[mid] <= e) lo = mid; else hi = mid - 1;
    }
    out_vtx[d0 + e] = vtx[s_src[lo] + (e - s_cum[lo])];
  }
}

hipError_t launch_gather(const int64_t* tp_off, const int32_t* tp_vtx, const int32_t* idx,
                         int64_t n, const int64_t* keep_pos, const int64_t* keep_voff,
                         const int64_t* keep_len, int64_t* out_off, int32_t* out_vtx,
                         hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_gather<<<(unsigned)((n + kSplicePaths - 1) / kSplicePaths), kBlock, 0, st>>>(
      tp_off, tp_vtx, idx, n, keep_pos, keep_voff, keep_len, out_off, out_vtx);
  return hipGetLastError();
}

// A workgroup writes the kept paths among kGatherPaths consecutive sorted
// positions from their packed words.  The kept paths are contiguous in the
// output, so the workgroup's output is one range [d0, d0 + tot) and the
// paths' packed words form one flat list.  The list is taken a window of
// words at a time: each thread decodes whole words into an LDS copy of the
// window's entries (the word's path from a map of the workgroup's words to
// paths built in LDS, or a search over the paths when the list is longer
// than the map; with the entry width a compile-time constant every entry is
// a shift and a mask), then the window's entries go out as aligned 16-byte
// stores, so a wave writes 1 KiB of consecutive addresses per instruction.
// The aligned groups at the two ends of a window are shared with the
// neighbouring windows (or workgroups); there only the entries inside the
// window are stored, one by one.  A thread loads its words of the next
// window into registers before the current window's stores, so that their
// latency overlaps those.
constexpr int kGatherPaths = 64;
constexpr int kUnpackMap = 4096;  // words a workgroup maps to paths in LDS
constexpr int kUnpackWin = 4096;  // entries of one window in LDS

template <int EB>
__global__ __launch_bounds__(kBlock) void k_unpack_gather(const int64_t* tp_off, const uint64_t* pk,
                                                          const int64_t* pp_off,
                                                          const int32_t* pp_vtx, BfsOut b,
                                                          const int32_t* idx, int64_t n,
                                                          const int64_t* keep_pos,
                                                          const int64_t* keep_voff,
                                                          const int64_t* keep_len,
                                                          int64_t* out_off, int32_t* out_vtx) {
  constexpr int pe = 64 / EB;  // a compile-time divisor: no division per entry
  constexpr uint64_t emask = (1ull << EB) - 1;
  constexpr int kWinWords = kUnpackWin / pe;
  constexpr int kWinIter = (kWinWords + kBlock - 1) / kBlock;  // a thread's words per window
  __shared__ int64_t s_src[kGatherPaths];
  __shared__ int64_t s_pfx[kGatherPaths];      // first word of the path's packed prefix row
  __shared__ int32_t s_lpw[kGatherPaths];      // its words that hold prefix entries only
  __shared__ int32_t s_cum[kGatherPaths + 1];  // entries before each kept path
  __shared__ int32_t s_wc[kGatherPaths + 1];   // packed words before each kept path
  __shared__ uint8_t s_map[kUnpackMap];        // word -> path
  __shared__ int32_t s_e[kUnpackWin];          // the window's entries
  __shared__ int64_t s_dst0;
  __shared__ int32_t s_w[kBlock / 64];
  const int tid = (int)threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.x * kGatherPaths;
  const int cnt = (int)(n - k0 < kGatherPaths ? n - k0 : kGatherPaths);
  int32_t len = 0;
  if (tid < cnt) {
    const int64_t k = k0 + tid;
    len = (int32_t)keep_len[k];  // 0 for a duplicate (every kept path has >= 1 entry)
    s_src[tid] = 0;
    s_pfx[tid] = 0;
    s_lpw[tid] = 0;
    if (len) {
      const int64_t a = idx[k];
      s_src[tid] = tp_pk_base(tp_off[a], a, pe);
      // test path a was spliced from prime path a: its prefix is the packed
      // prefix row of that path's first vertex
      const int v1 = pp_vtx[pp_off[a]];
      const int64_t p0 = b.pfx_off[v1];
      s_pfx[tid] = tbl_pk_base(p0, v1, pe);
      s_lpw[tid] = (int32_t)((b.pfx_off[v1 + 1] - p0) / pe);
      out_off[keep_pos[k]] = keep_voff[k];
    }
  }
  if (tid == 0) s_dst0 = keep_voff[k0];
  int32_t tot, nw_tot;
  const int32_t ex = block_excl_scan<kBlock, int32_t>(len, tot, s_w);
  const int32_t nw = (len + pe - 1) / pe;
  const int32_t wx = block_excl_scan<kBlock, int32_t>(nw, nw_tot, s_w);
  if (tid < cnt) {
    s_cum[tid] = ex;
    s_wc[tid] = wx;
  }
  if (tid == 0) {
    s_cum[cnt] = tot;
    s_wc[cnt] = nw_tot;
  }
  const bool mapped = nw_tot <= kUnpackMap;
  if (mapped && tid < cnt)
    for (int32_t w = 0; w < nw; ++w) s_map[wx + w] = (uint8_t)tid;
  __syncthreads();
  if (tot == 0) return;
  const int64_t d0 = s_dst0;
  // the path of word w (w < nw_tot), and the first entry of word w
  auto path_of = [&](int32_t w) -> int {
    if (mapped) return s_map[w];
    int lo = 0, hi = cnt - 1;  // the last path whose words start at or before w
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_wc[mid] <= w) lo = mid; else hi = mid - 1;
    }
    return lo;
  };
  auto entry_of = [&](int32_t w) -> int32_t {
    if (w >= nw_tot) return tot;
    const int t = path_of(w);
    return s_cum[t] + (w - s_wc[t]) * pe;
  };
  // a thread's words of the window starting at word w0: w0 + tid + u kBlock
  auto load_words = [&](int32_t w0, uint64_t (&wd)[kWinIter]) {
    const int32_t w1 = w0 + kWinWords < nw_tot ? w0 + kWinWords : nw_tot;
#pragma unroll
    for (int u = 0; u < kWinIter; ++u) {
      const int32_t w = w0 + tid + u * kBlock;
      wd[u] = 0;
      if (w < w1) {
        const int t = path_of(w);
        const int32_t qw = w - s_wc[t];
        wd[u] = qw < s_lpw[t] ? b.pfx_pk[s_pfx[t] + qw] : pk[s_src[t] + qw];
      }
    }
  };
  uint64_t cur[kWinIter];
  load_words(0, cur);
  for (int32_t w0 = 0; w0 < nw_tot; w0 += kWinWords) {
    const int32_t w1 = w0 + kWinWords < nw_tot ? w0 + kWinWords : nw_tot;
    const int32_t e_a = entry_of(w0), e_b = entry_of(w1);
#pragma unroll
    for (int u = 0; u < kWinIter; ++u) {
      const int32_t w = w0 + tid + u * kBlock;
      if (w < w1) {
        const int t = path_of(w);
        const int32_t qw = w - s_wc[t];
        const uint64_t word = cur[u];
        const int32_t e0 = s_cum[t] + qw * pe;
        const int32_t ne = s_cum[t + 1] - e0;  // entries of the path from this word on
#pragma unroll
        for (int j = 0; j < pe; ++j)
          if (j < ne) s_e[e0 - e_a + j] = (int32_t)((word >> ((pe - 1 - j) * EB)) & emask) - 1;
      }
    }
    __syncthreads();
    // the next window's words are loaded while this window's entries leave
    if (w1 < nw_tot) load_words(w1, cur);
    const int64_t ga = d0 + e_a, gb = d0 + e_b;  // the window's output range
    const int64_t g_first = ga & ~(int64_t)3;
    const int64_t ngroups = (gb - g_first + 3) >> 2;
    for (int64_t gi = tid; gi < ngroups; gi += kBlock) {
      const int64_t g0 = g_first + 4 * gi;
      const int32_t l0 = (int32_t)(g0 - ga);  // LDS position of the group's first entry
      if (g0 >= ga && g0 + 4 <= gb) {
        *reinterpret_cast<int4*>(out_vtx + g0) =
            make_int4(s_e[l0], s_e[l0 + 1], s_e[l0 + 2], s_e[l0 + 3]);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (g0 + j >= ga && g0 + j < gb) out_vtx[g0 + j] = s_e[l0 + j];
      }
    }
    __syncthreads();
  }
}

hipError_t launch_unpack_gather(const int64_t* tp_off, const uint64_t* pk, const int64_t* pp_off,
                                const int32_t* pp_vtx, const BfsOut& b, int eb,
                                const int32_t* idx, int64_t n, const int64_t* keep_pos,
                                const int64_t* keep_voff, const int64_t* keep_len,
                                int64_t* out_off, int32_t* out_vtx, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + kGatherPaths - 1) / kGatherPaths);
#define TPG_UNPACK_CASE(E)                                                                  \
  case E:                                                                                   \
    k_unpack_gather<E><<<grid, kBlock, 0, st>>>(tp_off, pk, pp_off, pp_vtx, b, idx, n,      \
                                                keep_pos, keep_voff, keep_len, out_off,     \
                                                out_vtx);                                   \
    break;
  switch (eb) {
    TPG_UNPACK_CASE(1) TPG_UNPACK_CASE(2) TPG_UNPACK_CASE(3) TPG_UNPACK_CASE(4)
    TPG_UNPACK_CASE(5) TPG_UNPACK_CASE(6) TPG_UNPACK_CASE(7) TPG_UNPACK_CASE(8)
    TPG_UNPACK_CASE(9) TPG_UNPACK_CASE(10) TPG_UNPACK_CASE(11) TPG_UNPACK_CASE(12)
    TPG_UNPACK_CASE(13) TPG_UNPACK_CASE(14) TPG_UNPACK_CASE(15) TPG_UNPACK_CASE(16)
    TPG_UNPACK_CASE(17) TPG_UNPACK_CASE(18)
    default:
      return hipErrorInvalidValue;  // more than 2^18 - 1 vertices in one union
  }
#undef TPG_UNPACK_CASE
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// prime paths grouped by last vertex (the paper's per-end-vertex output)
// ---------------------------------------------------------------------------
// A stable counting sort of the canonical list by last vertex: per tile of
// kGroupTile paths a histogram over the keys, an exclusive scan of the
// histograms taken key-major (so each key's slots run tile after tile),
// then each path's slot = its key's base in its tile + the number of
// earlier paths of the tile with the same key.
__global__ __launch_bounds__(kBlock) void k_last_hist(const int64_t* off, const int32_t* vtx,
                                                      int64_t n, int64_t ntiles, int32_t* key,
                                                      unsigned long long* hist) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t k = vtx[off[i + 1] - 1];
  key[i] = k;
  atomicAdd(&hist[(int64_t)k * ntiles + i / kGroupTile], 1ull);
}

__global__ __launch_bounds__(kGroupTile) void k_last_place(const int32_t* key, int64_t n,
                                                           int64_t ntiles, const int64_t* base,
                                                           int32_t* perm) {
  __shared__ int32_t s_key[kGroupTile];
  const int tid = (int)threadIdx.x;
  const int64_t t = blockIdx.x;
  const int64_t i = t * kGroupTile + tid;
  const int32_t k = i < n ? key[i] : -1;
  s_key[tid] = k;
  __syncthreads();
  if (i >= n) return;
  int r = 0;
  for (int j = 0; j < tid; ++j) r += s_key[j] == k ? 1 : 0;
  perm[base[(int64_t)k * ntiles + t] + r] = (int32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_perm_lens(const int64_t* off, const int32_t* perm,
                                                      int64_t n, int64_t* len, int64_t* pos) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  const int64_t a = perm[k];
  len[k] = off[a + 1] - off[a];
  pos[k] = k;
}

hipError_t launch_last_hist(const int64_t* off, const int32_t* vtx, int64_t n, int64_t ntiles,
                            int32_t* key, uint64_t* hist, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_last_hist<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      off, vtx, n, ntiles, key, reinterpret_cast<unsigned long long*>(hist));
  return hipGetLastError();
}

hipError_t launch_last_place(const int32_t* key, int64_t n, int64_t ntiles, const int64_t* base,
                             int32_t* perm, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_last_place<<<(unsigned)ntiles, kGroupTile, 0, st>>>(key, n, ntiles, base, perm);
  return hipGetLastError();
}

hipError_t launch_perm_lens(const int64_t* off, const int32_t* perm, int64_t n, int64_t* len,
                            int64_t* pos, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_perm_lens<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(off, perm, n, len, pos);
  return hipGetLastError();
}

int64_t group_tiles(int64_t n) { return (n + kGroupTile - 1) / kGroupTile; }

// Per-component starts of a sorted path list (components own contiguous
// id ranges, so the list is grouped by the component of the first vertex):
// start[c] = first path of component >= c, vstart[c] = its first entry
// (c = 0..n_comp); off[n] must hold the total.
__global__ void k_comp_bounds(const int64_t* off, const int32_t* vtx, int64_t n, const int32_t* comp,
                              int n_comp, int64_t* start, int64_t* vstart) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int cur = comp[vtx[off[k]]];
  const int prev = k == 0 ? -1 : comp[vtx[off[k - 1]]];
  for (int c = prev + 1; c <= cur; ++c) {
    start[c] = k;
    vstart[c] = off[k];
  }
  if (k == n - 1)
    for (int c = cur + 1; c <= n_comp; ++c) {
      start[c] = n;
      vstart[c] = off[n];
    }
}

hipError_t launch_comp_bounds(const int64_t* off, const int32_t* vtx, int64_t n,
                              const int32_t* comp, int n_comp, int64_t* start, int64_t* vstart,
                              hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_comp_bounds<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(off, vtx, n, comp, n_comp,
                                                                          start, vstart);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batched form: packing in caller order
// ---------------------------------------------------------------------------
// One workgroup per chunk of a union's segments: the chunk's segment is the
// last descriptor whose first chunk is at or before it (a segment with no
// chunks shares its first chunk with the next one, which wins the search).
// Fixed-size chunks keep the largest graphs of a batch from leaving one
// workgroup copying long after the others are done.
__global__ __launch_bounds__(kBlock) void k_pack(const int64_t* src_off, const int32_t* src_vtx,
                                                 const PackDesc* d, int32_t n_desc,
                                                 int64_t* dst_off, int32_t* dst_vtx) {
  const int64_t b = blockIdx.x;
  int lo = 0, hi = n_desc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].chunk0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const PackDesc e = d[lo];
  const int64_t c = b - e.chunk0;
  const int64_t n_oc = (e.n_paths + kPackPaths - 1) / kPackPaths;
  if (c < n_oc) {
    const int64_t j0 = c * kPackPaths, j1 = min(e.n_paths, j0 + kPackPaths);
    const int64_t shift = e.dst_v - e.src_v0;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += kBlock)
      dst_off[e.dst_path + j] = src_off[e.src_path + j] + shift;
  } else {
    const int64_t q0 = (c - n_oc) * kPackVtx, q1 = min(e.n_v, q0 + kPackVtx);
    for (int64_t q = q0 + threadIdx.x; q < q1; q += kBlock)
      dst_vtx[e.dst_v + q] = src_vtx[e.src_v0 + q];
  }
}

hipError_t launch_pack(const int64_t* src_off, const int32_t* src_vtx, const PackDesc* d,
                       int32_t n_desc, int64_t n_chunks, int64_t* dst_off, int32_t* dst_vtx,
                       hipStream_t st) {
  if (n_desc <= 0 || n_chunks <= 0) return hipSuccess;
  if (n_chunks > (int64_t)INT32_MAX) return hipErrorInvalidValue;
  k_pack<<<(unsigned)n_chunks, kBlock, 0, st>>>(src_off, src_vtx, d, n_desc, dst_off, dst_vtx);
  return hipGetLastError();
}

}  // namespace tpg
