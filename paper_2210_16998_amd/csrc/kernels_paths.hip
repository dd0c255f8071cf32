// Path-tree kernels: level-synchronous extension of simple paths, the
// backward-extendability filter, canonical-order ranking and prime-path
// materialization.
//
// What is computed (paper Sec. 5, Update-Vertex and ExtendPath; Def. 1):
//  * level 1 holds one path <v> per vertex (the host initialisation of the
//    paper's algorithm puts each vertex on its own list);
//  * a path p = (v1..vL) that has not closed a cycle is extended by every
//    successor w of vL that is not on p, and by w = v1, which closes a cycle;
//  * a path that gets no extension at all is terminal; a terminal path is a
//    prime path iff it cannot be extended backward, i.e. every predecessor of
//    v1 lies on p (the pruning of paths covered by a longer path ending at the
//    same vertex); every closed cycle is a prime path.
//
// How (the paper's asynchronous thread-per-vertex schedule and its per-vertex
// path tables are not used):
//  * All paths of one level form a frontier of (parent index, vertex) nodes;
//    the children of one parent are contiguous and in ascending successor
//    order, and each node records where its children start and how many
//    there are.
//  * The visited set of a frontier path lives as a bitmask of W 64-bit words
//    (registers while testing, HBM between levels, two levels alive).
//  * One workgroup handles a tile of 256 * ITEMS parents: choice masks over
//    successor slots, a block scan of child counts, then ONE device-scope
//    atomic claim of the tile's slice of the next level, then a
//    load-balanced expansion where consecutive threads write consecutive
//    children, so record and mask stores are coalesced.  No workgroup ever
//    waits for another one; the order of tile slices inside a level is the
//    order in which the claims landed, which ranking does not depend on.
//  * Levels follow each other on the device: the level index, per-level
//    counts and offsets live in device memory and a one-thread kernel after
//    each extension advances them, or raises the overflow flag when the
//    level did not fit; the host then grows the buffers and replays it.
//  * The plain two-pass form (count, scan, host-visible size, fill) keeps
//    children in parent order and serves as the exact reference form.

#include "kernels.h"

namespace tpg {

// ---------------------------------------------------------------------------
// level 1
// ---------------------------------------------------------------------------
__global__ void k_seed(ExtArgs a) {
  const int n = a.g.n;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  LevelState* ls = a.ls;
  // every level's claim counter starts at zero
  for (int64_t k = i; k < kMaxLevels; k += (int64_t)gridDim.x * blockDim.x) {
    ls->count[k] = k == 1 ? n : 0;
    ls->off[k] = 0;
  }
  if (i == 0) {
    ls->level = 1;
    ls->overflow = 0;
    ls->done = 0;
    ls->cur_count = n;
  }
  if (i < n) {
    const int v = (int)i;
    a.t.par[v] = -1;
    a.t.info[v] = make_info(v, a.g.loc[v], 0);
  }
  // masks of level 1 (parity 1): one bit each, at the vertex's local id
  const int W = a.t.mask_words;
  for (int64_t k = i; k < (int64_t)n * W; k += (int64_t)gridDim.x * blockDim.x) {
    const int v = (int)(k / W), q = (int)(k % W);
    const int l = a.g.loc[v];
    a.t.mask[1][k] = (q == (l >> 6)) ? (1ull << (l & 63)) : 0ull;
  }
}

hipError_t launch_seed(const ExtArgs& a, hipStream_t st) {
  const int64_t work = std::max<int64_t>(kMaxLevels, (int64_t)a.g.n * a.t.mask_words);
  const int grid = (int)std::min<int64_t>(1024, (work + kBlock - 1) / kBlock + 1);
  k_seed<<<grid, kBlock, 0, st>>>(a);
  return hipGetLastError();
}

// Resume after an overflow: the level is extended again from a zero claim.
__global__ void k_resume_fix(ExtArgs a, int level) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.ls->count[level + 1] = 0;
    a.ls->overflow = 0;
    a.ls->done = 0;
  }
}

hipError_t launch_resume_fix(const ExtArgs& a, int level, hipStream_t st) {
  if (level < 1 || level + 1 >= kMaxLevels) return hipErrorInvalidValue;
  k_resume_fix<<<1, 64, 0, st>>>(a, level);
  return hipGetLastError();
}

// Level advance after an extension launch: the claimed total is the next
// level's size; a level that does not fit raises the overflow flag instead
// (the extension kernel stored nothing beyond the capacities).
__global__ void k_advance(ExtArgs a) {
  if (threadIdx.x != 0) return;
  LevelState* ls = a.ls;
  if (ls->overflow) return;
  const int L = ls->level;
  const int64_t F = ls->count[L];
  if (F == 0 || L + 2 >= kMaxLevels) return;
  const int64_t total = ls->count[L + 1];
  const int64_t nbase = ls->off[L] + F;
  if (nbase + total + 1 > a.t.rec_cap || total > a.t.mask_cap ||
      nbase + total >= (int64_t)INT32_MAX) {
    ls->overflow = 1;
    return;
  }
  ls->off[L + 1] = nbase;
  ls->cur_count = total;
  ls->level = L + 1;
}

hipError_t launch_advance(const ExtArgs& a, hipStream_t st) {
  k_advance<<<1, 64, 0, st>>>(a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// shared per-parent step: choice mask over successor slots + terminal filter
// ---------------------------------------------------------------------------
// Choice mask over the successor slots of the path's last vertex v: slot k
// is set when successor w is not on the path, or is its first vertex (closes
// a cycle).  base = graph-wide id of local id 0 of v's component.
template <int W>
__device__ __forceinline__ uint64_t choices(const DGraph& g, uint32_t inf, const uint64_t (&m)[W],
                                            int& k0, int& base) {
  const int v = node_v(inf), v1l = node_v1l(inf);
  base = v - g.loc[v];
  k0 = g.sp[v];
  const int k1 = g.sp[v + 1];
  uint64_t vm = 0;
  for (int k = k0; k < k1; ++k) {
    const int wl = g.s[k] - base;
    const bool ok = (wl == v1l) || !mask_has<W>(m, wl);
    vm |= ok ? (1ull << (k - k0)) : 0ull;
  }
  return vm;
}

// Backward-extendability test of a terminal path: prime iff every
// predecessor of its first vertex is on it.
template <int W>
__device__ __forceinline__ bool all_preds_on(const DGraph& g, int base, int v1l,
                                             const uint64_t (&m)[W]) {
  const int v1 = base + v1l;
  for (int k = g.pp[v1]; k < g.pp[v1 + 1]; ++k)
    if (!mask_has<W>(m, g.p[k] - base)) return false;
  return true;
}

template <int W>
__device__ __forceinline__ void load_mask(const uint64_t* src, uint64_t (&m)[W]) {
  if constexpr (W == 1) {
    m[0] = src[0];
  } else {
    const ulonglong2* s2 = reinterpret_cast<const ulonglong2*>(src);
#pragma unroll
    for (int k = 0; k < W / 2; ++k) {
      const ulonglong2 x = s2[k];
      m[2 * k] = x.x;
      m[2 * k + 1] = x.y;
    }
  }
}

template <int W>
__device__ __forceinline__ void store_child_mask(uint64_t* dst, const uint64_t (&m)[W], int w) {
  const int q = w >> 6;
  const uint64_t bit = 1ull << (w & 63);
  if constexpr (W == 1) {
    dst[0] = m[0] | bit;
  } else {
    ulonglong2* d2 = reinterpret_cast<ulonglong2*>(dst);
#pragma unroll
    for (int k = 0; k < W / 2; ++k) {
      ulonglong2 x;
      x.x = m[2 * k] | ((2 * k == q) ? bit : 0ull);
      x.y = m[2 * k + 1] | ((2 * k + 1 == q) ? bit : 0ull);
      d2[k] = x;
    }
  }
}

// ---------------------------------------------------------------------------
// one-pass extension of level L -> L+1 (device-sized, claim per tile)
// ---------------------------------------------------------------------------
// A tile is ITEMS * 256 consecutive parents; tile t goes to workgroup
// t mod grid.  Loads are strided by the workgroup size (coalesced); the scan
// gives each thread ITEMS consecutive parents; the expansion gives each
// thread every 256th child of the tile.
template <int W, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_extend(ExtArgs a) {
  constexpr int TILE = kBlock * ITEMS;
  constexpr bool kLdsMask = W * ITEMS <= 16;  // visited sets of the tile in LDS (<= 32 KiB)
  __shared__ int64_t s_prefix;
  __shared__ int32_t s_off[TILE];
  __shared__ uint64_t s_vm[TILE];
  __shared__ uint32_t s_inf[TILE];
  __shared__ uint64_t s_mask[kLdsMask ? TILE * W : 1];
  __shared__ int32_t s_w[kBlock / 64];

  LevelState* ls = a.ls;
  if (ls->overflow) return;
  const int L = ls->level;
  const int64_t F = ls->count[L];
  if (F == 0 || L + 2 >= kMaxLevels) return;
  const int64_t base = ls->off[L];
  const int64_t nbase = base + F;
  const int par = L & 1;
  const uint64_t* mcur = a.t.mask[par];
  uint64_t* mnxt = a.t.mask[par ^ 1];
  unsigned long long* claim = reinterpret_cast<unsigned long long*>(&ls->count[L + 1]);
  const int tid = (int)threadIdx.x;

  const int64_t ntiles = (F + TILE - 1) / TILE;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t tb = t * TILE;
    // load + choices + filter, parent p = i * 256 + tid
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int p = i * kBlock + tid;
      const int64_t j = tb + p;
      uint32_t inf = j < F ? a.t.info[base + j] : F_CYC;
      uint64_t m[W];
#pragma unroll
      for (int q = 0; q < W; ++q) m[q] = 0;
      uint64_t vm = 0;
      int k0 = 0, cb = 0;
      if (!(inf & F_CYC)) {
        load_mask<W>(mcur + j * W, m);
        vm = choices<W>(a.g, inf, m, k0, cb);
        if (vm == 0) {
          const bool pp = all_preds_on<W>(a.g, cb, node_v1l(inf), m);
          inf |= F_TERM | (pp ? F_PP : 0u);
          a.t.info[base + j] = inf;
        }
      }
      s_off[p] = __builtin_popcountll(vm);
      s_vm[p] = vm;
      s_inf[p] = inf;
      if constexpr (kLdsMask) {
#pragma unroll
        for (int q = 0; q < W; ++q) s_mask[p * W + q] = m[q];
      }
    }
    __syncthreads();
    // exclusive scan of the child counts in parent order
    int c[ITEMS];
    int sum = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      c[i] = s_off[tid * ITEMS + i];
      sum += c[i];
    }
    int32_t total32;
    int32_t run = block_excl_scan<kBlock, int32_t>(sum, total32, s_w);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      s_off[tid * ITEMS + i] = run;
      run += c[i];
    }
    // one claim per tile (tiles without children claim nothing)
    if (tid == 0)
      s_prefix = total32 ? (int64_t)atomicAdd(claim, (unsigned long long)total32) : 0;
    __syncthreads();
    const int64_t prefix = s_prefix;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int p = i * kBlock + tid;
      if (tb + p < F) {
        a.t.cstart[base + tb + p] = (int32_t)(nbase + prefix + s_off[p]);
        a.t.nch[base + tb + p] = (uint8_t)__builtin_popcountll(s_vm[p]);
      }
    }
    // load-balanced expansion: thread k writes the k-th child of the tile
    for (int k = tid; k < total32; k += kBlock) {
      int lo = 0, hi = TILE - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= k) lo = mid; else hi = mid - 1;
      }
      const int o = lo;
      const int slot = select_bit(s_vm[o], k - s_off[o]);
      const uint32_t pinf = s_inf[o];
      const int v1l = node_v1l(pinf);
      const int pv = node_v(pinf);
      const int w = a.g.s[a.g.sp[pv] + slot];
      const int wl = w - (pv - a.g.loc[pv]);
      const int64_t cl = prefix + k;
      const int64_t cg = nbase + cl;
      if (cg < a.t.rec_cap) {
        a.t.par[cg] = (int32_t)(base + tb + o);
        a.t.info[cg] = make_info(w, v1l, wl == v1l ? F_CYC : 0u);
      }
      if (wl != v1l && cl < a.t.mask_cap) {
        uint64_t pm[W];
        if constexpr (kLdsMask) {
#pragma unroll
          for (int q = 0; q < W; ++q) pm[q] = s_mask[o * W + q];
        } else {
          load_mask<W>(mcur + (tb + o) * W, pm);
        }
        store_child_mask<W>(mnxt + cl * W, pm, wl);
      }
    }
    __syncthreads();
  }
}

template <int ITEMS>
static hipError_t launch_extend_items(int W, const ExtArgs& a, int grid, hipStream_t st) {
  switch (W) {
    case 1: k_extend<1, ITEMS><<<grid, kBlock, 0, st>>>(a); break;
    case 2: k_extend<2, ITEMS><<<grid, kBlock, 0, st>>>(a); break;
    case 4: k_extend<4, ITEMS><<<grid, kBlock, 0, st>>>(a); break;
    case 8: k_extend<8, ITEMS><<<grid, kBlock, 0, st>>>(a); break;
    case 16: k_extend<16, ITEMS><<<grid, kBlock, 0, st>>>(a); break;
    case 32: k_extend<32, ITEMS><<<grid, kBlock, 0, st>>>(a); break;
    case 64: k_extend<64, ITEMS><<<grid, kBlock, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_extend(int W, int items, const ExtArgs& a, int grid, hipStream_t st) {
  switch (items) {
    case 2: return launch_extend_items<2>(W, a, grid, st);
    case 4: return launch_extend_items<4>(W, a, grid, st);
    case 8: return launch_extend_items<8>(W, a, grid, st);
    case 16: return launch_extend_items<16>(W, a, grid, st);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// two-pass (plain) form: count, host-visible scan, fill
// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(kBlock) void k_count(ExtArgs a, int L, int64_t base, int64_t F) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= F) return;
  uint32_t inf = a.t.info[base + j];
  int cnt = 0;
  if (!(inf & F_CYC)) {
    uint64_t m[W];
    load_mask<W>(a.t.mask[L & 1] + j * W, m);
    int k0, cb;
    const uint64_t vm = choices<W>(a.g, inf, m, k0, cb);
    cnt = __builtin_popcountll(vm);
    if (cnt == 0) {
      const bool pp = all_preds_on<W>(a.g, cb, node_v1l(inf), m);
      a.t.info[base + j] = inf | F_TERM | (pp ? F_PP : 0u);
    }
  }
  a.t.cstart[base + j] = cnt;
  a.t.nch[base + j] = (uint8_t)cnt;
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_fill(ExtArgs a, int L, int64_t base, int64_t F) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= F) return;
  const uint32_t inf = a.t.info[base + j];
  if (inf & F_CYC) return;
  uint64_t m[W];
  load_mask<W>(a.t.mask[L & 1] + j * W, m);
  int k0, cb;
  uint64_t vm = choices<W>(a.g, inf, m, k0, cb);
  const int v1l = node_v1l(inf);
  const int64_t nbase = base + F;
  int64_t c = a.t.cstart[base + j];
  uint64_t* mnxt = a.t.mask[(L + 1) & 1];
  while (vm) {
    const int slot = __builtin_ctzll(vm);
    vm &= vm - 1;
    const int w = a.g.s[k0 + slot];
    const int wl = w - cb;
    a.t.par[c] = (int32_t)(base + j);
    a.t.info[c] = make_info(w, v1l, wl == v1l ? F_CYC : 0u);
    if (wl != v1l) store_child_mask<W>(mnxt + (c - nbase) * W, m, wl);
    ++c;
  }
}

#define TPG_W_SWITCH(W, KERNEL, GRID, ...)                                        \
  switch (W) {                                                                      \
    case 1: KERNEL<1><<<GRID, kBlock, 0, st>>>(__VA_ARGS__); break;                 \
    case 2: KERNEL<2><<<GRID, kBlock, 0, st>>>(__VA_ARGS__); break;                 \
    case 4: KERNEL<4><<<GRID, kBlock, 0, st>>>(__VA_ARGS__); break;                 \
    case 8: KERNEL<8><<<GRID, kBlock, 0, st>>>(__VA_ARGS__); break;                 \
    case 16: KERNEL<16><<<GRID, kBlock, 0, st>>>(__VA_ARGS__); break;               \
    case 32: KERNEL<32><<<GRID, kBlock, 0, st>>>(__VA_ARGS__); break;               \
    case 64: KERNEL<64><<<GRID, kBlock, 0, st>>>(__VA_ARGS__); break;               \
    default: return hipErrorInvalidValue;                                           \
  }

hipError_t launch_count(int W, const ExtArgs& a, int L, int64_t base, int64_t F, hipStream_t st) {
  if (F == 0) return hipSuccess;
  const int64_t grid = (F + kBlock - 1) / kBlock;
  TPG_W_SWITCH(W, k_count, (unsigned)grid, a, L, base, F);
  return hipGetLastError();
}

hipError_t launch_fill(int W, const ExtArgs& a, int L, int64_t base, int64_t F, hipStream_t st) {
  if (F == 0) return hipSuccess;
  const int64_t grid = (F + kBlock - 1) / kBlock;
  TPG_W_SWITCH(W, k_fill, (unsigned)grid, a, L, base, F);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// canonical order: subtree sums bottom-up, ranks top-down
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_up(ExtArgs a, int L, int64_t base, int64_t F,
                                               uint32_t* sub_cnt, int64_t* sub_len,
                                               unsigned long long* n_cycles) {
  __shared__ int32_t s_w[kBlock / 64];
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int cyc = 0;
  if (j < F) {
    const int64_t g = base + j;
    const uint32_t inf = a.t.info[g];
    uint32_t c = 0;
    int64_t l = 0;
    if (inf & (F_CYC | F_PP)) {
      c = 1;
      l = L;
      cyc = (inf & F_CYC) ? 1 : 0;
    } else if (!(inf & F_TERM)) {
      const int64_t c0 = a.t.cstart[g], c1 = c0 + a.t.nch[g];
      for (int64_t x = c0; x < c1; ++x) {
        c += sub_cnt[x];
        l += sub_len[x];
      }
    }
    sub_cnt[g] = c;
    sub_len[g] = l;
  }
  int32_t tot;
  block_excl_scan<kBlock, int32_t>(cyc, tot, s_w);
  if (threadIdx.x == 0 && tot) atomicAdd(n_cycles, (unsigned long long)tot);
}

hipError_t launch_up(const ExtArgs& a, int L, int64_t base, int64_t F, uint32_t* sub_cnt,
                     int64_t* sub_len, unsigned long long* n_cycles, hipStream_t st) {
  if (F == 0) return hipSuccess;
  k_up<<<(unsigned)((F + kBlock - 1) / kBlock), kBlock, 0, st>>>(a, L, base, F, sub_cnt, sub_len,
                                                                  n_cycles);
  return hipGetLastError();
}

// Level-1 nodes: exclusive scans of their subtree sums give the rank of the
// first PP and the offset of its first vertex.  totals[0] = #PP,
// totals[1] = #PP vertices.  One workgroup of 1024 threads (n <= 4096).
__global__ __launch_bounds__(1024) void k_roots(ExtArgs a, int64_t n_roots, uint32_t* sub_cnt,
                                                int64_t* sub_len, int64_t* leaf_by_rank,
                                                int64_t* totals, int mode) {
  __shared__ int64_t s_w[16];
  __shared__ int64_t s_w2[16];
  int64_t carry_c = 0, carry_l = 0;
  for (int64_t b = 0; b < n_roots; b += 1024) {
    const int64_t i = b + threadIdx.x;
    const int64_t c = i < n_roots ? (int64_t)sub_cnt[i] : 0;
    const int64_t l = i < n_roots ? sub_len[i] : 0;
    int64_t tc, tl;
    const int64_t pc = block_excl_scan<1024, int64_t>(c, tc, s_w);
    const int64_t pl = block_excl_scan<1024, int64_t>(l, tl, s_w2);
    if (i < n_roots && mode == 1) {
      const int64_t rank = carry_c + pc;
      sub_cnt[i] = (uint32_t)rank;
      sub_len[i] = carry_l + pl;
      if (a.t.info[i] & (F_PP | F_CYC)) leaf_by_rank[rank] = i;
    }
    carry_c += tc;
    carry_l += tl;
  }
  if (threadIdx.x == 0 && mode == 0) {
    totals[0] = carry_c;
    totals[1] = carry_l;
  }
}

hipError_t launch_roots(const ExtArgs& a, int64_t n_roots, uint32_t* sub_cnt, int64_t* sub_len,
                        int64_t* leaf_by_rank, int64_t* totals, int mode, hipStream_t st) {
  k_roots<<<1, 1024, 0, st>>>(a, n_roots, sub_cnt, sub_len, leaf_by_rank, totals, mode);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_down(ExtArgs a, int64_t base, int64_t F,
                                                 uint32_t* sub_cnt, int64_t* sub_len,
                                                 int64_t* leaf_by_rank) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= F) return;
  const int64_t g = base + j;
  const uint32_t inf = a.t.info[g];
  if (inf & (F_CYC | F_TERM)) return;
  int64_t r = sub_cnt[g];
  int64_t o = sub_len[g];
  const int64_t c0 = a.t.cstart[g], c1 = c0 + a.t.nch[g];
  for (int64_t x = c0; x < c1; ++x) {
    const uint32_t cc = sub_cnt[x];
    const int64_t cl = sub_len[x];
    sub_cnt[x] = (uint32_t)r;
    sub_len[x] = o;
    if (a.t.info[x] & (F_PP | F_CYC)) leaf_by_rank[r] = x;
    r += cc;
    o += cl;
  }
}

hipError_t launch_down(const ExtArgs& a, int64_t base, int64_t F, uint32_t* sub_cnt,
                       int64_t* sub_len, int64_t* leaf_by_rank, hipStream_t st) {
  if (F == 0) return hipSuccess;
  k_down<<<(unsigned)((F + kBlock - 1) / kBlock), kBlock, 0, st>>>(a, base, F, sub_cnt, sub_len,
                                                                    leaf_by_rank);
  return hipGetLastError();
}

__global__ void k_pp_offsets(const int64_t* leaf_by_rank, const int64_t* sub_len, int64_t n_pp,
                             int64_t total, int64_t* pp_off) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_pp) pp_off[i] = sub_len[leaf_by_rank[i]];
  if (i == n_pp) pp_off[i] = total;
}

hipError_t launch_pp_offsets(const int64_t* leaf_by_rank, const int64_t* sub_len, int64_t n_pp,
                             int64_t total, int64_t* pp_off, hipStream_t st) {
  k_pp_offsets<<<(unsigned)((n_pp + 1 + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      leaf_by_rank, sub_len, n_pp, total, pp_off);
  return hipGetLastError();
}

// Each thread writes one prime path by walking parent links from its leaf.
// The walk yields entries back to front; they are buffered 32 at a time in
// registers and stored as one burst of consecutive addresses, so that lines
// are written whole instead of one word per dependent load.
__global__ __launch_bounds__(kBlock) void k_pp_write(ExtArgs a, const int64_t* leaf_by_rank,
                                                     const int64_t* pp_off, int64_t n_pp,
                                                     int32_t* pp_vtx) {
  constexpr int kBuf = 32;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n_pp) return;
  int64_t x = leaf_by_rank[i];
  int64_t pos = pp_off[i + 1] - 1;
  const int64_t lo = pp_off[i];
  while (pos >= lo && x >= 0) {
    int32_t buf[kBuf];
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < kBuf; ++j) {
      if (pos - j >= lo && x >= 0) {
        buf[j] = node_v(a.t.info[x]);
        x = a.t.par[x];
        cnt = j + 1;
      }
    }
#pragma unroll
    for (int j = kBuf - 1; j >= 0; --j)
      if (j < cnt) pp_vtx[pos - j] = buf[j];
    pos -= cnt;
  }
}

hipError_t launch_pp_write(const ExtArgs& a, const int64_t* leaf_by_rank, const int64_t* pp_off,
                           int64_t n_pp, int32_t* pp_vtx, hipStream_t st) {
  if (n_pp == 0) return hipSuccess;
  k_pp_write<<<(unsigned)((n_pp + kBlock - 1) / kBlock), kBlock, 0, st>>>(a, leaf_by_rank, pp_off,
                                                                          n_pp, pp_vtx);
  return hipGetLastError();
}

}  // namespace tpg

namespace tpg {

__global__ void k_comp_pp_starts(DGraph g, const uint32_t* sub_cnt, const int64_t* sub_len,
                                 const int64_t* totals, int64_t* pp_start, int64_t* ppv_start) {
  const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (c < g.n_comp) {
    pp_start[c] = sub_cnt[g.cbase[c]];
    ppv_start[c] = sub_len[g.cbase[c]];
  }
  if (c == g.n_comp) {
    pp_start[c] = totals[0];
    ppv_start[c] = totals[1];
  }
}

hipError_t launch_comp_pp_starts(const DGraph& g, const uint32_t* sub_cnt, const int64_t* sub_len,
                                 const int64_t* totals, int64_t* pp_start, int64_t* ppv_start,
                                 hipStream_t st) {
  k_comp_pp_starts<<<(unsigned)((g.n_comp + 1 + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      g, sub_cnt, sub_len, totals, pp_start, ppv_start);
  return hipGetLastError();
}

__global__ void k_level_comp_counts(ExtArgs a, int L, int64_t base, int64_t F, int64_t* lvl) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= F) return;
  const int c = a.g.comp[node_v(a.t.info[base + j])];
  const int b = (L < 64 ? L : 64) - 1;
  atomicAdd((unsigned long long*)&lvl[(int64_t)c * 64 + b], 1ull);
}

hipError_t launch_level_comp_counts(const ExtArgs& a, int L, int64_t base, int64_t F,
                                    int64_t* lvl_comp, hipStream_t st) {
  if (F == 0) return hipSuccess;
  k_level_comp_counts<<<(unsigned)((F + kBlock - 1) / kBlock), kBlock, 0, st>>>(a, L, base, F,
                                                                                lvl_comp);
  return hipGetLastError();
}

}  // namespace tpg
