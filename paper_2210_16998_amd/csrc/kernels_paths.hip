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
//    (registers while testing).  In HBM only the odd levels' sets are kept,
//    two stored levels alive: a path on an even level is a path of the odd
//    level before plus its last vertex, so its set is rebuilt from its
//    parent's (siblings read the same stored set).  Sets are stored
//    word-major: word q of slot j sits at q * stride + j, so the threads of
//    a wave, which own consecutive slots, read and write consecutive words.
//  * One workgroup handles a tile of 256 * ITEMS parents: choice masks over
//    successor slots, a block scan of child counts, then ONE device-scope
//    atomic claim of the tile's slice of the next level, then a
//    load-balanced expansion where consecutive threads write consecutive
//    children, so record and mask stores are coalesced.  No workgroup ever
//    waits for another one; the order of tile slices inside a level is the
//    order in which the claims landed, which ranking does not depend on.
//  * Levels follow each other on the device: per-level counts and offsets
//    live in device memory; launch li of a batch extends level
//    batch_start + li and derives its offset from the level before, or
//    raises the overflow flag when that level's children did not fit; the
//    host then grows the buffers to the exact size and replays the level.
//  * The plain two-pass form (count, scan, host-visible size, fill) keeps
//    children in parent order and serves as the exact reference form.

#include <hip/hip_ext.h>

#include "kernels.h"
#include "sizing.h"

namespace tpg {

// ---------------------------------------------------------------------------
// level 1
// ---------------------------------------------------------------------------
__global__ void k_seed(ExtArgs a) {
  const int n = a.seed_n;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  LevelState* ls = a.ls;
  // every level's claim counter starts at zero
  for (int64_t k = i; k < kMaxLevels; k += (int64_t)gridDim.x * blockDim.x) {
    ls->count[k] = k == 1 ? n : 0;
    ls->off[k] = 0;
  }
  if (i == 0) {
    ls->batch_start = 1;
    ls->overflow = 0;
    ls->overflow_level = 0;
  }
  if (i < n) {
    const int v = a.seed_lo + (int)i;
    a.t.par[i] = -1;
    a.t.info[i] = make_info(v, a.g.loc[v], 0);
  }
  // visited sets of level 1 (stored, buffer 0): one bit each, at the
  // vertex's local id
  const int W = a.t.mask_words;
  for (int64_t k = i; k < (int64_t)n * W; k += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(k / n), j = (int)(k % n);
    const int l = a.g.loc[a.seed_lo + j];
    a.t.mask[0][(int64_t)q * a.t.mask_cap + j] = (q == (l >> 6)) ? (1ull << (l & 63)) : 0ull;
  }
}

hipError_t launch_seed(const ExtArgs& a, hipStream_t st) {
  if (a.seed_lo < 0 || a.seed_n < 1 || a.seed_lo + a.seed_n > a.g.n) return hipErrorInvalidValue;
  const int64_t work = std::max<int64_t>(kMaxLevels, (int64_t)a.seed_n * a.t.mask_words);
  const int grid = (int)std::min<int64_t>(1024, (work + kBlock - 1) / kBlock + 1);
  k_seed<<<grid, kBlock, 0, st>>>(a);
  return hipGetLastError();
}

// Resume after an overflow: the level is extended again from a zero claim.
__global__ void k_resume_fix(ExtArgs a, int level) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.ls->count[level + 1] = 0;
    a.ls->overflow = 0;
    a.ls->overflow_level = 0;
  }
}

hipError_t launch_resume_fix(const ExtArgs& a, int level, hipStream_t st) {
  if (level < 1 || level + 1 >= kMaxLevels) return hipErrorInvalidValue;
  k_resume_fix<<<1, 64, 0, st>>>(a, level);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// shared per-parent step: choice mask over successor slots + terminal filter
// ---------------------------------------------------------------------------
// Choice mask over the successor slots [k0, k1) of the path's last vertex:
// slot k is set when successor w is not on the path, or is its first vertex
// (closes a cycle).  cb = graph-wide id of local id 0 of the component.
template <int W>
__device__ __forceinline__ uint64_t choices(const DGraph& g, uint32_t inf, const uint64_t (&m)[W],
                                            int k0, int k1, int cb) {
  const int v1l = node_v1l(inf);
  uint64_t vm = 0;
  for (int k = k0; k < k1; ++k) {
    const int wl = g.s[k] - cb;
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

// Visited set of slot j of a level (word-major, stride S slots).  Only the
// first Wu words are stored (ceil(largest component / 64)); the register
// copy is padded with zero words up to W.
template <int W>
__device__ __forceinline__ void load_mask(const uint64_t* src, int64_t S, int Wu, int64_t j,
                                          uint64_t (&m)[W]) {
#pragma unroll
  for (int q = 0; q < W; ++q) m[q] = q < Wu ? src[q * S + j] : 0ull;
}

// Visited set of child slot c: the parent's set plus local vertex w.
template <int W>
__device__ __forceinline__ void store_child_mask(uint64_t* dst, int64_t S, int Wu, int64_t c,
                                                 const uint64_t (&m)[W], int w) {
  const int q = w >> 6;
  const uint64_t bit = 1ull << (w & 63);
#pragma unroll
  for (int k = 0; k < W; ++k)
    if (k < Wu) dst[k * S + c] = m[k] | (k == q ? bit : 0ull);
}

// Stored levels (odd) alternate between the two buffers.
__device__ __forceinline__ int mask_buf(int L) { return ((L - 1) >> 1) & 1; }

// Visited set of the path in slot j of level L: an odd level's set is
// stored; an even level's is its parent's (slot par - prev of level L - 1,
// which starts at node prev) plus its own last vertex, local id vl.
template <int W>
__device__ __forceinline__ void path_mask_load(const ExtArgs& a, int L, int64_t prev, int64_t node,
                                               int64_t j, uint64_t (&m)[W]) {
  if (L & 1) {
    load_mask<W>(a.t.mask[mask_buf(L)], a.t.mask_cap, a.t.mask_words, j, m);
  } else {
    const int64_t jp = (int64_t)a.t.par[node] - prev;
    load_mask<W>(a.t.mask[mask_buf(L - 1)], a.t.mask_cap, a.t.mask_words, jp, m);
  }
}
template <int W>
__device__ __forceinline__ void path_mask_own(int L, int vl, uint64_t (&m)[W]) {
  if (L & 1) return;  // stored sets already hold the last vertex
  const int q = vl >> 6;
  const uint64_t bit = 1ull << (vl & 63);
#pragma unroll
  for (int k = 0; k < W; ++k) m[k] |= (k == q) ? bit : 0ull;
}

// ---------------------------------------------------------------------------
// one-pass extension of level L -> L+1 (device-sized, claim per tile)
// ---------------------------------------------------------------------------
// Launch `li` of a batch extends level L = batch_start + li.  Its offset is
// derived from the previous level's final offset and size, so no kernel has
// to advance a level counter; a level whose nodes did not fit (claimed
// beyond the capacities by the launch before) raises the overflow flag and
// ends the batch.
//
// A tile is 256 * ir consecutive parents (ir <= ITEMS, chosen per level so
// that large levels need few claims and small ones still spread over the
// grid); tile t goes to workgroup t mod grid.  Thread tid owns parents
// i * 256 + tid (i < ir): their records and visited sets are loaded together
// (coalesced), the visited sets stay in registers, and the thread writes its
// own parents' children.  Children are laid out item-major and, inside an
// item, in thread order, so a wave's stores land on neighbouring slots.  A
// level that fits one tile stores its size instead of claiming.
//
// GL: the CSR (row pointers, successors, predecessors, local ids) is copied
// into LDS by every workgroup that has a tile, so the per-parent chain of
// graph lookups (row range -> successor ids -> predecessor ids) reads LDS
// instead of L2.
template <int W, int ITEMS, int NT, bool GL>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT == 1024 && ITEMS == 1 && W <= 8 ? 8 : 1))) void k_extend_tp(ExtArgs a, int li) {
  constexpr int NW = NT / 64;
  __shared__ int32_t s_tot[ITEMS][NW];
  __shared__ int64_t s_prefix;
  extern __shared__ int32_t s_graph[];

  LevelState* ls = a.ls;
  if (ls->overflow) return;
  const int L = ls->batch_start + li;
  if (L < 1 || L + 2 >= kMaxLevels) return;
  const int64_t F = ls->count[L];
  if (F == 0) return;
  const int64_t base = ls->off[L - 1] + ls->count[L - 1];
  const int tid = (int)threadIdx.x;
  const int lane = lane_id(), wave = tid >> 6;
  if (!level_fits(L, base, F, a.t.rec_cap, a.t.mask_cap)) {
    // the previous launch's children did not fit: replay that level
    if (blockIdx.x == 0 && tid == 0) {
      ls->overflow_level = L - 1;
      ls->overflow = 1;
    }
    return;
  }
  if (blockIdx.x == 0 && tid == 0) ls->off[L] = base;
  const int64_t nbase = base + F;
  const int64_t prev = ls->off[L - 1];
  // children's sets are stored when they land on an odd level
  uint64_t* mnxt = (L & 1) ? nullptr : a.t.mask[mask_buf(L + 1)];
  unsigned long long* claim = reinterpret_cast<unsigned long long*>(&ls->count[L + 1]);

  int ir = 1;
  while (ir < ITEMS && (F + (int64_t)NT * ir - 1) / ((int64_t)NT * ir) > a.tiles_target) ir <<= 1;
  const int64_t TR = (int64_t)NT * ir;
  const int64_t ntiles = (F + TR - 1) / TR;
  DGraph g = a.g;
  if constexpr (GL) {
    if ((int64_t)blockIdx.x >= ntiles) return;
    for (int i = tid; i < a.g.n_stage; i += NT) s_graph[i] = a.g.sp[i];
    __syncthreads();
    g.sp = s_graph;
    g.s = s_graph + (a.g.s - a.g.sp);
    g.pp = s_graph + (a.g.pp - a.g.sp);
    g.p = s_graph + (a.g.p - a.g.sp);
    g.loc = s_graph + (a.g.loc - a.g.sp);
  }
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t tb = t * TR;
    // records and visited sets of the thread's parents (independent loads;
    // rows outside the level read parent 0's set and are ignored)
    uint32_t inf[ITEMS];
    uint64_t m[ITEMS][W];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int64_t j = tb + i * NT + tid;
      const bool ok = i < ir && j < F;
      inf[i] = ok ? a.t.info[base + j] : F_CYC;
      path_mask_load<W>(a, L, prev, base + (ok ? j : 0), ok ? j : 0, m[i]);
    }
    // choice masks and the terminal filter
    uint64_t vm[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      vm[i] = 0;
      if (!(inf[i] & F_CYC)) {
        const int v = node_v(inf[i]);
        const int cb = v - g.loc[v];
        path_mask_own<W>(L, v - cb, m[i]);
        vm[i] = choices<W>(g, inf[i], m[i], g.sp[v], g.sp[v + 1], cb);
        if (vm[i] == 0) {
          const bool pp = all_preds_on<W>(g, cb, node_v1l(inf[i]), m[i]);
          inf[i] |= F_TERM | (pp ? F_PP : 0u);  // recorded through nch_code below
        }
      }
    }
    // child offsets: item-major, thread order inside an item
    int excl[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int c = __builtin_popcountll(vm[i]);
      const int inc = wave_incl_scan(c);
      excl[i] = inc - c;
      if (lane == 63) s_tot[i][wave] = inc;
    }
    __syncthreads();
    int total = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      int before = 0, all = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const int x = i < ir ? s_tot[i][w] : 0;
        before += w < wave ? x : 0;
        all += x;
      }
      excl[i] += total + before;
      total += all;
    }
    if (tid == 0) {
      int64_t pre = 0;
      if (ntiles == 1) {
        *claim = (unsigned long long)total;  // the only tile of the level
      } else if (total) {
        pre = (int64_t)atomicAdd(claim, (unsigned long long)total);
      }
      s_prefix = pre;
    }
    __syncthreads();
    const int64_t prefix = s_prefix;
    // expansion: each thread writes its parents' children in slot order
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int64_t j = tb + i * NT + tid;
      if (i < ir && j < F) {
        int64_t cl = prefix + excl[i];
        a.t.cstart[base + j] = (int32_t)(nbase + cl);
        a.t.nch[base + j] = nch_code(inf[i], __builtin_popcountll(vm[i]));
        const int v1l = node_v1l(inf[i]);
        uint64_t rest = vm[i];
        const int pv = node_v(inf[i]);
        const int k0 = rest ? g.sp[pv] : 0;
        const int cb = rest ? pv - g.loc[pv] : 0;
        while (rest) {
          const int slot = __builtin_ctzll(rest);
          rest &= rest - 1;
          const int w = g.s[k0 + slot];
          const int wl = w - cb;
          const int64_t cg = nbase + cl;
          if (cg < a.t.rec_cap) {
            a.t.par[cg] = (int32_t)(base + j);
            a.t.info[cg] = make_info(w, v1l, wl == v1l ? F_CYC : 0u);
          }
          if (mnxt && wl != v1l && cl < a.t.mask_cap)
            store_child_mask<W>(mnxt, a.t.mask_cap, a.t.mask_words, cl, m[i], wl);
          ++cl;
        }
      }
    }
    __syncthreads();
  }
}

// Load-balanced form of the same step: the tile's parents are staged in LDS
// (choice masks, records, successor-row starts, visited sets when they fit)
// and thread k writes the k-th child of the tile, found by binary search
// over the parents' child offsets.
template <int W, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_extend_lb(ExtArgs a, int li) {
  constexpr int TILE = kBlock * ITEMS;
  constexpr bool kLdsMask = W * ITEMS <= 16;  // visited sets of the tile in LDS (<= 32 KiB)
  __shared__ int64_t s_prefix;
  __shared__ int32_t s_off[TILE];
  __shared__ uint64_t s_vm[TILE];
  __shared__ uint32_t s_inf[TILE];
  __shared__ int32_t s_kk[TILE];
  __shared__ uint64_t s_mask[kLdsMask ? TILE * W : 1];
  __shared__ int32_t s_w[kBlock / 64];

  LevelState* ls = a.ls;
  if (ls->overflow) return;
  const int L = ls->batch_start + li;
  if (L < 1 || L + 2 >= kMaxLevels) return;
  const int64_t F = ls->count[L];
  if (F == 0) return;
  const int64_t base = ls->off[L - 1] + ls->count[L - 1];
  const int tid = (int)threadIdx.x;
  if (!level_fits(L, base, F, a.t.rec_cap, a.t.mask_cap)) {
    if (blockIdx.x == 0 && tid == 0) {
      ls->overflow_level = L - 1;
      ls->overflow = 1;
    }
    return;
  }
  if (blockIdx.x == 0 && tid == 0) ls->off[L] = base;
  const int64_t nbase = base + F;
  const int64_t prev = ls->off[L - 1];
  uint64_t* mnxt = (L & 1) ? nullptr : a.t.mask[mask_buf(L + 1)];
  unsigned long long* claim = reinterpret_cast<unsigned long long*>(&ls->count[L + 1]);

  int ir = 1;
  while (ir < ITEMS && (F + (int64_t)kBlock * ir - 1) / ((int64_t)kBlock * ir) > a.tiles_target) ir <<= 1;
  const int TR = kBlock * ir;
  const int64_t ntiles = (F + TR - 1) / TR;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t tb = t * TR;
    uint32_t inf[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int64_t j = tb + i * kBlock + tid;
      inf[i] = (i < ir && j < F) ? a.t.info[base + j] : F_CYC;
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      if (i < ir) {
        const int p = i * kBlock + tid;
        const int64_t j = tb + p;
        uint32_t in = inf[i];
        uint64_t m[W];
#pragma unroll
        for (int q = 0; q < W; ++q) m[q] = 0;
        uint64_t vm = 0;
        int k0 = 0;
        if (!(in & F_CYC)) {
          const int v = node_v(in);
          const int cb = v - a.g.loc[v];
          k0 = a.g.sp[v];
          path_mask_load<W>(a, L, prev, base + j, j, m);
          path_mask_own<W>(L, v - cb, m);
          vm = choices<W>(a.g, in, m, k0, a.g.sp[v + 1], cb);
          if (vm == 0) {
            const bool pp = all_preds_on<W>(a.g, cb, node_v1l(in), m);
            in |= F_TERM | (pp ? F_PP : 0u);  // recorded through nch_code
          }
        }
        s_off[p] = __builtin_popcountll(vm);
        s_vm[p] = vm;
        s_inf[p] = in;
        s_kk[p] = k0;
        if constexpr (kLdsMask) {
#pragma unroll
          for (int q = 0; q < W; ++q) s_mask[p * W + q] = m[q];
        }
      }
    }
    __syncthreads();
    int c[ITEMS];
    int sum = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      c[i] = i < ir ? s_off[tid * ir + i] : 0;
      sum += c[i];
    }
    int32_t total32;
    int32_t run = block_excl_scan<kBlock, int32_t>(sum, total32, s_w);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      if (i < ir) s_off[tid * ir + i] = run;
      run += c[i];
    }
    if (tid == 0) {
      int64_t pre = 0;
      if (ntiles == 1) *claim = (unsigned long long)total32;
      else if (total32) pre = (int64_t)atomicAdd(claim, (unsigned long long)total32);
      s_prefix = pre;
    }
    __syncthreads();
    const int64_t prefix = s_prefix;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int p = i * kBlock + tid;
      if (i < ir && tb + p < F) {
        a.t.cstart[base + tb + p] = (int32_t)(nbase + prefix + s_off[p]);
        a.t.nch[base + tb + p] = nch_code(s_inf[p], __builtin_popcountll(s_vm[p]));
      }
    }
    for (int k = tid; k < total32; k += kBlock) {
      int lo = 0, hi = TR - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= k) lo = mid; else hi = mid - 1;
      }
      const int o = lo;
      const int slot = select_bit(s_vm[o], k - s_off[o]);
      const uint32_t pinf = s_inf[o];
      const int v1l = node_v1l(pinf);
      const int pv = node_v(pinf);
      const int w = a.g.s[s_kk[o] + slot];
      const int wl = w - (pv - a.g.loc[pv]);
      const int64_t cl = prefix + k;
      const int64_t cg = nbase + cl;
      if (cg < a.t.rec_cap) {
        a.t.par[cg] = (int32_t)(base + tb + o);
        a.t.info[cg] = make_info(w, v1l, wl == v1l ? F_CYC : 0u);
      }
      if (mnxt && wl != v1l && cl < a.t.mask_cap) {
        uint64_t pm[W];
        if constexpr (kLdsMask) {
#pragma unroll
          for (int q = 0; q < W; ++q) pm[q] = s_mask[o * W + q];
        } else {
          path_mask_load<W>(a, L, prev, base + tb + o, tb + o, pm);
          path_mask_own<W>(L, a.g.loc[pv], pm);
        }
        store_child_mask<W>(mnxt, a.t.mask_cap, a.t.mask_words, cl, pm, wl);
      }
    }
    __syncthreads();
  }
}

// Launch with optional start / stop events recorded by the dispatch itself
// (the kernel's own execution interval, without queueing around it).
template <class K>
static hipError_t launch_timed(K kernel, int grid, int threads, hipEvent_t e0, hipEvent_t e1,
                               const ExtArgs& a, int li, hipStream_t st, size_t lds = 0) {
  if (e0 && e1)
    hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(threads), lds, st, e0, e1, 0, a, li);
  else
    kernel<<<grid, threads, lds, st>>>(a, li);
  return hipGetLastError();
}

// variant 0: load-balanced (256 threads); 1: thread-per-parent, 256
// threads; 2: thread-per-parent, 1024 threads.  Register-resident visited
// sets are capped at 32 words per thread; wider sets always take variant 0.
template <int W, int ITEMS>
static hipError_t launch_extend_wi(int variant, const ExtArgs& a, int grid, int li, hipStream_t st,
                                   hipEvent_t e0, hipEvent_t e1) {
  if constexpr (ITEMS * W <= 32) {
    const size_t gb = sizeof(int32_t) * (size_t)a.g.n_stage;
    if (gb <= (size_t)kGraphLdsBytes) {
      if (variant == 1)
        return launch_timed(k_extend_tp<W, ITEMS, 256, true>, grid, 256, e0, e1, a, li, st, gb);
      if (variant == 2)
        return launch_timed(k_extend_tp<W, ITEMS, 1024, true>, grid, 1024, e0, e1, a, li, st, gb);
    }
    if (variant == 1) return launch_timed(k_extend_tp<W, ITEMS, 256, false>, grid, 256, e0, e1, a, li, st);
    if (variant == 2) return launch_timed(k_extend_tp<W, ITEMS, 1024, false>, grid, 1024, e0, e1, a, li, st);
  }
  return launch_timed(k_extend_lb<W, ITEMS>, grid, kBlock, e0, e1, a, li, st);
}

template <int W>
static hipError_t launch_extend_w(int items, int variant, const ExtArgs& a, int grid, int li,
                                  hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  int it = items;
  if (variant != 0)
    while (it > 1 && it * W > 32) it >>= 1;
  switch (it) {
    case 1: return launch_extend_wi<W, 1>(variant, a, grid, li, st, e0, e1);
    case 2: return launch_extend_wi<W, 2>(variant, a, grid, li, st, e0, e1);
    case 4: return launch_extend_wi<W, 4>(variant, a, grid, li, st, e0, e1);
    case 8: return launch_extend_wi<W, 8>(variant, a, grid, li, st, e0, e1);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_extend(int W, int items, int variant, const ExtArgs& a, int grid, int li,
                         hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (variant < 0 || variant > 2) return hipErrorInvalidValue;
  switch (W) {
    case 1: return launch_extend_w<1>(items, variant, a, grid, li, st, e0, e1);
    case 2: return launch_extend_w<2>(items, variant, a, grid, li, st, e0, e1);
    case 4: return launch_extend_w<4>(items, variant, a, grid, li, st, e0, e1);
    case 8: return launch_extend_w<8>(items, variant, a, grid, li, st, e0, e1);
    case 16: return launch_extend_w<16>(items, variant, a, grid, li, st, e0, e1);
    case 32: return launch_extend_w<32>(items, variant, a, grid, li, st, e0, e1);
    case 64: return launch_extend_w<64>(items, variant, a, grid, li, st, e0, e1);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// two-pass (plain) form: count, host-visible scan, fill
// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(kBlock) void k_count(ExtArgs a, int L, int64_t prev, int64_t base,
                                                  int64_t F) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= F) return;
  uint32_t inf = a.t.info[base + j];
  int cnt = 0;
  if (!(inf & F_CYC)) {
    uint64_t m[W];
    path_mask_load<W>(a, L, prev, base + j, j, m);
    const int v = node_v(inf);
    const int cb = v - a.g.loc[v];
    path_mask_own<W>(L, v - cb, m);
    const uint64_t vm = choices<W>(a.g, inf, m, a.g.sp[v], a.g.sp[v + 1], cb);
    cnt = __builtin_popcountll(vm);
    if (cnt == 0) {
      const bool pp = all_preds_on<W>(a.g, cb, node_v1l(inf), m);
      inf |= F_TERM | (pp ? F_PP : 0u);  // recorded through nch_code
    }
  }
  a.t.cstart[base + j] = cnt;
  a.t.nch[base + j] = nch_code(inf, cnt);
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_fill(ExtArgs a, int L, int64_t prev, int64_t base,
                                                 int64_t F) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= F) return;
  const uint32_t inf = a.t.info[base + j];
  if (inf & F_CYC) return;
  uint64_t m[W];
  path_mask_load<W>(a, L, prev, base + j, j, m);
  const int v = node_v(inf);
  const int k0 = a.g.sp[v];
  const int cb = v - a.g.loc[v];
  path_mask_own<W>(L, v - cb, m);
  uint64_t vm = choices<W>(a.g, inf, m, k0, a.g.sp[v + 1], cb);
  const int v1l = node_v1l(inf);
  const int64_t nbase = base + F;
  int64_t c = a.t.cstart[base + j];
  uint64_t* mnxt = (L & 1) ? nullptr : a.t.mask[mask_buf(L + 1)];
  while (vm) {
    const int slot = __builtin_ctzll(vm);
    vm &= vm - 1;
    const int w = a.g.s[k0 + slot];
    const int wl = w - cb;
    a.t.par[c] = (int32_t)(base + j);
    a.t.info[c] = make_info(w, v1l, wl == v1l ? F_CYC : 0u);
    if (mnxt && wl != v1l) store_child_mask<W>(mnxt, a.t.mask_cap, a.t.mask_words, c - nbase, m, wl);
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

hipError_t launch_count(int W, const ExtArgs& a, int L, int64_t prev, int64_t base, int64_t F,
                        hipStream_t st) {
  if (F == 0) return hipSuccess;
  const int64_t grid = (F + kBlock - 1) / kBlock;
  TPG_W_SWITCH(W, k_count, (unsigned)grid, a, L, prev, base, F);
  return hipGetLastError();
}

hipError_t launch_fill(int W, const ExtArgs& a, int L, int64_t prev, int64_t base, int64_t F,
                       hipStream_t st) {
  if (F == 0) return hipSuccess;
  const int64_t grid = (F + kBlock - 1) / kBlock;
  TPG_W_SWITCH(W, k_fill, (unsigned)grid, a, L, prev, base, F);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// canonical order: subtree counts bottom-up, ranks top-down
// ---------------------------------------------------------------------------
// sub_cnt[g] = prime-path leaves in g's subtree (k_up), then rewritten top-down
// into the rank of the subtree's first prime path, or kNoRank when the
// subtree holds none (k_down then skips it after one 4-byte read).
constexpr uint32_t kNoRank = 0xFFFFFFFFu;

__global__ __launch_bounds__(kBlock) void k_up(ExtArgs a, int L, int64_t base, int64_t F,
                                               uint32_t* sub_cnt, unsigned long long* n_cycles) {
  __shared__ int32_t s_w[kBlock / 64];
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int cyc = 0;
  if (j < F) {
    const int64_t g = base + j;
    const uint8_t k = a.t.nch[g];
    uint32_t c = 0;
    if (k >= kNchPP) {
      c = 1;
      cyc = k == kNchCycle ? 1 : 0;
    } else if (k) {
      const int64_t c0 = a.t.cstart[g], c1 = c0 + k;
      for (int64_t x = c0; x < c1; ++x) c += sub_cnt[x];
    }
    sub_cnt[g] = c;
  }
  int32_t tot;
  block_excl_scan<kBlock, int32_t>(cyc, tot, s_w);
  if (threadIdx.x == 0 && tot) atomicAdd(n_cycles + blockIdx.x % kCycleSlots, (unsigned long long)tot);
}

hipError_t launch_up(const ExtArgs& a, int L, int64_t base, int64_t F, uint32_t* sub_cnt,
                     unsigned long long* n_cycles, hipStream_t st) {
  if (F == 0) return hipSuccess;
  k_up<<<(unsigned)((F + kBlock - 1) / kBlock), kBlock, 0, st>>>(a, L, base, F, sub_cnt, n_cycles);
  return hipGetLastError();
}

// Level-1 nodes: an exclusive scan of their subtree counts gives the rank of
// their first prime path.  totals[0] = #PP.  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_roots(ExtArgs a, int64_t n_roots, uint32_t* sub_cnt,
                                                int64_t* leaf_by_rank, int32_t* pp_len,
                                                int64_t* totals, int mode, int64_t* rb,
                                                unsigned long long* n_cycles) {
  __shared__ int64_t s_w[16];
  int64_t carry = 0;
  for (int64_t b = 0; b < n_roots; b += 1024) {
    const int64_t i = b + threadIdx.x;
    const int64_t c = i < n_roots ? (int64_t)sub_cnt[i] : 0;
    int64_t tc;
    const int64_t pc = block_excl_scan<1024, int64_t>(c, tc, s_w);
    if (i < n_roots && mode == 1) {
      const int64_t rank = carry + pc;
      if (rb) rb[i] = rank;  // root i is vertex i: its first prime path's rank
      sub_cnt[i] = (uint32_t)rank;
      if (a.t.nch[i] >= kNchPP) {
        leaf_by_rank[rank] = i;
        pp_len[rank] = 1;
      }
    }
    carry += tc;
  }
  if (threadIdx.x == 0 && mode == 0) totals[0] = carry;
  if (mode == 0 && n_cycles && threadIdx.x < 64) {  // the first wave sums the cycle slots
    unsigned long long c = 0;
    for (int s = (int)threadIdx.x; s < kCycleSlots; s += 64) c += n_cycles[s];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      const unsigned lo = __shfl_xor((unsigned)c, d, 64), hi = __shfl_xor((unsigned)(c >> 32), d, 64);
      c += ((unsigned long long)hi << 32) | lo;
    }
    if (threadIdx.x == 0) n_cycles[kCycleSlots] = c;
  }
  if (threadIdx.x == 0 && mode == 1 && rb) rb[n_roots] = carry;
}

hipError_t launch_roots(const ExtArgs& a, int64_t n_roots, uint32_t* sub_cnt, int64_t* leaf_by_rank,
                        int32_t* pp_len, int64_t* totals, int mode, int64_t* rb,
                        unsigned long long* n_cycles, hipStream_t st) {
  k_roots<<<1, 1024, 0, st>>>(a, n_roots, sub_cnt, leaf_by_rank, pp_len, totals, mode, rb,
                              n_cycles);
  return hipGetLastError();
}

// Parents of level L hand ranks to their children in slot order; a prime
// path leaf records its node and length (L + 1 entries) under its rank.
__global__ __launch_bounds__(kBlock) void k_down(ExtArgs a, int L, int64_t base, int64_t F,
                                                 uint32_t* sub_cnt, int64_t* leaf_by_rank,
                                                 int32_t* pp_len) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= F) return;
  const int64_t g = base + j;
  uint32_t r = sub_cnt[g];
  const uint8_t k = a.t.nch[g];
  if (r == kNoRank || k == 0 || k >= kNchPP) return;
  const int64_t c0 = a.t.cstart[g], c1 = c0 + k;
  for (int64_t x = c0; x < c1; ++x) {
    const uint32_t cc = sub_cnt[x];
    sub_cnt[x] = cc ? r : kNoRank;
    if (cc && a.t.nch[x] >= kNchPP) {
      leaf_by_rank[r] = x;
      pp_len[r] = L + 1;
    }
    r += cc;
  }
}

hipError_t launch_down(const ExtArgs& a, int L, int64_t base, int64_t F, uint32_t* sub_cnt,
                       int64_t* leaf_by_rank, int32_t* pp_len, hipStream_t st) {
  if (F == 0) return hipSuccess;
  k_down<<<(unsigned)((F + kBlock - 1) / kBlock), kBlock, 0, st>>>(a, L, base, F, sub_cnt,
                                                                    leaf_by_rank, pp_len);
  return hipGetLastError();
}

// D + 1 levels per launch (D = 1, 2): a launch costs ~7 us however little it
// does, and a sweep has one per level.  One thread per node x of the run's
// top level does the per-level work for x and for its descendants down to D
// levels below (they are x's alone, and each count or rank is read right
// after this thread wrote it); the recursion unrolls at compile time.
template <int D>
__device__ __forceinline__ uint32_t up_node(const ExtArgs& a, int64_t x, uint32_t* sub_cnt,
                                            int& cyc) {
  const uint8_t k = a.t.nch[x];
  uint32_t c = 0;
  if (k >= kNchPP) {
    c = 1;
    cyc += k == kNchCycle ? 1 : 0;
  } else if (k) {
    const int64_t c0 = a.t.cstart[x], c1 = c0 + k;
    for (int64_t y = c0; y < c1; ++y) {
      if constexpr (D > 0)
        c += up_node<D - 1>(a, y, sub_cnt, cyc);
      else
        c += sub_cnt[y];
    }
  }
  sub_cnt[x] = c;
  return c;
}

// The same for D = 1 with the loads batched: x's children's codes and child
// ranges kSweepBatch at a time, then their own children's counts all
// together, so that a thread waits for about three load latencies instead of
// a few per child.  (The down sweep keeps its per-child loop: batched the
// same way it measured slower, its stores and rank chain per child.)
constexpr int kSweepBatch = 4;
__device__ __forceinline__ bool nch_internal(uint8_t k) { return k >= 1 && k < kNchPP; }

__device__ __forceinline__ void up_node_batched(const ExtArgs& a, int64_t x, uint32_t* sub_cnt,
                                                int& cyc) {
  const uint8_t k = a.t.nch[x];
  uint32_t c = 0;
  if (k >= kNchPP) {
    c = 1;
    cyc += k == kNchCycle ? 1 : 0;
  } else if (k) {
    const int64_t c0 = a.t.cstart[x];
    for (int j0 = 0; j0 < k; j0 += kSweepBatch) {
      uint8_t ky[kSweepBatch];
      int64_t cs[kSweepBatch];
#pragma unroll
      for (int j = 0; j < kSweepBatch; ++j) {
        const bool in = j0 + j < k;
        ky[j] = in ? a.t.nch[c0 + j0 + j] : (uint8_t)0;
        cs[j] = in ? (int64_t)a.t.cstart[c0 + j0 + j] : 0;
      }
      uint32_t cy[kSweepBatch];
#pragma unroll
      for (int j = 0; j < kSweepBatch; ++j) {
        cy[j] = ky[j] >= kNchPP ? 1u : 0u;
        cyc += ky[j] == kNchCycle ? 1 : 0;
      }
      for (int g0 = 0;; g0 += kSweepBatch) {
        uint32_t v[kSweepBatch][kSweepBatch];
#pragma unroll
        for (int j = 0; j < kSweepBatch; ++j)
#pragma unroll
          for (int g = 0; g < kSweepBatch; ++g)
            v[j][g] = nch_internal(ky[j]) && g0 + g < ky[j] ? sub_cnt[cs[j] + g0 + g] : 0u;
        bool more = false;
#pragma unroll
        for (int j = 0; j < kSweepBatch; ++j) {
#pragma unroll
          for (int g = 0; g < kSweepBatch; ++g) cy[j] += v[j][g];
          more |= nch_internal(ky[j]) && g0 + kSweepBatch < ky[j];
        }
        if (!more) break;
      }
#pragma unroll
      for (int j = 0; j < kSweepBatch; ++j) {
        if (j0 + j < k) {
          sub_cnt[c0 + j0 + j] = cy[j];
          c += cy[j];
        }
      }
    }
  }
  sub_cnt[x] = c;
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_up_run(ExtArgs a, int64_t base, int64_t F,
                                                   uint32_t* sub_cnt,
                                                   unsigned long long* n_cycles) {
  __shared__ int32_t s_w[kBlock / 64];
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int cyc = 0;
  if (j < F) {
    if constexpr (D == 1)
      up_node_batched(a, base + j, sub_cnt, cyc);
    else
      up_node<D>(a, base + j, sub_cnt, cyc);
  }
  int32_t tot;
  block_excl_scan<kBlock, int32_t>(cyc, tot, s_w);
  if (threadIdx.x == 0 && tot) atomicAdd(n_cycles + blockIdx.x % kCycleSlots, (unsigned long long)tot);
}

hipError_t launch_up_run(const ExtArgs& a, int depth, int64_t base, int64_t F, uint32_t* sub_cnt,
                         unsigned long long* n_cycles, hipStream_t st) {
  if (F == 0) return hipSuccess;
  const unsigned grid = (unsigned)((F + kBlock - 1) / kBlock);
  if (depth == 1)
    k_up_run<1><<<grid, kBlock, 0, st>>>(a, base, F, sub_cnt, n_cycles);
  else if (depth == 2)
    k_up_run<2><<<grid, kBlock, 0, st>>>(a, base, F, sub_cnt, n_cycles);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// x (level L, rank r, nch code k) hands ranks to its children; with D > 0
// each ranked internal child then does the same for its own children.
template <int D>
__device__ __forceinline__ void down_node(const ExtArgs& a, int L, int64_t x, uint8_t k,
                                          uint32_t r, uint32_t* sub_cnt, int64_t* leaf_by_rank,
                                          int32_t* pp_len) {
  if (k == 0 || k >= kNchPP) return;
  const int64_t c0 = a.t.cstart[x], c1 = c0 + k;
  for (int64_t y = c0; y < c1; ++y) {
    const uint32_t cc = sub_cnt[y];
    const uint8_t ky = a.t.nch[y];
    sub_cnt[y] = cc ? r : kNoRank;
    if (cc) {
      if (ky >= kNchPP) {
        leaf_by_rank[r] = y;
        pp_len[r] = L + 1;
      } else if constexpr (D > 0) {
        down_node<D - 1>(a, L + 1, y, ky, r, sub_cnt, leaf_by_rank, pp_len);
      }
    }
    r += cc;
  }
}

// Parents of levels L .. L + D in one launch (thread per node of L).
template <int D>
__global__ __launch_bounds__(kBlock) void k_down_run(ExtArgs a, int L, int64_t base, int64_t F,
                                                     uint32_t* sub_cnt, int64_t* leaf_by_rank,
                                                     int32_t* pp_len) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= F) return;
  const uint32_t r = sub_cnt[base + j];
  if (r != kNoRank) down_node<D>(a, L, base + j, a.t.nch[base + j], r, sub_cnt, leaf_by_rank, pp_len);
}

hipError_t launch_down_run(const ExtArgs& a, int depth, int L, int64_t base, int64_t F,
                           uint32_t* sub_cnt, int64_t* leaf_by_rank, int32_t* pp_len,
                           hipStream_t st) {
  if (F == 0) return hipSuccess;
  const unsigned grid = (unsigned)((F + kBlock - 1) / kBlock);
  if (depth == 1)
    k_down_run<1><<<grid, kBlock, 0, st>>>(a, L, base, F, sub_cnt, leaf_by_rank, pp_len);
  else if (depth == 2)
    k_down_run<2><<<grid, kBlock, 0, st>>>(a, L, base, F, sub_cnt, leaf_by_rank, pp_len);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Each wave writes the prime paths of 64 consecutive ranks, one per lane, by
// walking parent links from their leaves.  The walks are aligned by depth: a
// lane starts when the wave reaches the depth of its leaf, so at every step
// the active lanes stand on one tree level, mostly at nodes close together
// in that level's array (consecutive ranks are neighbours in depth-first
// order, and a tile's children are stored in its parents' order), and a load
// touches few cache lines.  The entries of kPPSeg consecutive depths
// go to LDS, one row per lane; then the wave stores the rows, kPPSeg lanes
// per row, so that a store covers a few whole row segments instead of one
// word in each of 64 lines.  With the BFS tables given, the walk also checks
// each entry against the BFS parent of the one after it and records the test
// path's length and where the path leaves the BFS tree, with the entries on
// either side of that point and the first vertex, from which the test-path
// keys are built.
constexpr int kPPSeg = 16;
constexpr int kPPRow = kPPSeg + 1;  // LDS row stride (odd: rows fall in different banks)

__global__ __launch_bounds__(kBlock) void k_pp_write(ExtArgs a, const int64_t* leaf_by_rank,
                                                     const int64_t* pp_off, int64_t n_pp,
                                                     int32_t* pp_vtx, PPWriteTp tp) {
  __shared__ int32_t s_row[kBlock * kPPRow];
  __shared__ int64_t s_lo[kBlock];
  __shared__ int32_t s_len[kBlock];
  __shared__ int32_t s_done[kBlock];
  const int tid = (int)threadIdx.x, lane = lane_id(), wb = tid - lane;
  const int64_t i = (int64_t)blockIdx.x * kBlock + tid;
  int64_t lo = 0;
  int32_t len = 0;
  int32_t x = -1;
  if (i < n_pp) {
    lo = pp_off[i];
    len = (int32_t)(pp_off[i + 1] - lo);
    x = (int32_t)leaf_by_rank[i];
  }
  s_lo[tid] = lo;
  s_len[tid] = len;
  int32_t lmax = len;  // the wave's longest path
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const int32_t y = __shfl_xor(lmax, d, 64);
    lmax = y > lmax ? y : lmax;
  }
  const bool with_tp = tp.tp_len != nullptr;
  int32_t done = len;  // entries done .. len - 1 are walked
  int32_t nxt = -1, vk = -1, lead = len;  // the entry after the current one; the last entry
  int32_t pn = -1;                        // BFS parent of nxt
  int32_t lw = -1, le = -1;               // the entries at lead - 1 and lead
  int32_t* row = s_row + tid * kPPRow;
  for (int kb = lmax > 0 ? (lmax - 1) / kPPSeg * kPPSeg : -1; kb >= 0; kb -= kPPSeg) {
    // depths kb + kPPSeg - 1 down to kb: one dependent load per step
    const int32_t top = done;
    int32_t v[kPPSeg];
#pragma unroll
    for (int m = kPPSeg - 1; m >= 0; --m) {
      const int k = kb + m;
      v[m] = -1;
      if (k < len && x >= 0) {
        v[m] = node_v(a.t.info[x]);
        x = a.t.par[x];
        done = k;
      }
    }
#pragma unroll
    for (int m = 0; m < kPPSeg; ++m) row[m] = v[m];
    if (with_tp) {
      // the BFS parents of the round's entries, loaded together, then the
      // pairs (entry k, entry k + 1) checked from the last one down
      int32_t pv[kPPSeg];
#pragma unroll
      for (int m = 0; m < kPPSeg; ++m) {
        const int k = kb + m;
        pv[m] = k >= done && k < top ? tp.parent[v[m]] : -1;
      }
#pragma unroll
      for (int m = kPPSeg - 1; m >= 0; --m) {
        const int k = kb + m;
        if (k >= done && k < top) {
          if (nxt < 0) vk = v[m];
          else if (pn != v[m]) {
            lead = k + 1;
            lw = v[m];
            le = nxt;
          }
          nxt = v[m];
          pn = pv[m];
        }
      }
    }
    s_done[tid] = done;
    wave_sync();
    // the wave's rows, kPPSeg lanes per row: depths kb .. kb + kPPSeg - 1 of
    // each path, those walked in this round
#pragma unroll
    for (int r0 = 0; r0 < 64; r0 += 64 / kPPSeg) {
      const int r = wb + r0 + lane / kPPSeg, k = kb + lane % kPPSeg;
      if (k >= s_done[r] && k < s_len[r]) pp_vtx[s_lo[r] + k] = s_row[r * kPPRow + (k - kb)];
    }
    wave_sync();  // the rows are read before the next round writes them
  }
  if (with_tp && nxt >= 0) {
    const int32_t v1 = nxt;
    const int64_t lp = tp.pfx_off[v1 + 1] - tp.pfx_off[v1];
    tp.tp_len[i] = lp + len + (tp.sfx_off[vk + 1] - tp.sfx_off[vk]);
    tp.lead[i] = make_int4(lead, lw, le, v1);
  }
}

hipError_t launch_pp_write(const ExtArgs& a, const int64_t* leaf_by_rank, const int64_t* pp_off,
                           int64_t n_pp, int32_t* pp_vtx, const PPWriteTp& tp, hipStream_t st) {
  if (n_pp == 0) return hipSuccess;
  k_pp_write<<<(unsigned)((n_pp + kBlock - 1) / kBlock), kBlock, 0, st>>>(a, leaf_by_rank, pp_off,
                                                                          n_pp, pp_vtx, tp);
  return hipGetLastError();
}

}  // namespace tpg

namespace tpg {

// After the ranks and the offsets exist: first prime path of each component
// (its first root's rank) and the offset of that path's first entry.
__global__ void k_comp_pp_starts(DGraph g, const uint32_t* sub_cnt, const int64_t* pp_off,
                                 const int64_t* totals, int64_t* pp_start, int64_t* ppv_start) {
  const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (c < g.n_comp) {
    const int64_t r = sub_cnt[g.cbase[c]];
    pp_start[c] = r;
    ppv_start[c] = pp_off[r];
  }
  if (c == g.n_comp) {
    pp_start[c] = totals[0];
    ppv_start[c] = pp_off[totals[0]];
  }
}

hipError_t launch_comp_pp_starts(const DGraph& g, const uint32_t* sub_cnt, const int64_t* pp_off,
                                 const int64_t* totals, int64_t* pp_start, int64_t* ppv_start,
                                 hipStream_t st) {
  k_comp_pp_starts<<<(unsigned)((g.n_comp + 1 + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      g, sub_cnt, pp_off, totals, pp_start, ppv_start);
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
