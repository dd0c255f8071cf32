// Device-side building blocks shared by the kernels of libtpg (gfx950,
// wave64): node encoding, wave/block scans, visited-set bit tests.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tpg {

constexpr int kBlock = 256;  // threads per workgroup for path kernels (4 waves)

// A path-tree node is stored as two 32-bit words:
//   par  : global index of the parent node (-1 for a single-vertex path)
//   info : last vertex, graph-wide id (bits 0-16) | first vertex, id local to
//          its component (bits 17-28) | flags (bits 29-31)
// Several CFGs can be processed as one disjoint union ("components"); a
// visited set indexes the local ids of the path's own component.
constexpr uint32_t kVMask = 0x1FFFFu;
constexpr int kV1Shift = 17;
constexpr uint32_t kV1Mask = 0xFFFu;
constexpr uint32_t F_CYC = 1u << 29;   // closes a cycle (last vertex = first)
// F_PP and F_TERM live only in registers while a level is extended; the
// stored leaf kind is the node's nch code
constexpr uint32_t F_PP = 1u << 30;    // prime path leaf (terminal and not backward-extendable)
constexpr uint32_t F_TERM = 1u << 31;  // acyclic, cannot be extended forward
constexpr int kMaxUnionVertices = 1 << 17;

__device__ __forceinline__ int node_v(uint32_t info) { return (int)(info & kVMask); }
__device__ __forceinline__ int node_v1l(uint32_t info) { return (int)((info >> kV1Shift) & kV1Mask); }
__device__ __forceinline__ uint32_t make_info(int v, int v1l, uint32_t flags) {
  return (uint32_t)v | ((uint32_t)v1l << kV1Shift) | flags;
}

// A node's child count with its leaf kind folded in, so that the ranking
// sweeps read one byte per node: a node with children stores their number
// (1..64); a leaf stores kNchCycle for a closed cycle, kNchPP for an acyclic
// prime path and 0 for a terminal path that is not prime.
constexpr uint8_t kNchPP = 254;
constexpr uint8_t kNchCycle = 255;
__device__ __forceinline__ uint8_t nch_code(uint32_t info, int nchildren) {
  return nchildren ? (uint8_t)nchildren
                   : (info & F_CYC) ? kNchCycle : (info & F_PP) ? kNchPP : (uint8_t)0;
}

struct DGraph {
  const int32_t* sp;    // successor row pointers [n+1] (graph-wide ids)
  const int32_t* s;     // successors, ascending per row
  const int32_t* pp;    // predecessor row pointers [n+1]
  const int32_t* p;     // predecessors
  const int32_t* loc;   // [n] id of each vertex inside its component
  const int32_t* comp;  // [n] component of each vertex
  const int32_t* cbase; // [n_comp+1] first graph-wide id of each component
  const int32_t* centry;// [n_comp] entry (graph-wide id)
  const int32_t* cexit; // [n_comp] exit (graph-wide id)
  int32_t n, n_comp;
  // sp, s, pp, p and loc lie back to back in one buffer starting at sp:
  // int32 words from sp through the end of loc (what a kernel stages in LDS)
  int32_t n_stage;
};

// Largest CSR (sp .. loc, bytes) that the extension kernel stages in LDS.
constexpr int kGraphLdsBytes = 16384;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

template <class T>
__device__ __forceinline__ T wave_incl_scan(T x) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T y = __shfl_up(x, d, 64);
    if (lane_id() >= d) x += y;
  }
  return x;
}

// Words 0 and 1 of a test path's comparison key, from where the path leaves
// the BFS tree: w, the tree path's last vertex, at entry index first - 1;
// the entry e after it (has_e: the path goes on past w); v1, the prime
// path's first vertex.  Word 0: pre(w) | pend(w) << 18 | (first - 1) << 36 |
// has_e << 49.  Word 1: e | split << 17 | pre(v1) << 35, where split is the
// preorder rank of w's first tree child with an id above e (pend(w) if none;
// pre(w) + 1 without e).  pre, pend: BFS-tree preorder ranks; w's tree
// children are bq[cfirst[w] .. cfirst[w] + ccnt[w]), ascending.  kk: 16-byte
// aligned.
__device__ __forceinline__ void tp_tree_key(const int32_t* pre, const int32_t* pend,
                                            const int32_t* cfirst, const int32_t* ccnt,
                                            const int32_t* bq, int w, int first, bool has_e,
                                            int ev, int v1, uint64_t* kk) {
  const uint32_t prew = (uint32_t)pre[w], pendw = (uint32_t)pend[w];
  uint32_t split;
  if (has_e) {
    split = pendw;
    const int cf = cfirst[w], cn = ccnt[w];
    // the children eight at a time, their loads in flight together
    for (int q0 = 0; q0 < cn; q0 += 8) {
      int cv[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) cv[j] = q0 + j < cn ? bq[cf + q0 + j] : -1;
      int hit = -1;
#pragma unroll
      for (int j = 7; j >= 0; --j)
        if (cv[j] > ev) hit = cv[j];
      if (hit >= 0) {
        split = (uint32_t)pre[hit];
        break;
      }
    }
  } else {
    split = prew + 1;
  }
  // one 16-byte store (kk is 16-byte aligned)
  ulonglong2 kw;
  kw.x = (uint64_t)prew | ((uint64_t)pendw << 18) | ((uint64_t)(first - 1) << 36) |
         ((uint64_t)(has_e ? 1 : 0) << 49);
  kw.y = (uint64_t)(uint32_t)(has_e ? ev : 0) | ((uint64_t)split << 17) |
         ((uint64_t)(uint32_t)pre[v1] << 35);
  *reinterpret_cast<ulonglong2*>(kk) = kw;
}

// Orders the LDS accesses of one wave's lanes: what a lane wrote before it is
// seen by the other lanes of its wave after it (a wave runs in lockstep; this
// keeps the compiler from moving LDS accesses across it and waits for them).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exclusive scan across a workgroup of NT threads; s_w needs NT/64 slots.
template <int NT, class T>
__device__ __forceinline__ T block_excl_scan(T x, T& total, T* s_w) {
  T inc = wave_incl_scan(x);
  const int w = (int)(threadIdx.x >> 6);
  if (lane_id() == 63) s_w[w] = inc;
  __syncthreads();
  T pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    T v = s_w[i];
    pre += (i < w) ? v : (T)0;
    tot += v;
  }
  __syncthreads();
  total = tot;
  return pre + inc - x;
}

// Visited-set bit test on a register-resident mask of W 64-bit words.
template <int W>
__device__ __forceinline__ bool mask_has(const uint64_t (&m)[W], int w) {
  const int q = w >> 6;
  uint64_t word = 0;
#pragma unroll
  for (int k = 0; k < W; ++k) word = (k == q) ? m[k] : word;
  return (word >> (w & 63)) & 1ull;
}

// r-th set bit (0-based) of x; x has more than r set bits.
__device__ __forceinline__ int select_bit(uint64_t x, int r) {
  for (int i = 0; i < r; ++i) x &= x - 1;
  return __builtin_ctzll(x);
}

}  // namespace tpg
