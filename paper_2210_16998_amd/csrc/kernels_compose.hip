// The compositional method of Sec. 2.1 on the device: the component graph's
// arcs (Def. 3), the extraction of SccEntryExitPaths, SccExitPaths and
// SccEntryPaths (Defs. 6-8) from path trees of the components with a cycle,
// and the classification of the merged paths.
//
// Extraction.  The components with a cycle, each taken alone (its vertices
// and the arcs between them), form one disjoint union whose path tree holds
// every simple path inside a component from every vertex (the extension
// kernels build it).  A node's path is acyclic unless it closed a cycle.
//  * Forward tree: a node from an SccEntryVertex to an SccExitVertex is an
//    SccEntryExitPath; one from an SccEntryVertex to another vertex is an
//    entry path, and an SccEntryPath when no descendant is an entry path
//    (Def. 8, maximal among the entry paths from the same vertex: a longer
//    entry path from the same vertex that contains it extends it forward).
//  * Tree of the reversed components: a node is a reversed exit path when
//    its root is an SccExitVertex and its last vertex is not an
//    SccEntryVertex, and the reversal of an SccExitPath when no descendant
//    is one (Def. 7, maximal among the exit paths to the same vertex).
// The marks go bottom-up over the levels with the number of emitted nodes
// in every subtree; ranks then go top-down in preorder, which is the
// lexicographic order of the paths in the tree's vertex order.
#include "kernels.h"

namespace tpg {

// ---------------------------------------------------------------------------
// component graph: the arcs of g between different components
// ---------------------------------------------------------------------------
__global__ void k_ccfg_count(DGraph g, const int32_t* comp, int32_t* cnt) {
  const int u = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (u >= g.n) return;
  int c = 0;
  for (int k = g.sp[u]; k < g.sp[u + 1]; ++k) c += comp[g.s[k]] != comp[u] ? 1 : 0;
  cnt[u] = c;
}

__global__ void k_ccfg_write(DGraph g, const int32_t* comp, const int64_t* off, int32_t* src,
                             int32_t* dst) {
  const int u = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (u >= g.n) return;
  int64_t o = off[u];
  for (int k = g.sp[u]; k < g.sp[u + 1]; ++k) {
    const int w = g.s[k];
    if (comp[w] != comp[u]) {
      src[o] = u;
      dst[o] = w;
      ++o;
    }
  }
}

hipError_t launch_ccfg_count(const DGraph& g, const int32_t* comp, int32_t* cnt, hipStream_t st) {
  if (g.n <= 0) return hipSuccess;
  k_ccfg_count<<<(unsigned)((g.n + kBlock - 1) / kBlock), kBlock, 0, st>>>(g, comp, cnt);
  return hipGetLastError();
}

hipError_t launch_ccfg_write(const DGraph& g, const int32_t* comp, const int64_t* off, int32_t* src,
                             int32_t* dst, hipStream_t st) {
  if (g.n <= 0) return hipSuccess;
  k_ccfg_write<<<(unsigned)((g.n + kBlock - 1) / kBlock), kBlock, 0, st>>>(g, comp, off, src, dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// extraction marks
// ---------------------------------------------------------------------------
// vfl[v] (union vertex): bit 0 SccEntryVertex, bit 1 SccExitVertex in g.
// Qualification bits of node x: mode 0 (forward) bit 0 = entry -> exit,
// bit 1 = entry path; mode 1 (reversed) bit 0 = reversed exit path.
__device__ __forceinline__ uint8_t ex_qual(const ExtArgs& a, int64_t x, const uint8_t* vfl,
                                           int mode) {
  const uint32_t inf = a.t.info[x];
  if (inf & F_CYC) return 0;
  const int v = node_v(inf);
  const int first = v - a.g.loc[v] + node_v1l(inf);
  const uint8_t fa = vfl[first], fb = vfl[v];
  if (mode == 0)
    return (uint8_t)(((fa & 1) && (fb & 2) ? 1 : 0) | ((fa & 1) && !(fb & 2) ? 2 : 0));
  return (uint8_t)(((fa & 2) && !(fb & 1)) ? 1 : 0);
}

// Emitted in set s: mode 0 set 0 every entry -> exit path, set 1 the entry
// paths with no entry path below; mode 1 set 0 the reversed exit paths with
// none below.  qb = qualification bits | (bits of the subtree below) << 4.
__device__ __forceinline__ uint32_t ex_emit(uint8_t qb, int mode, int set) {
  const uint8_t q = qb & 15, b = qb >> 4;
  if (mode == 0 && set == 0) return q & 1;
  if (mode == 0) return ((q & 2) && !(b & 2)) ? 1u : 0u;
  return ((q & 1) && !(b & 1)) ? 1u : 0u;
}

// Level L, bottom-up (its children's marks exist): marks and emitted counts.
__global__ __launch_bounds__(kBlock) void k_ex_up(ExtArgs a, int64_t base, int64_t F,
                                                  const uint8_t* vfl, int mode, uint8_t* qb,
                                                  uint32_t* cnt0, uint32_t* cnt1) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= F) return;
  const int64_t x = base + j;
  const uint8_t k = a.t.nch[x];
  uint8_t below = 0;
  uint32_t c0 = 0, c1 = 0;
  if (k > 0 && k < kNchPP) {
    const int64_t y0 = a.t.cstart[x];
    for (int64_t y = y0; y < y0 + k; ++y) {
      const uint8_t qy = qb[y];
      below |= (uint8_t)((qy & 15) | (qy >> 4));
      c0 += cnt0[y];
      if (cnt1) c1 += cnt1[y];
    }
  }
  const uint8_t q = (uint8_t)(ex_qual(a, x, vfl, mode) | (below << 4));
  qb[x] = q;
  cnt0[x] = c0 + ex_emit(q, mode, 0);
  if (cnt1) cnt1[x] = c1 + ex_emit(q, mode, 1);
}

constexpr uint32_t kExNoRank = 0xFFFFFFFFu;

// Level-1 nodes: exclusive scan of their subtree counts = the rank of the
// subtree's first emitted path (kExNoRank when it has none); total[0] = all.
// One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_ex_roots(uint32_t* cnt, int64_t n_roots,
                                                   int64_t* total) {
  __shared__ int64_t s_w[16];
  int64_t carry = 0;
  for (int64_t b = 0; b < n_roots; b += 1024) {
    const int64_t i = b + threadIdx.x;
    const int64_t c = i < n_roots ? (int64_t)cnt[i] : 0;
    int64_t tc;
    const int64_t pc = block_excl_scan<1024, int64_t>(c, tc, s_w);
    if (i < n_roots) cnt[i] = c ? (uint32_t)(carry + pc) : kExNoRank;
    carry += tc;
  }
  if (threadIdx.x == 0) total[0] = carry;
}

// Level L, top-down: a node with a rank records itself when emitted and
// hands ranks to its children in slot order (cnt becomes ranks in place).
__global__ __launch_bounds__(kBlock) void k_ex_down(ExtArgs a, int L, int64_t base, int64_t F,
                                                    const uint8_t* qb, uint32_t* cnt, int mode,
                                                    int set, int64_t* out_node, int32_t* out_len) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= F) return;
  const int64_t x = base + j;
  uint32_t r = cnt[x];
  if (r == kExNoRank) return;
  if (ex_emit(qb[x], mode, set)) {
    out_node[r] = x;
    out_len[r] = L;
    ++r;
  }
  const uint8_t k = a.t.nch[x];
  if (k == 0 || k >= kNchPP) return;
  const int64_t y0 = a.t.cstart[x];
  for (int64_t y = y0; y < y0 + k; ++y) {
    const uint32_t cc = cnt[y];
    cnt[y] = cc ? r : kExNoRank;
    r += cc;
  }
}

// Path i: its node's entries, mapped to g's ids by orig[]; reversed = 0
// stores them root first (the tree's path), 1 leaf first (a reversed tree's
// node gives the exit path in its own direction).
__global__ __launch_bounds__(kBlock) void k_ex_write(ExtArgs a, const int64_t* out_node,
                                                     const int64_t* off, int64_t n, int reversed,
                                                     const int32_t* orig, int32_t* vtx) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int64_t x = out_node[i];
  const int64_t o0 = off[i], o1 = off[i + 1];
  for (int64_t k = 0; k < o1 - o0 && x >= 0; ++k) {
    const int32_t v = orig[node_v(a.t.info[x])];
    vtx[reversed ? o0 + k : o1 - 1 - k] = v;
    x = a.t.par[x];
  }
}

hipError_t launch_ex_up(const ExtArgs& a, int64_t base, int64_t F, const uint8_t* vfl, int mode,
                        uint8_t* qb, uint32_t* cnt0, uint32_t* cnt1, hipStream_t st) {
  if (F == 0) return hipSuccess;
  k_ex_up<<<(unsigned)((F + kBlock - 1) / kBlock), kBlock, 0, st>>>(a, base, F, vfl, mode, qb,
                                                                    cnt0, cnt1);
  return hipGetLastError();
}

hipError_t launch_ex_roots(uint32_t* cnt, int64_t n_roots, int64_t* total, hipStream_t st) {
  k_ex_roots<<<1, 1024, 0, st>>>(cnt, n_roots, total);
  return hipGetLastError();
}

hipError_t launch_ex_down(const ExtArgs& a, int L, int64_t base, int64_t F, const uint8_t* qb,
                          uint32_t* cnt, int mode, int set, int64_t* out_node, int32_t* out_len,
                          hipStream_t st) {
  if (F == 0) return hipSuccess;
  k_ex_down<<<(unsigned)((F + kBlock - 1) / kBlock), kBlock, 0, st>>>(a, L, base, F, qb, cnt, mode,
                                                                      set, out_node, out_len);
  return hipGetLastError();
}

hipError_t launch_ex_write(const ExtArgs& a, const int64_t* out_node, const int64_t* off,
                           int64_t n, int reversed, const int32_t* orig, int32_t* vtx,
                           hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_ex_write<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(a, out_node, off, n,
                                                                      reversed, orig, vtx);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// merged paths: classification of the macro graph's prime paths
// ---------------------------------------------------------------------------
// The merge runs the extension on a macro graph H whose prime paths are the
// merged candidates (see the host side); hkind[h] tells what H vertex h is:
// 0 a vertex of g outside the components with a cycle, 1 a node of a
// component's trie of paths from its SccEntryVertices, 2 a node of a trie
// of SccExitPaths, 3 the terminal mark that ends an SccEntryPath.  horig[h]
// is the vertex of g (none for a terminal mark).  Class of an H path:
// 1 complete (from the entry to the exit), 3 SccExitPP candidate (from an
// exit-path trie to the exit), 4 SccEntryPP candidate (from the entry to a
// terminal mark), 0 otherwise.  A candidate is kept when neither of its
// ends can be extended in g (the local prime test).  len: entries in g.
__global__ __launch_bounds__(kBlock) void k_merge_class(const int64_t* off, const int32_t* vtx,
                                                        int64_t n, const uint8_t* hkind,
                                                        const int32_t* horig, DGraph g,
                                                        int h_entry, int h_exit, uint8_t* cls,
                                                        int32_t* len) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t o0 = off[i], o1 = off[i + 1];
  const int a = vtx[o0], b = vtx[o1 - 1];
  uint8_t c = 0;
  int64_t e1 = o1;  // end of the entries that are vertices of g
  if (a == h_entry && b == h_exit) {
    c = 1;
  } else if (hkind[a] == 2 && b == h_exit) {
    c = 3;
  } else if (a == h_entry && hkind[b] == 3) {
    c = 4;
    e1 = o1 - 1;
  }
  if (c == 3 || c == 4) {
    // the local prime test in g: no predecessor of the first vertex and no
    // successor of the last one off the path
    const int u = horig[vtx[o0]], w = horig[vtx[e1 - 1]];
    bool ext = false;
    for (int k = g.pp[u]; k < g.pp[u + 1] && !ext; ++k) {
      const int p = g.p[k];
      bool on = false;
      for (int64_t q = o0; q < e1 && !on; ++q) on = horig[vtx[q]] == p;
      ext = !on;
    }
    for (int k = g.sp[w]; k < g.sp[w + 1] && !ext; ++k) {
      const int s = g.s[k];
      bool on = false;
      for (int64_t q = o0; q < e1 && !on; ++q) on = horig[vtx[q]] == s;
      ext = !on;
    }
    if (ext) c = 0;
  }
  cls[i] = c;
  len[i] = c ? (int32_t)(e1 - o0) : 0;
}

// Paths of class c, in order: entries mapped to g's vertices (pos: exclusive
// scan of the class flags, voff: of the lengths of the class's paths).
__global__ __launch_bounds__(kBlock) void k_merge_emit(const int64_t* off, const int32_t* vtx,
                                                       int64_t n, const uint8_t* cls, int c,
                                                       const int64_t* pos, const int64_t* voff,
                                                       const int32_t* len, const int32_t* horig,
                                                       int64_t* out_off, int32_t* out_vtx) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n || cls[i] != c) return;
  const int64_t o0 = off[i], d0 = voff[i];
  out_off[pos[i]] = d0;
  for (int32_t k = 0; k < len[i]; ++k) out_vtx[d0 + k] = horig[vtx[o0 + k]];
}

// Prime paths of the components with a cycle, each taken alone (union ids,
// vfl as for the extraction): class 1 for an SccInternalPP (Def. 9: a
// cycle, or an acyclic path that neither starts at an SccEntryVertex nor
// ends at an SccExitVertex), else 0.
__global__ void k_internal_class(const int64_t* off, const int32_t* vtx, int64_t n,
                                 const uint8_t* vfl, uint8_t* cls, int32_t* len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o0 = off[i], o1 = off[i + 1];
  const int a = vtx[o0], b = vtx[o1 - 1];
  const bool cyclic = o1 - o0 > 1 && a == b;
  const bool keep = cyclic || (!(vfl[a] & 1) && !(vfl[b] & 2));
  cls[i] = keep ? 1 : 0;
  len[i] = keep ? (int32_t)(o1 - o0) : 0;
}

hipError_t launch_internal_class(const int64_t* off, const int32_t* vtx, int64_t n,
                                 const uint8_t* vfl, uint8_t* cls, int32_t* len, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_internal_class<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(off, vtx, n, vfl, cls,
                                                                            len);
  return hipGetLastError();
}

// flag[i] = 1 and lens[i] = len[i] for the paths of class c, else 0.
__global__ void k_merge_sel(const uint8_t* cls, const int32_t* len, int64_t n, int c, int32_t* flag,
                            int32_t* lens) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool on = cls[i] == c;
  flag[i] = on ? 1 : 0;
  lens[i] = on ? len[i] : 0;
}

hipError_t launch_merge_sel(const uint8_t* cls, const int32_t* len, int64_t n, int c, int32_t* flag,
                            int32_t* lens, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_merge_sel<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(cls, len, n, c, flag, lens);
  return hipGetLastError();
}

hipError_t launch_merge_class(const int64_t* off, const int32_t* vtx, int64_t n,
                              const uint8_t* hkind, const int32_t* horig, const DGraph& g,
                              int h_entry, int h_exit, uint8_t* cls, int32_t* len, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_merge_class<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      off, vtx, n, hkind, horig, g, h_entry, h_exit, cls, len);
  return hipGetLastError();
}

hipError_t launch_merge_emit(const int64_t* off, const int32_t* vtx, int64_t n, const uint8_t* cls,
                             int c, const int64_t* pos, const int64_t* voff, const int32_t* len,
                             const int32_t* horig, int64_t* out_off, int32_t* out_vtx,
                             hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_merge_emit<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      off, vtx, n, cls, c, pos, voff, len, horig, out_off, out_vtx);
  return hipGetLastError();
}

}  // namespace tpg
