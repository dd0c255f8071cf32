// Strongly connected components and the prime-path types of Sec. 2 on the
// device: the component graph's vertices (Def. 3), SccEntryVertex and
// SccExitVertex (Defs. 4-5), and the types CompletePP, SccInternalPP,
// SccExitPP, SccEntryPP (Defs. 2, 9, 10, 11) of a prime-path set.
#include <climits>

#include "device.h"
#include "kernels.h"

namespace tpg {

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_fill_i32<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(p, v, n);
  return hipGetLastError();
}

// One thread per graph of the union (its vertices are the contiguous ids
// cbase[c] .. cbase[c + 1] - 1): Tarjan's depth-first search with explicit
// stacks.  CFGs are small and a batch holds many of them, so a thread per
// graph keeps the search sequential where it has to be and parallel across
// graphs.  Scratch w holds 6 n int32: index, low, on-stack, the component
// stack, and the call stack's vertices and next-arc positions; index must
// be -1 on entry.  comp[v] = the smallest vertex of v's component.
__global__ __launch_bounds__(kBlock) void k_scc_tarjan(DGraph g, int32_t* w, int32_t* comp) {
  const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (c >= g.n_comp) return;
  const int n = g.n;
  int32_t* index = w;
  int32_t* low = w + n;
  int32_t* on = w + 2 * (int64_t)n;
  int32_t* stk = w + 3 * (int64_t)n;
  int32_t* cv = w + 4 * (int64_t)n;
  int32_t* ce = w + 5 * (int64_t)n;
  const int v0 = g.cbase[c], v1 = g.cbase[c + 1];
  int next = 0, top = v0, csz = 0;  // stacks of graph c use slots v0 .. v1 - 1
  for (int root = v0; root < v1; ++root) {
    if (index[root] >= 0) continue;
    index[root] = low[root] = next++;
    stk[top++] = root;
    on[root] = 1;
    cv[v0 + csz] = root;
    ce[v0 + csz] = g.sp[root];
    ++csz;
    while (csz > 0) {
      const int v = cv[v0 + csz - 1];
      const int e = ce[v0 + csz - 1];
      if (e < g.sp[v + 1]) {
        ce[v0 + csz - 1] = e + 1;
        const int x = g.s[e];
        if (index[x] < 0) {
          index[x] = low[x] = next++;
          stk[top++] = x;
          on[x] = 1;
          cv[v0 + csz] = x;
          ce[v0 + csz] = g.sp[x];
          ++csz;
        } else if (on[x] && index[x] < low[v]) {
          low[v] = index[x];
        }
        continue;
      }
      --csz;  // v is finished
      if (csz > 0) {
        const int u = cv[v0 + csz - 1];
        if (low[v] < low[u]) low[u] = low[v];
      }
      if (low[v] == index[v]) {  // v roots a component: pop it
        int pos = top, m = INT_MAX, x;
        do {
          x = stk[--pos];
          if (x < m) m = x;
        } while (x != v);
        for (int i = pos; i < top; ++i) {
          comp[stk[i]] = m;
          on[stk[i]] = 0;
        }
        top = pos;
      }
    }
  }
}

// The same search for a single graph small enough for LDS: the workgroup
// copies the successor CSR in, then one thread runs the search on LDS
// arrays (each step's loads then take LDS latency instead of a trip to
// memory).  Dynamic LDS: sp (n + 1), s (m), index, low, on, stack, call
// stack (2 n) = 7 n + m + 1 int32.
__global__ __launch_bounds__(kBlock) void k_scc_tarjan_lds(DGraph g, int32_t m, int32_t* comp) {
  extern __shared__ int32_t s_mem[];
  const int n = g.n;
  int32_t* sp = s_mem;
  int32_t* sc = sp + n + 1;
  int32_t* index = sc + m;
  int32_t* low = index + n;
  int32_t* on = low + n;
  int32_t* stk = on + n;
  int32_t* cv = stk + n;
  int32_t* ce = cv + n;
  for (int i = threadIdx.x; i <= n; i += kBlock) sp[i] = g.sp[i];
  for (int i = threadIdx.x; i < m; i += kBlock) sc[i] = g.s[i];
  for (int i = threadIdx.x; i < n; i += kBlock) index[i] = -1;
  __syncthreads();
  if (threadIdx.x != 0) return;
  int next = 0, top = 0, csz = 0;
  for (int root = 0; root < n; ++root) {
    if (index[root] >= 0) continue;
    index[root] = low[root] = next++;
    stk[top++] = root;
    on[root] = 1;
    cv[csz] = root;
    ce[csz] = sp[root];
    ++csz;
    while (csz > 0) {
      const int v = cv[csz - 1];
      const int e = ce[csz - 1];
      if (e < sp[v + 1]) {
        ce[csz - 1] = e + 1;
        const int x = sc[e];
        if (index[x] < 0) {
          index[x] = low[x] = next++;
          stk[top++] = x;
          on[x] = 1;
          cv[csz] = x;
          ce[csz] = sp[x];
          ++csz;
        } else if (on[x] && index[x] < low[v]) {
          low[v] = index[x];
        }
        continue;
      }
      --csz;
      if (csz > 0) {
        const int u = cv[csz - 1];
        if (low[v] < low[u]) low[u] = low[v];
      }
      if (low[v] == index[v]) {
        int pos = top, mn = INT_MAX, x;
        do {
          x = stk[--pos];
          if (x < mn) mn = x;
        } while (x != v);
        for (int i = pos; i < top; ++i) {
          comp[stk[i]] = mn;
          on[stk[i]] = 0;
        }
        top = pos;
      }
    }
  }
}

// Per vertex: cyclic (an arc to its own component: the component has two or
// more vertices, each with an arc inside, or v has a self-loop), entry
// vertex (an arc from another component), exit vertex (an arc to another
// component); n_comp[0] += components (vertices that label their own).
__global__ __launch_bounds__(kBlock) void k_scc_flags(DGraph g, const int32_t* comp,
                                                      uint8_t* flags, int32_t* n_comp) {
  __shared__ int32_t s_w[kBlock / 64];
  const int v = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  int roots = 0;
  if (v < g.n) {
    const int cv = comp[v];
    uint8_t f = 0;
    for (int e = g.sp[v]; e < g.sp[v + 1]; ++e)
      f |= comp[g.s[e]] == cv ? (uint8_t)kSccCyclic : (uint8_t)kSccExitVertex;
    for (int e = g.pp[v]; e < g.pp[v + 1]; ++e)
      if (comp[g.p[e]] != cv) f |= (uint8_t)kSccEntryVertex;
    flags[v] = f;
    roots = cv == v ? 1 : 0;
  }
  int32_t tot;
  block_excl_scan<kBlock, int32_t>(roots, tot, s_w);
  if (threadIdx.x == 0 && tot) atomicAdd(n_comp, tot);
}

// Largest LDS the single-graph search takes (bytes).
constexpr int64_t kSccLdsBytes = 48 * 1024;

hipError_t launch_scc(const DGraph& g, int32_t m, int32_t* work, int32_t* comp, uint8_t* flags,
                      int32_t* n_comp, hipStream_t st) {
  if (g.n == 0) return hipSuccess;
  hipError_t e = launch_fill_i32(n_comp, 0, 1, st);
  if (e != hipSuccess) return e;
  const int64_t lds = 4 * (7 * (int64_t)g.n + m + 1);
  if (g.n_comp == 1 && lds <= kSccLdsBytes) {
    k_scc_tarjan_lds<<<1, kBlock, (size_t)lds, st>>>(g, m, comp);
  } else {
    e = launch_fill_i32(work, -1, g.n, st);  // index = -1
    if (e != hipSuccess) return e;
    k_scc_tarjan<<<(unsigned)((g.n_comp + kBlock - 1) / kBlock), kBlock, 0, st>>>(g, work, comp);
  }
  k_scc_flags<<<(unsigned)((g.n + kBlock - 1) / kBlock), kBlock, 0, st>>>(g, comp, flags, n_comp);
  return hipGetLastError();
}

// One thread per prime path: its type from its end vertices (a simple path
// whose ends lie in one component stays inside it), Defs. 2, 9, 10, 11 in
// that order of precedence; counts[t] += paths of type t.
__global__ __launch_bounds__(kBlock) void k_pp_types(DGraph g, const int32_t* comp,
                                                     const uint8_t* flags, const int64_t* off,
                                                     const int32_t* vtx, int64_t n_pp,
                                                     uint8_t* types, unsigned long long* counts) {
  __shared__ unsigned long long s_cnt[kPpTypes];
  const int tid = (int)threadIdx.x;
  if (tid < kPpTypes) s_cnt[tid] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kBlock + tid;
  if (i < n_pp) {
    const int64_t o0 = off[i], o1 = off[i + 1];
    const int a = vtx[o0], b = vtx[o1 - 1];
    const bool cyclic = o1 - o0 > 1 && a == b;
    const int gc = g.comp[a];  // graph of the union the path belongs to
    const uint8_t fa = flags[a], fb = flags[b];
    const bool in_cycle_a = fa & kSccCyclic, in_cycle_b = fb & kSccCyclic;
    uint8_t t;
    if (a == g.centry[gc] && b == g.cexit[gc])
      t = kPpComplete;
    else if (in_cycle_a && comp[a] == comp[b] &&
             (cyclic || !((fa & kSccEntryVertex) || (fb & kSccExitVertex))))
      t = kPpSccInternal;
    else if (in_cycle_a && b == g.cexit[gc])
      t = kPpSccExit;
    else if (a == g.centry[gc] && in_cycle_b)
      t = kPpSccEntry;
    else
      t = kPpOther;
    if (types) types[i] = t;
    atomicAdd(&s_cnt[t], 1ull);
  }
  __syncthreads();
  if (tid < kPpTypes && s_cnt[tid]) atomicAdd(&counts[tid], s_cnt[tid]);
}

hipError_t launch_pp_types(const DGraph& g, const int32_t* comp, const uint8_t* flags,
                           const int64_t* off, const int32_t* vtx, int64_t n_pp, uint8_t* types,
                           unsigned long long* counts, hipStream_t st) {
  hipError_t e = launch_zero_u64((uint64_t*)counts, kPpTypes, st);
  if (e != hipSuccess || n_pp == 0) return e;
  k_pp_types<<<(unsigned)((n_pp + kBlock - 1) / kBlock), kBlock, 0, st>>>(g, comp, flags, off, vtx,
                                                                          n_pp, types, counts);
  return hipGetLastError();
}

}  // namespace tpg
