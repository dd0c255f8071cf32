// The paper's own schedule, kept as a comparison variant (Sec. 5, the
// Update-Vertex kernel and its ExtendPath step): every vertex owns a list of
// whole paths that end at it, one thread per vertex extends the paths its
// predecessors added last, and no atomic is used (a row's "extended" mark is
// a plain store of 1 by whichever successor extends it).  The paper runs the
// threads asynchronously until no list changes; here each round is one pair
// of launches (count, then fill) that every vertex takes part in, so no
// thread waits on another.  Round L holds the paths with L entries, as rows
// of L int32; rows of vertex v are rows voff[v] .. voff[v + 1] - 1.
#include "device.h"
#include "kernels.h"

namespace tpg {

// q (a row ending at a predecessor of v) may be extended by v when q is not a
// cycle and v is absent from q or is its first entry (then q + v is a cycle).
__device__ __forceinline__ bool pv_eligible(const int32_t* q, int L, int v) {
  if (L > 1 && q[0] == q[L - 1]) return false;
  for (int k = 1; k < L; ++k)
    if (q[k] == v) return false;
  return true;
}

__global__ __launch_bounds__(kBlock) void k_pv_init(int n, int64_t* voff, int32_t* rows) {
  const int v = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (v < n) {
    rows[v] = v;
    voff[v] = v;
  }
  if (v == n) voff[n] = n;
}

// cnt[v] = paths of round L + 1 that end at v.
__global__ __launch_bounds__(kBlock) void k_pv_count(DGraph g, int L, const int64_t* voff,
                                                     const int32_t* rows, int32_t* cnt) {
  const int v = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (v >= g.n) return;
  int32_t c = 0;
  for (int e = g.pp[v]; e < g.pp[v + 1]; ++e) {
    const int u = g.p[e];
    for (int64_t q = voff[u]; q < voff[u + 1]; ++q) c += pv_eligible(rows + q * L, L, v) ? 1 : 0;
  }
  cnt[v] = c;
}

// Writes v's rows of round L + 1 (from nvoff[v] on) and marks every row of
// round L that some successor extends.
__global__ __launch_bounds__(kBlock) void k_pv_fill(DGraph g, int L, const int64_t* voff,
                                                    const int32_t* rows, uint8_t* extended,
                                                    const int64_t* nvoff, int32_t* nrows) {
  const int v = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (v >= g.n) return;
  int64_t j = nvoff[v];
  for (int e = g.pp[v]; e < g.pp[v + 1]; ++e) {
    const int u = g.p[e];
    for (int64_t q = voff[u]; q < voff[u + 1]; ++q) {
      const int32_t* src = rows + q * L;
      if (!pv_eligible(src, L, v)) continue;
      int32_t* dst = nrows + j * (L + 1);
      for (int k = 0; k < L; ++k) dst[k] = src[k];
      dst[L] = v;
      extended[q] = 1;
      ++j;
    }
  }
}

// flag[i] = row i of round L is prime: a cycle, or neither extended by a
// successor nor extendable backwards (a predecessor of its first entry that
// is absent from it, or that is its last entry, closing a cycle).
__global__ __launch_bounds__(kBlock) void k_pv_prime(DGraph g, int L, const int32_t* rows,
                                                     const uint8_t* extended, int64_t n_rows,
                                                     int32_t* flag) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n_rows) return;
  const int32_t* r = rows + i * L;
  const int a = r[0], b = r[L - 1];
  int prime = 1;
  if (!(L > 1 && a == b)) {
    if (extended[i]) {
      prime = 0;
    } else {
      for (int e = g.pp[a]; e < g.pp[a + 1] && prime; ++e) {
        const int w = g.p[e];
        bool in = false;
        for (int k = 0; k < L && !in; ++k) in = r[k] == w;
        if (w == b || !in) prime = 0;
      }
    }
  }
  flag[i] = prime;
}

// The prime rows of round L, appended in row order: path base + pos[i] gets
// entries at voff0 + pos[i] * L.
__global__ __launch_bounds__(kBlock) void k_pv_emit(int L, const int32_t* rows,
                                                    const int32_t* flag, const int64_t* pos,
                                                    int64_t n_rows, int64_t base, int64_t voff0,
                                                    int64_t* out_off, int32_t* out_vtx) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n_rows || !flag[i]) return;
  const int64_t o = voff0 + pos[i] * L;
  out_off[base + pos[i]] = o;
  for (int k = 0; k < L; ++k) out_vtx[o + k] = rows[i * L + k];
}

hipError_t launch_pv_init(int n, int64_t* voff, int32_t* rows, hipStream_t st) {
  k_pv_init<<<(unsigned)((n + 1 + kBlock - 1) / kBlock), kBlock, 0, st>>>(n, voff, rows);
  return hipGetLastError();
}

hipError_t launch_pv_count(const DGraph& g, int L, const int64_t* voff, const int32_t* rows,
                           int32_t* cnt, hipStream_t st) {
  k_pv_count<<<(unsigned)((g.n + kBlock - 1) / kBlock), kBlock, 0, st>>>(g, L, voff, rows, cnt);
  return hipGetLastError();
}

hipError_t launch_pv_fill(const DGraph& g, int L, const int64_t* voff, const int32_t* rows,
                          uint8_t* extended, const int64_t* nvoff, int32_t* nrows,
                          hipStream_t st) {
  k_pv_fill<<<(unsigned)((g.n + kBlock - 1) / kBlock), kBlock, 0, st>>>(g, L, voff, rows, extended,
                                                                        nvoff, nrows);
  return hipGetLastError();
}

hipError_t launch_pv_prime(const DGraph& g, int L, const int32_t* rows, const uint8_t* extended,
                           int64_t n_rows, int32_t* flag, hipStream_t st) {
  if (n_rows == 0) return hipSuccess;
  k_pv_prime<<<(unsigned)((n_rows + kBlock - 1) / kBlock), kBlock, 0, st>>>(g, L, rows, extended,
                                                                           n_rows, flag);
  return hipGetLastError();
}

hipError_t launch_pv_emit(int L, const int32_t* rows, const int32_t* flag, const int64_t* pos,
                          int64_t n_rows, int64_t base, int64_t voff0, int64_t* out_off,
                          int32_t* out_vtx, hipStream_t st) {
  if (n_rows == 0) return hipSuccess;
  k_pv_emit<<<(unsigned)((n_rows + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      L, rows, flag, pos, n_rows, base, voff0, out_off, out_vtx);
  return hipGetLastError();
}

}  // namespace tpg
