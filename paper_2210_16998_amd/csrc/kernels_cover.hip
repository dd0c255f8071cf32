// Test paths by longest-first covering (the Ammann-Offutt generation the
// paper cites among the methods for TPs): prime paths are taken in order of
// decreasing length (ties: canonical order); a prime path already contained,
// as a contiguous subpath, in the test path of a prime path taken before it
// gets no test path of its own.
//
// How it runs on the device:
//  * every spliced test path t finds the prime paths it contains.  A prime
//    path is a simple path that cannot be extended either way, or a simple
//    cycle, so among the windows of t starting at position i only the
//    longest simple one, t[i..j), can be a prime path (a shorter simple
//    window is extended by t's next entry), or the cycle t[i..j] when
//    t[j] = t[i].  A two-pointer sweep with the window's vertex set in
//    registers visits these candidates in O(|t|), the local prime rule
//    (no successor of the last vertex outside the window or equal to the
//    first; every predecessor of the first vertex inside) accepts them, and
//    a hash table of the prime paths gives the accepted window's index.  The
//    table is exact for these lookups: an accepted window is a prime path,
//    and the table is built only when no two prime paths share a hash.
//  * The sequential rule "chosen iff no earlier chooser covers it" is
//    resolved in rounds: a path with a chosen earlier coverer is dropped, a
//    path whose earlier coverers are all dropped is chosen.  The first
//    undecided path in the order is decided in every round, so the rounds
//    end; in practice a handful suffice.  A round is one pass over the
//    covering pairs that only stores constant flags (a few short prime
//    paths are contained in most test paths, so per-path atomics or lists
//    would serialize), then one pass that decides.

#include "kernels.h"

namespace tpg {

namespace {

constexpr uint64_t kHashMul = 0x9E3779B97F4A7C15ull;  // odd multiplier of the polynomial hash

// Polynomial hash of a vertex sequence: h = h * mul + (v + 1), never 0.
__device__ __forceinline__ uint64_t seq_hash_step(uint64_t h, int32_t v, uint64_t mul) {
  return h * mul + (uint64_t)(v + 1);
}
__device__ __forceinline__ uint64_t seq_hash_fix(uint64_t h) { return h ? h : 1ull; }

__global__ __launch_bounds__(kBlock) void k_pp_hash_insert(const int64_t* off, const int32_t* vtx,
                                                           int64_t n, uint64_t mul,
                                                           unsigned long long* keys, int32_t* vals,
                                                           int64_t mask, unsigned long long* dups) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  uint64_t h = 0;
  for (int64_t k = off[i]; k < off[i + 1]; ++k) h = seq_hash_step(h, vtx[k], mul);
  h = seq_hash_fix(h);
  int64_t s = (int64_t)(h & (uint64_t)mask);
  for (int64_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long prev = atomicCAS(&keys[s], 0ull, (unsigned long long)h);
    if (prev == 0ull) {
      vals[s] = (int32_t)i;
      return;
    }
    if (prev == h) {  // two prime paths share this hash: the table cannot be used
      atomicAdd(dups, 1ull);
      return;
    }
    s = (s + 1) & mask;
  }
  atomicAdd(dups, 1ull);  // table full (cannot happen at load factor 1/2)
}

__device__ __forceinline__ int32_t table_find(const unsigned long long* keys, const int32_t* vals,
                                              int64_t mask, uint64_t h) {
  int64_t s = (int64_t)(h & (uint64_t)mask);
  for (int64_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long k = keys[s];
    if (k == h) return vals[s];
    if (k == 0ull) return -1;
    s = (s + 1) & mask;
  }
  return -1;
}

template <int W>
__device__ __forceinline__ bool set_has(const uint64_t (&m)[W], int l) {
  return mask_has<W>(m, l);
}
template <int W>
__device__ __forceinline__ void set_flip(uint64_t (&m)[W], int l) {
  const int q = l >> 6;
  const uint64_t bit = 1ull << (l & 63);
#pragma unroll
  for (int k = 0; k < W; ++k) m[k] ^= (k == q) ? bit : 0ull;
}

// Pass 0 counts, pass 1 writes the pairs (chooser p, covered q) of each
// spliced test path p (offsets tp_off over the prime paths' indices).
// Window hashes roll in O(1): with prefix hashes P[k] of t (P[0] = 0,
// P[k+1] = P[k] * mul + t[k] + 1), the window t[i..j) hashes to
// P[j] - P[i] * mul^(j-i); mul^(j-i) is kept up to date with mul and its
// inverse mod 2^64 (mul is odd).
template <int W>
__global__ __launch_bounds__(kBlock) void k_cover(DGraph g, const int64_t* tp_off,
                                                  const int32_t* tp_vtx, int64_t n, uint64_t mul,
                                                  uint64_t mul_inv,
                                                  const unsigned long long* keys, const int32_t* vals,
                                                  int64_t mask, int64_t* cnt, const int64_t* at,
                                                  int32_t* pair_p, int32_t* pair_q, int pass,
                                                  unsigned long long* missing) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  const int32_t* t = tp_vtx + tp_off[p];
  const int64_t L = tp_off[p + 1] - tp_off[p];
  uint64_t m[W];
#pragma unroll
  for (int k = 0; k < W; ++k) m[k] = 0;
  int64_t j = 0, found = 0, w0 = pass ? at[p] : 0;
  uint64_t Pi = 0, Pj = 0, pw = 1;  // P[i], P[j], mul^(j - i)
  // One action per iteration (extend the window, or test it and advance its
  // start), so the lanes of a wave stay in step: at most 2 |t| iterations.
  int64_t i = 0;
  while (i < L) {
    if (j < L) {
      const int x = t[j];
      if (!set_has<W>(m, g.loc[x])) {
        set_flip<W>(m, g.loc[x]);
        Pj = seq_hash_step(Pj, x, mul);
        pw *= mul;
        ++j;
        continue;
      }
    }
    // t[i..j) is the longest simple window starting at i
    const int v1 = t[i];
    int64_t end = -1;  // exclusive end of the accepted window
    if (j < L && t[j] == v1) {
      end = j + 1;  // a simple cycle
    } else {
      const int vk = t[j - 1];
      bool ok = true;
      for (int k = g.sp[vk]; k < g.sp[vk + 1] && ok; ++k) {
        const int w = g.s[k];
        ok = w != v1 && set_has<W>(m, g.loc[w]);
      }
      for (int k = g.pp[v1]; k < g.pp[v1 + 1] && ok; ++k) ok = set_has<W>(m, g.loc[g.p[k]]);
      if (ok) end = j;
    }
    if (end > 0) {
      uint64_t h = Pj - Pi * pw;
      if (end > j) h = seq_hash_step(Pj, t[j], mul) - Pi * (pw * mul);  // the cycle's closing entry
      const int32_t q = table_find(keys, vals, mask, seq_hash_fix(h));
      if (q < 0) {
        atomicAdd(missing, 1ull);  // not a prime path: a bug, reported to the host
      } else {
        if (pass) {
          pair_p[w0 + found] = (int32_t)p;
          pair_q[w0 + found] = q;
        }
        ++found;
      }
    }
    // drop t[i]: the window now starts at i + 1 (j > i always holds here)
    set_flip<W>(m, g.loc[v1]);
    Pi = seq_hash_step(Pi, v1, mul);
    pw *= mul_inv;
    ++i;
  }
  if (!pass) cnt[p] = found;
}

// Position of every prime path in the order of decreasing length.
__global__ __launch_bounds__(kBlock) void k_len_key(const int64_t* off, int64_t n, int64_t max_len,
                                                    int32_t* key) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) key[i] = (int32_t)(max_len - (off[i + 1] - off[i]));
}

__global__ __launch_bounds__(kBlock) void k_key_hist(const int32_t* key, int64_t n, int64_t ntiles,
                                                     unsigned long long* hist) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) atomicAdd(&hist[(int64_t)key[i] * ntiles + i / kGroupTile], 1ull);
}

__global__ __launch_bounds__(kBlock) void k_invert(const int32_t* perm, int64_t n, int32_t* pos) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < n) pos[perm[k]] = (int32_t)k;
}

// One round over the pairs (p covers q, p before q in the order): q is
// dropped if p is chosen, and blocked (cannot be chosen yet) if p is still
// undecided.  Only constant values are stored.
__global__ __launch_bounds__(kBlock) void k_round_pairs(const int32_t* pair_p, const int32_t* pair_q,
                                                        int64_t np, const int32_t* pos,
                                                        const uint8_t* state, uint8_t* drop,
                                                        uint8_t* block) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= np) return;
  const int32_t p = pair_p[k], q = pair_q[k];
  if (pos[p] >= pos[q] || state[q] != 0) return;
  const uint8_t sp = state[p];
  if (sp == 1) drop[q] = 1;
  else if (sp == 0) block[q] = 1;
}

// Decide: 1 chosen, 2 dropped, 0 undecided; clears the flags for the next
// round and counts the undecided paths (one atomic per wave).
__global__ __launch_bounds__(kBlock) void k_round_decide(int64_t n, uint8_t* state, uint8_t* drop,
                                                         uint8_t* block,
                                                         unsigned long long* undecided) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int und = 0;
  if (q < n && state[q] == 0) {
    if (drop[q]) state[q] = 2;
    else if (!block[q]) state[q] = 1;
    else und = 1;
    drop[q] = 0;
    block[q] = 0;
  }
  const uint64_t b = __ballot(und);
  if (lane_id() == 0 && b) atomicAdd(undecided, (unsigned long long)__builtin_popcountll(b));
}

// Chosen paths in prime-path order: flags for a scan, then the list and the
// per-first-vertex run counts of the merge.
__global__ __launch_bounds__(kBlock) void k_chosen_flags(const uint8_t* state, int64_t n,
                                                         int32_t* flag) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q < n) flag[q] = state[q] == 1 ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_chosen_list(const uint8_t* state, const int64_t* at,
                                                        int64_t n, int32_t* list) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q < n && state[q] == 1) list[at[q]] = (int32_t)q;
}

// Runs of the chosen list by first vertex (the list is in prime-path order,
// hence grouped by first vertex): rb[u] = first position whose first vertex
// is >= u, rb[nv] = m.
__global__ __launch_bounds__(kBlock) void k_chosen_runs(const int32_t* list, int64_t m,
                                                        const int64_t* pp_off, const int32_t* pp_vtx,
                                                        int nv, int64_t* rb) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= m) return;
  const int cur = pp_vtx[pp_off[list[k]]];
  const int prev = k == 0 ? -1 : pp_vtx[pp_off[list[k - 1]]];
  for (int u = prev + 1; u <= cur; ++u) rb[u] = k;
  if (k == m - 1)
    for (int u = cur + 1; u <= nv; ++u) rb[u] = m;
}

template <int W>
hipError_t launch_cover_w(const DGraph& g, const int64_t* tp_off, const int32_t* tp_vtx, int64_t n,
                          uint64_t mul, const uint64_t* keys, const int32_t* vals, int64_t mask,
                          int64_t* cnt, const int64_t* at, int32_t* pair_p, int32_t* pair_q,
                          int pass, uint64_t* missing, hipStream_t st) {
  uint64_t inv = mul;  // Newton's iteration for the inverse of an odd number mod 2^64
  for (int r = 0; r < 6; ++r) inv *= 2 - mul * inv;
  k_cover<W><<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      g, tp_off, tp_vtx, n, mul, inv, reinterpret_cast<const unsigned long long*>(keys), vals, mask,
      cnt, at, pair_p, pair_q, pass, reinterpret_cast<unsigned long long*>(missing));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pp_hash_insert(const int64_t* off, const int32_t* vtx, int64_t n, uint64_t mul,
                                 uint64_t* keys, int32_t* vals, int64_t mask, uint64_t* dups,
                                 hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_pp_hash_insert<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      off, vtx, n, mul, reinterpret_cast<unsigned long long*>(keys), vals, mask,
      reinterpret_cast<unsigned long long*>(dups));
  return hipGetLastError();
}

uint64_t cover_hash_mul(int attempt) { return kHashMul + 2ull * (uint64_t)attempt * 0x2545F4914F6CDD1Dull; }

hipError_t launch_cover(int W, const DGraph& g, const int64_t* tp_off, const int32_t* tp_vtx,
                        int64_t n, uint64_t mul, const uint64_t* keys, const int32_t* vals,
                        int64_t mask, int64_t* cnt, const int64_t* at, int32_t* pair_p,
                        int32_t* pair_q, int pass, uint64_t* missing, hipStream_t st) {
  if (n == 0) return hipSuccess;
  switch (W) {
    case 1: return launch_cover_w<1>(g, tp_off, tp_vtx, n, mul, keys, vals, mask, cnt, at, pair_p, pair_q, pass, missing, st);
    case 2: return launch_cover_w<2>(g, tp_off, tp_vtx, n, mul, keys, vals, mask, cnt, at, pair_p, pair_q, pass, missing, st);
    case 4: return launch_cover_w<4>(g, tp_off, tp_vtx, n, mul, keys, vals, mask, cnt, at, pair_p, pair_q, pass, missing, st);
    case 8: return launch_cover_w<8>(g, tp_off, tp_vtx, n, mul, keys, vals, mask, cnt, at, pair_p, pair_q, pass, missing, st);
    case 16: return launch_cover_w<16>(g, tp_off, tp_vtx, n, mul, keys, vals, mask, cnt, at, pair_p, pair_q, pass, missing, st);
    case 32: return launch_cover_w<32>(g, tp_off, tp_vtx, n, mul, keys, vals, mask, cnt, at, pair_p, pair_q, pass, missing, st);
    case 64: return launch_cover_w<64>(g, tp_off, tp_vtx, n, mul, keys, vals, mask, cnt, at, pair_p, pair_q, pass, missing, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_len_key(const int64_t* off, int64_t n, int64_t max_len, int32_t* key,
                          hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_len_key<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(off, n, max_len, key);
  return hipGetLastError();
}

hipError_t launch_key_hist(const int32_t* key, int64_t n, int64_t ntiles, uint64_t* hist,
                           hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_key_hist<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      key, n, ntiles, reinterpret_cast<unsigned long long*>(hist));
  return hipGetLastError();
}

hipError_t launch_invert(const int32_t* perm, int64_t n, int32_t* pos, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_invert<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(perm, n, pos);
  return hipGetLastError();
}

hipError_t launch_round_pairs(const int32_t* pair_p, const int32_t* pair_q, int64_t np,
                              const int32_t* pos, const uint8_t* state, uint8_t* drop,
                              uint8_t* block, hipStream_t st) {
  if (np == 0) return hipSuccess;
  k_round_pairs<<<(unsigned)((np + kBlock - 1) / kBlock), kBlock, 0, st>>>(pair_p, pair_q, np, pos,
                                                                          state, drop, block);
  return hipGetLastError();
}

hipError_t launch_round_decide(int64_t n, uint8_t* state, uint8_t* drop, uint8_t* block,
                               uint64_t* undecided, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_round_decide<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      n, state, drop, block, reinterpret_cast<unsigned long long*>(undecided));
  return hipGetLastError();
}

hipError_t launch_chosen_flags(const uint8_t* state, int64_t n, int32_t* flag, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_chosen_flags<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(state, n, flag);
  return hipGetLastError();
}

hipError_t launch_chosen_list(const uint8_t* state, const int64_t* at, int64_t n, int32_t* list,
                              hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_chosen_list<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(state, at, n, list);
  return hipGetLastError();
}

hipError_t launch_chosen_runs(const int32_t* list, int64_t m, const int64_t* pp_off,
                              const int32_t* pp_vtx, int nv, int64_t* rb, hipStream_t st) {
  if (m == 0) return hipSuccess;
  k_chosen_runs<<<(unsigned)((m + kBlock - 1) / kBlock), kBlock, 0, st>>>(list, m, pp_off, pp_vtx,
                                                                         nv, rb);
  return hipGetLastError();
}

}  // namespace tpg
