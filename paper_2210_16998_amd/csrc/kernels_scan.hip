// Device-wide exclusive scans (reduce, scan of tile sums, scan down: three
// launches, no workgroup waits on another) and small fill helpers.  Fills are
// kernels rather than memsets so that the sequences that use them can be
// captured in HIP graphs.

#include "kernels.h"

namespace tpg {

constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;  // 4096 items per tile

int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

__global__ void k_zero_u64(uint64_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}
__global__ void k_zero_u32(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

hipError_t launch_zero_u64(uint64_t* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_zero_u64<<<(unsigned)std::min<int64_t>(1024, (n + kBlock - 1) / kBlock), kBlock, 0, st>>>(p, n);
  return hipGetLastError();
}
// FNV-1a 64 over the int32 little-endian bytes (k, v_1 .. v_k) of each path,
// one thread per path; sums and xors are reduced per wave and added to out
// with one 64-bit atomic pair per wave.
__device__ __forceinline__ uint64_t fnv1a_word(uint64_t h, uint32_t w) {
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    h ^= (w >> (8 * b)) & 0xFFu;
    h *= 0x100000001b3ull;
  }
  return h;
}

__global__ __launch_bounds__(kBlock) void k_digest(const int64_t* off, const int32_t* vtx, int64_t n,
                                                   unsigned long long* out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  uint64_t h = 0;
  bool have = i < n;
  if (have) {
    const int64_t o0 = off[i], o1 = off[i + 1];
    h = fnv1a_word(0xcbf29ce484222325ull, (uint32_t)(o1 - o0));
    for (int64_t k = o0; k < o1; ++k) h = fnv1a_word(h, (uint32_t)vtx[k]);
  }
  uint64_t sum = have ? h : 0, x = have ? h : 0;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    sum += __shfl_xor(sum, d, 64);
    x ^= __shfl_xor(x, d, 64);
  }
  if (lane_id() == 0) {
    atomicAdd(&out[0], (unsigned long long)sum);
    atomicXor(&out[1], (unsigned long long)x);
  }
}

hipError_t launch_digest(const int64_t* off, const int32_t* vtx, int64_t n, uint64_t* out,
                         hipStream_t st) {
  k_zero_u64<<<1, 64, 0, st>>>(out, 2);
  if (n > 0)
    k_digest<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        off, vtx, n, reinterpret_cast<unsigned long long*>(out));
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_zero_u32<<<(unsigned)std::min<int64_t>(1024, (n + kBlock - 1) / kBlock), kBlock, 0, st>>>(p, n);
  return hipGetLastError();
}

__global__ void k_set_i64(int64_t* p, const int64_t* src) { *p = *src; }
__global__ void k_set_value_i64(int64_t* p, int64_t v) { *p = v; }
hipError_t launch_set_value_i64(int64_t* p, int64_t value, hipStream_t st) {
  k_set_value_i64<<<1, 1, 0, st>>>(p, value);
  return hipGetLastError();
}
hipError_t launch_set_i64(int64_t* p, const int64_t* src, hipStream_t st) {
  k_set_i64<<<1, 1, 0, st>>>(p, src);
  return hipGetLastError();
}

// Phase 1: sums[t] = sum of tile t (loads strided by the workgroup size).
template <class Tin>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const Tin* in, int64_t n, int64_t* sums) {
  __shared__ int64_t s_w[kBlock / 64];
  const int64_t t = blockIdx.x;
  const int64_t b = t * kScanTile + threadIdx.x;
  int64_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = b + (int64_t)k * kBlock;
    sum += i < n ? (int64_t)in[i] : 0;
  }
  int64_t tot;
  block_excl_scan<kBlock, int64_t>(sum, tot, s_w);
  if (threadIdx.x == 0) sums[t] = tot;
}

// Phase 2 (one workgroup): sums[t] <- add + sum(sums[0..t)), sums[ntile] and
// *total <- add + everything.
__global__ __launch_bounds__(1024) void k_scan_tiles(int64_t* sums, int64_t ntile, int64_t add,
                                                     int64_t* total) {
  __shared__ int64_t s_w[16];
  int64_t carry = add;
  for (int64_t c = 0; c < ntile; c += 1024) {
    const int64_t i = c + threadIdx.x;
    const int64_t v = i < ntile ? sums[i] : 0;
    int64_t tot;
    const int64_t pre = block_excl_scan<1024, int64_t>(v, tot, s_w);
    if (i < ntile) sums[i] = carry + pre;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    sums[ntile] = carry;
    if (total) *total = carry;
  }
}

// Phase 3: out[i] = sums[t] + exclusive prefix inside the tile; the last tile
// also writes out[n].  Staged through LDS so that global loads and stores are
// strided by the workgroup size while each thread scans 16 consecutive items.
template <class Tin, class Tout>
__global__ __launch_bounds__(kBlock) void k_scan_down(const Tin* in, Tout* out, int64_t n,
                                                      const int64_t* sums, int64_t ntile) {
  constexpr int PAD = kScanTile + kScanTile / kScanItems;  // one pad slot per 16 items
  __shared__ int64_t s_v[PAD];
  __shared__ int64_t s_w[kBlock / 64];
  const int64_t t = blockIdx.x;
  const int64_t b = t * kScanTile;
  const int tid = (int)threadIdx.x;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int x = k * kBlock + tid;
    const int64_t i = b + x;
    s_v[x + x / kScanItems] = i < n ? (int64_t)in[i] : 0;
  }
  __syncthreads();
  int64_t v[kScanItems];
  int64_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = s_v[tid * (kScanItems + 1) + k];
    sum += v[k];
  }
  int64_t tot;
  int64_t run = sums[t] + block_excl_scan<kBlock, int64_t>(sum, tot, s_w);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    s_v[tid * (kScanItems + 1) + k] = run;
    run += v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int x = k * kBlock + tid;
    const int64_t i = b + x;
    if (i < n) out[i] = (Tout)s_v[x + x / kScanItems];
  }
  if (t == ntile - 1 && tid == 0) out[n] = (Tout)sums[ntile];
}

template <class Tout>
__global__ void k_scan_empty(Tout* out, int64_t add, int64_t* total) {
  out[0] = (Tout)add;
  if (total) *total = add;
}

// out[i] = add + sum(in[0..i)) for i <= n (out has n+1 entries; in == out is
// allowed); *total = add + sum(in).  `status` holds scan_tiles(n) tile sums;
// `ctr` is not used.
template <class Tin, class Tout>
static hipError_t scan_impl(const Tin* in, Tout* out, int64_t n, int64_t add, int64_t* total,
                            uint64_t* status, uint32_t* ctr, hipStream_t st) {
  (void)ctr;
  if (n <= 0) {
    k_scan_empty<Tout><<<1, 1, 0, st>>>(out, add, total);
    return hipGetLastError();
  }
  const int64_t ntile = (n + kScanTile - 1) / kScanTile;
  int64_t* sums = reinterpret_cast<int64_t*>(status);
  k_scan_reduce<Tin><<<(unsigned)ntile, kBlock, 0, st>>>(in, n, sums);
  k_scan_tiles<<<1, 1024, 0, st>>>(sums, ntile, add, total);
  k_scan_down<Tin, Tout><<<(unsigned)ntile, kBlock, 0, st>>>(in, out, n, sums, ntile);
  return hipGetLastError();
}

hipError_t scan_i32_to_i32(const int32_t* in, int32_t* out, int64_t n, int64_t add,
                           int64_t* total, uint64_t* status, uint32_t* ctr, hipStream_t st) {
  return scan_impl<int32_t, int32_t>(in, out, n, add, total, status, ctr, st);
}

hipError_t scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, int64_t add,
                           int64_t* total, uint64_t* status, uint32_t* ctr, hipStream_t st) {
  return scan_impl<int32_t, int64_t>(in, out, n, add, total, status, ctr, st);
}

hipError_t scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t add, int64_t* total,
                    uint64_t* status, uint32_t* ctr, hipStream_t st) {
  return scan_impl<int64_t, int64_t>(in, out, n, add, total, status, ctr, st);
}

}  // namespace tpg
