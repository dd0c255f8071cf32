// Device-wide exclusive scans (single pass, decoupled look-back) and small
// fill helpers.  Fills are kernels rather than memsets so that the sequences
// that use them can be captured in HIP graphs.

#include "kernels.h"

namespace tpg {

constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

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

// out[i] = add + sum(in[0..i)) for i <= n (out has n+1 entries; in == out is
// allowed); *total = add + sum(in).  status / ctr must be zero on entry
// (status: scan_tiles(n) slots).
template <class Tin, class Tout>
__global__ __launch_bounds__(kBlock) void k_scan(const Tin* in, Tout* out, int64_t n, int64_t add,
                                                 int64_t* total, uint64_t* status, uint32_t* ctr) {
  __shared__ int64_t s_tile, s_prefix;
  __shared__ int64_t s_w[kBlock / 64];
  if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(ctr, 1u);
  __syncthreads();
  const int64_t t = s_tile;
  const int64_t b = t * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (b + k < n) ? (int64_t)in[b + k] : 0;
    sum += v[k];
  }
  int64_t agg;
  const int64_t pre = block_excl_scan<kBlock, int64_t>(sum, agg, s_w);
  if (threadIdx.x == 0) s_prefix = lookback_prefix(status, t, agg);
  __syncthreads();
  int64_t run = add + s_prefix + pre;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (b + k < n) out[b + k] = (Tout)run;
    run += v[k];
  }
  const int64_t ntile = (n + kScanTile - 1) / kScanTile;
  if (t == (ntile > 0 ? ntile - 1 : 0) && threadIdx.x == kBlock - 1) {
    out[n] = (Tout)run;
    if (total) *total = run;
  }
}

template <class Tin, class Tout>
static hipError_t scan_impl(const Tin* in, Tout* out, int64_t n, int64_t add, int64_t* total,
                            uint64_t* status, uint32_t* ctr, hipStream_t st) {
  const int64_t ntile = std::max<int64_t>(1, (n + kScanTile - 1) / kScanTile);
  hipError_t e = launch_zero_u64(status, ntile + 1, st);
  if (e != hipSuccess) return e;
  e = launch_zero_u32(ctr, 1, st);
  if (e != hipSuccess) return e;
  k_scan<Tin, Tout><<<(unsigned)ntile, kBlock, 0, st>>>(in, out, n, add, total, status, ctr);
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
