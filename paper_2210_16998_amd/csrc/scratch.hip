// Prime-path types without device allocation (tpg_prime_path_types_noalloc).
//
// The same computation as tpg_prime_path_types (Sec. 2: components, Defs.
// 4-5 entry/exit vertices, the types of Defs. 2, 9, 10, 11) for callers that
// cannot allocate device memory.  Everything the kernels need beyond the
// caller's inputs and outputs -- the graph's CSR and reverse CSR staged on
// the device, the component search's work arrays, labels, flags and the
// per-type counters -- lives in one fixed device array, `scratch`, of
// kScratchBytes.  Every call on a device shares that device's copy and
// overwrites it, so calls that overlap on one device race; what must start
// at a known value (vertex ids, component labels of the single graph, the
// search's index array, the counters) is written by a kernel at the start
// of every call.
#include <algorithm>
#include <mutex>

#include "internal.h"
#include "kernels.h"

namespace tpg {
namespace {

// 1 MiB: the CSR and reverse CSR (8 B per arc, 8 B per vertex), the search's
// arrays, labels and flags (29 B per vertex) and the counters; a graph of
// 4096 vertices fits with up to about 108 000 arcs.
constexpr size_t kScratchBytes = size_t(1) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each device (the host-side symbol is only a
// stand-in), looked up once per device with that device current.
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

tpg_status scratch_on_current_device(void** out) {
  int dev = -1;
  TPG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(TPG_ERR_DEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(TPG_ERR_DEVICE, "no device address for the scratch array on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TPG_OK;
}

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

// One graph's vertex ids are its own (loc[v] = v) and every vertex belongs
// to graph 0 (comp[v] = 0); cbase = {0, n}, centry / cexit = the graph's.
__global__ __launch_bounds__(kBlock) void k_single_graph_ids(int32_t* loc, int32_t* comp,
                                                             int32_t* tail, int32_t n,
                                                             int32_t entry, int32_t exit) {
  const int32_t v = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (v < n) {
    loc[v] = v;
    comp[v] = 0;
  }
  if (v == 0) {
    tail[0] = 0;  // cbase[0]
    tail[1] = n;  // cbase[1]
    tail[2] = entry;
    tail[3] = exit;
  }
}

}  // namespace
}  // namespace tpg

using namespace tpg;

extern "C" tpg_status tpg_prime_path_types_noalloc(const tpg_graph* g, const int64_t* d_offsets,
                                                   const int32_t* d_vertices, int64_t n_paths,
                                                   void* stream, uint8_t* d_types,
                                                   int64_t* counts) {
  if (!g) return fail(TPG_ERR_INVALID_ARG, "graph is NULL");
  if (n_paths < 0) return fail(TPG_ERR_INVALID_ARG, "negative path count");
  if (n_paths > 0 && (!d_offsets || !d_vertices))
    return fail(TPG_ERR_INVALID_ARG, "path arrays are NULL");
  const int32_t n = g->n;
  const size_t m = g->succ.size();
  // layout: sp, s (+1), pp, p (+1), loc, comp, cbase/centry/cexit (4 words)
  // back to back, as the kernels' staging expects; then the search's 6 n
  // work words, the labels, the flags and the counters
  const size_t csr_words = 2 * ((size_t)n + 1) + 2 * (m + 1) + 2 * (size_t)n + 4;
  const size_t off_work = up256(4 * csr_words);
  const size_t off_comp = off_work + up256(4 * 6 * (size_t)n);
  const size_t off_flags = off_comp + up256(4 * (size_t)n);
  const size_t off_misc = off_flags + up256((size_t)n);
  const size_t need = off_misc + 64 + sizeof(uint64_t) * kPpTypes;
  if (need > kScratchBytes)
    return fail(TPG_ERR_CAPACITY,
                "the graph needs %zu bytes of scratch (%d vertices, %zu arcs); the fixed "
                "scratch holds %zu",
                need, n, m, kScratchBytes);
  hipStream_t st = (hipStream_t)stream;
  void* base = nullptr;
  TPG_TRY(scratch_on_current_device(&base));
  unsigned char* b = (unsigned char*)base;
  int32_t* q = (int32_t*)b;
  DGraph d{};
  auto put = [&](const std::vector<int32_t>& v, size_t pad) -> const int32_t* {
    int32_t* at = q;
    q += v.size() + pad;
    return at;
  };
  d.sp = put(g->succ_ptr, 0);
  d.s = put(g->succ, 1);
  d.pp = put(g->pred_ptr, 0);
  d.p = put(g->pred, 1);
  int32_t* loc = q;
  q += n;
  int32_t* comp_of = q;
  q += n;
  int32_t* tail = q;
  d.loc = loc;
  d.comp = comp_of;
  d.cbase = tail;
  d.centry = tail + 2;
  d.cexit = tail + 3;
  d.n = n;
  d.n_comp = 1;
  d.n_stage = (int32_t)(d.comp - d.sp);
  TPG_HIP(hipMemcpyAsync((void*)d.sp, g->succ_ptr.data(), 4 * g->succ_ptr.size(),
                         hipMemcpyHostToDevice, st));
  if (m)
    TPG_HIP(hipMemcpyAsync((void*)d.s, g->succ.data(), 4 * m, hipMemcpyHostToDevice, st));
  TPG_HIP(hipMemcpyAsync((void*)d.pp, g->pred_ptr.data(), 4 * g->pred_ptr.size(),
                         hipMemcpyHostToDevice, st));
  if (m)
    TPG_HIP(hipMemcpyAsync((void*)d.p, g->pred.data(), 4 * m, hipMemcpyHostToDevice, st));
  const unsigned grid = (unsigned)std::max<int64_t>(1, ((int64_t)n + kBlock - 1) / kBlock);
  k_single_graph_ids<<<grid, kBlock, 0, st>>>(loc, comp_of, tail, n, g->entry, g->exit);
  TPG_HIP(hipGetLastError());
  int32_t* work = (int32_t*)(b + off_work);
  int32_t* comp = (int32_t*)(b + off_comp);
  uint8_t* flags = b + off_flags;
  int32_t* n_comp = (int32_t*)(b + off_misc);
  unsigned long long* d_cnt = (unsigned long long*)(b + off_misc + 64);
  TPG_HIP(launch_scc(d, (int32_t)m, work, comp, flags, n_comp, st));
  TPG_HIP(launch_pp_types(d, comp, flags, d_offsets, d_vertices, n_paths, d_types, d_cnt, st));
  if (counts) {
    // pageable destination: the copy returns once the counters are read
    uint64_t h[kPpTypes];
    TPG_HIP(hipMemcpyAsync(h, d_cnt, sizeof h, hipMemcpyDeviceToHost, st));
    TPG_HIP(hipStreamSynchronize(st));
    for (int t = 0; t < kPpTypes; ++t) counts[t] = (int64_t)h[t];
  } else {
    TPG_HIP(hipStreamSynchronize(st));
  }
  return TPG_OK;
}
