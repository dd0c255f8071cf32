// Internal declarations shared by the host-side sources of libtpg.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tpg.h"

struct tpg_graph {
  int32_t n = 0;
  int32_t entry = 0, exit = 0;
  uint32_t load_flags = 0;
  int32_t max_out_degree = 0;
  // canonical forward CSR (rows ascending, unique) and reverse CSR
  std::vector<int32_t> succ_ptr, succ;
  std::vector<int32_t> pred_ptr, pred;
  uint64_t uid = 0;  // identifies the graph in device caches
  // structural features, computed once on first use
  mutable std::once_flag feat_once;
  mutable float feat[32];
};

namespace tpg {

void set_error(const char* fmt, ...);
tpg_status fail(tpg_status s, const char* fmt, ...);

#define TPG_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::tpg::fail(e_ == hipErrorOutOfMemory ? TPG_ERR_OOM_DEVICE : TPG_ERR_DEVICE, \
                         "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),  \
                         __FILE__, __LINE__);                                      \
  } while (0)

#define TPG_TRY(call)                       \
  do {                                      \
    tpg_status s_ = (call);                 \
    if (s_ != TPG_OK) return s_;            \
  } while (0)

// A device buffer that grows on demand (contents are not preserved unless
// grow_keep is used).
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  template <class T>
  T* as() const { return reinterpret_cast<T*>(p); }
};

}  // namespace tpg
