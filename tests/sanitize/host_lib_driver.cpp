// Drives the host-only part of libtpg (CSR loading, validation,
// canonicalization, binarization, features) on valid and malformed inputs,
// for a build with AddressSanitizer and UndefinedBehaviorSanitizer.  Prints
// the number of loads that succeeded and failed; a sanitizer report aborts.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../include/tpg.h"

namespace {

uint64_t rng_state = 0x9E3779B97F4A7C15ull;
uint64_t next_u64() {  // xorshift64*
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return rng_state * 2685821657736338717ull;
}
int below(int k) { return (int)(next_u64() % (uint64_t)k); }

struct Csr {
  int n = 0;
  std::vector<int64_t> rp{0};
  std::vector<int32_t> ci;
};

// A CFG-shaped graph: a spine 0 -> 1 -> ... -> n-1 plus random forward and
// backward arcs that keep the entry without predecessors and the exit
// without successors.
Csr cfg_like(int n, int extra) {
  Csr g;
  g.n = n;
  std::vector<std::vector<int32_t>> out(n);
  for (int v = 0; v + 1 < n; ++v) out[v].push_back(v + 1);
  for (int k = 0; k < extra && n > 3; ++k) {
    const int a = 1 + below(n - 2), b = 1 + below(n - 2);
    out[a].push_back(b);
  }
  for (int v = 0; v < n; ++v) {
    for (int w : out[v]) g.ci.push_back(w);
    g.rp.push_back((int64_t)g.ci.size());
  }
  return g;
}

int ok = 0, failed = 0;

tpg_graph* load(const Csr& g, int entry, int exit, uint32_t flags) {
  tpg_graph* h = nullptr;
  const tpg_status s = tpg_load_cfg_csr(g.n, g.rp.data(), g.ci.empty() ? nullptr : g.ci.data(),
                                        entry, exit, flags, &h);
  if (s == TPG_OK) {
    ++ok;
    int32_t n = 0, e = 0, x = 0;
    int64_t m = 0;
    tpg_graph_info(h, &n, &m, &e, &x);
    std::vector<int64_t> rp((size_t)n + 1);
    std::vector<int32_t> ci((size_t)m + 1);
    tpg_graph_csr(h, rp.data(), ci.data());
  } else {
    ++failed;
    if (h) std::printf("error left a handle\n");
    (void)tpg_last_error();
    (void)tpg_status_str(s);
  }
  return h;
}

}  // namespace

int main() {
  std::vector<tpg_graph*> keep;
  for (int it = 0; it < 400; ++it) {
    const int n = 2 + below(150);
    Csr g = cfg_like(n, below(3 * n));
    const uint32_t flags = (it % 3 == 0) ? TPG_LOAD_BINARIZE : (it % 7 == 0 ? TPG_LOAD_STRICT : 0);
    if (tpg_graph* h = load(g, 0, n - 1, flags)) keep.push_back(h);
    // malformed variants of the same graph
    Csr bad = g;
    switch (it % 6) {
      case 0: bad.rp[0] = 1; break;
      case 1: if (!bad.ci.empty()) bad.ci[below((int)bad.ci.size())] = n + below(5); break;
      case 2: if (n > 2) bad.rp[1 + below(n - 1)] = -1; break;
      case 3: if (!bad.ci.empty()) bad.ci[0] = -1; break;
      case 4: bad.ci.push_back(0); bad.rp.back() += 1; break;  // an arc into the entry
      case 5: break;
    }
    if (tpg_graph* h = load(bad, 0, n - 1, flags)) tpg_graph_free(h);
    if (tpg_graph* h = load(g, n, -1, 0)) tpg_graph_free(h);
    if (tpg_graph* h = load(g, 0, n - 1, TPG_LOAD_ANY_DIGRAPH)) tpg_graph_free(h);
  }
  // self-loops, duplicate arcs, a single vertex, a wide switch
  {
    Csr g;
    g.n = 4;
    g.rp = {0, 2, 5, 6, 6};
    g.ci = {1, 1, 2, 2, 1, 3};
    if (tpg_graph* h = load(g, 0, 3, 0)) tpg_graph_free(h);
    if (tpg_graph* h = load(g, 0, 3, TPG_LOAD_STRICT)) tpg_graph_free(h);
    Csr one;
    one.n = 1;
    one.rp = {0, 0};
    if (tpg_graph* h = load(one, 0, 0, 0)) tpg_graph_free(h);
    Csr sw;
    sw.n = 40;
    for (int v = 1; v < 39; ++v) sw.ci.push_back(v);
    sw.rp.push_back((int64_t)sw.ci.size());
    for (int v = 1; v < 39; ++v) {
      sw.ci.push_back(39);
      sw.rp.push_back((int64_t)sw.ci.size());
    }
    sw.rp.push_back((int64_t)sw.ci.size());
    if (tpg_graph* h = load(sw, 0, 39, TPG_LOAD_BINARIZE)) keep.push_back(h);
  }
  std::vector<float> feat(keep.size() * 32);
  if (tpg_features((const tpg_graph* const*)keep.data(), (int32_t)keep.size(), feat.data()) !=
      TPG_OK)
    std::printf("features failed: %s\n", tpg_last_error());
  double sum = 0;
  for (float f : feat) sum += f;
  for (tpg_graph* h : keep) tpg_graph_free(h);
  std::printf("loads ok %d failed %d features %zu checksum %.3f\n", ok, failed, keep.size(), sum);
  return 0;
}
