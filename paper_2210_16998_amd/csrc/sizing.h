// Sizing of the one-pass level loop: the fit test the extension kernels apply
// to a level before extending it, the capacities the host asks for, and the
// host loop that runs batches of levels, grows the buffers after an overflow
// and replays the level whose children did not fit.
//
// Plain C++ with no runtime calls: the loop drives the device through a small
// interface (below), so the same code runs on the CPU against known level
// sizes.  constexpr functions are usable from device code as well.
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

namespace tpg {

// Level L holds F paths at node indices [base, base + F).  It can be
// extended when its records end below the record capacity (one spare slot
// for the child-range sentinel), its visited sets fit the set buffers (only
// odd levels store them) and node indices stay below 2^31.
constexpr bool level_fits(int L, int64_t base, int64_t F, int64_t rec_cap, int64_t mask_cap) {
  return base + F + 1 <= rec_cap && (!(L & 1) || F <= mask_cap) &&
         base + F < (int64_t)INT32_MAX;
}

// Capacities asked for: nodes over all levels, and slots of one stored level.
struct TreeCaps {
  int64_t rec = 0, msk = 0;
};

// Node indices are int32 (one spare slot for the child-range sentinel): a
// request never goes beyond this many nodes unless the tree needs more,
// whatever the workspace holds or the caller predicted.
constexpr int64_t kMaxTreeNodes = (int64_t)INT32_MAX - 2;

// First request of a run: what the workspace already holds (held_rec, and
// held_msk slots at the run's set width), a floor from the vertex count, and
// the caller's predicted sizes (0: none).
constexpr TreeCaps onepass_first_caps(int64_t held_rec, int64_t held_msk, int n, int64_t rec0,
                                      int64_t msk0) {
  return TreeCaps{std::min(std::max({held_rec, (int64_t)n * 64 + 4096, rec0}), kMaxTreeNodes),
                  std::max({(int64_t)n * 16 + 1024, msk0, held_msk})};
}

// After level Lo (F paths from node base) claimed nxt children that did not
// fit: room for every node up to the end of level Lo + 1 with 25% to spare,
// and when Lo + 1 is odd (its sets are stored) room for its nxt sets.
constexpr TreeCaps onepass_grown_caps(int64_t rec_cap, int64_t mask_cap, int Lo, int64_t base,
                                      int64_t F, int64_t nxt) {
  const int64_t need = base + F + nxt + 1;
  return TreeCaps{std::max(need, std::min(std::max(rec_cap, need + need / 4), kMaxTreeNodes)),
                  ((Lo + 1) & 1) ? std::max(mask_cap, nxt + nxt / 4 + 1024) : mask_cap};
}

// Stored level whose sets the extension of level L reads (L itself when odd,
// else the odd level before it).
constexpr int stored_level_read_by(int L) { return (L & 1) ? L : L - 1; }

// What a batch of launches reports: the overflow flag and level, and the
// per-level sizes count[L] for L = L0 .. L0 + len (count[L + 1] is the
// number of children level L claimed).
struct BatchReport {
  bool overflow = false;
  int overflow_level = 0;
  const int64_t* count = nullptr;  // indexed by level
};

enum class LoopEnd { ok, device_failed, too_deep, bad_report, repeated_overflow };

struct LoopFailure {
  int level = 0;
  int64_t rec_cap = 0, mask_cap = 0, base = 0, F = 0, nxt = 0;
};

// The one-pass level loop.  Dev provides:
//   int64_t rec_cap() const, mask_cap() const;      current capacities
//   bool reserve(const TreeCaps&, int64_t keep_rec, int keep_level, int64_t keep_mask);
//        grow to at least these capacities, keeping nodes [0, keep_rec) and
//        the first keep_mask sets of stored level keep_level (0: none)
//   bool run(int L0, int len, BatchReport& r);        launches extending
//        levels L0 .. L0 + len - 1, then the report
//   bool resume(int Lo);                              clear level Lo's claim
// cnt[1] holds the seeded level's size on entry; on return cnt[L] is the size
// of level L for L <= Lmax (the deepest level holding paths).  Levels run in
// batches of first_batch, doubling up to 64.  With exact sizes from the
// device a level overflows at most once (it is grown to the exact size of its
// children), so a second overflow of the same level ends the loop with
// repeated_overflow instead of replaying it again.
template <class Dev>
LoopEnd onepass_levels(Dev& d, int first_batch, int max_levels, std::vector<int64_t>& cnt,
                       int& Lmax, int64_t& n_overflows, LoopFailure& fail_info) {
  if ((int)cnt.size() < max_levels + 1) cnt.resize(max_levels + 1, 0);
  std::vector<uint8_t> overflowed(max_levels + 1, 0);
  int L0 = 1;
  int batch = std::max(1, first_batch);
  for (;;) {
    const int len = std::min(batch, max_levels - 2 - L0);
    if (len <= 0) return LoopEnd::too_deep;
    BatchReport r;
    if (!d.run(L0, len, r)) return LoopEnd::device_failed;
    const int Lo = r.overflow ? r.overflow_level : -1;
    if (r.overflow && (Lo < std::max(1, L0 - 1) || Lo > L0 + len - 2)) {
      fail_info.level = Lo;
      return LoopEnd::bad_report;
    }
    // levels extended for good in this batch: L0 .. last_ok
    const int last_ok = r.overflow ? Lo - 1 : L0 + len - 1;
    for (int L = L0; L <= std::min(last_ok + 1, L0 + len); ++L) cnt[L] = r.count[L];
    if (r.overflow) {
      cnt[Lo + 1] = r.count[Lo + 1];
      int64_t base = 0;
      for (int L = 1; L < Lo; ++L) base += cnt[L];
      const int64_t F = cnt[Lo], nxt = cnt[Lo + 1];
      if (overflowed[Lo]) {
        fail_info = LoopFailure{Lo, d.rec_cap(), d.mask_cap(), base, F, nxt};
        return LoopEnd::repeated_overflow;
      }
      overflowed[Lo] = 1;
      const TreeCaps c = onepass_grown_caps(d.rec_cap(), d.mask_cap(), Lo, base, F, nxt);
      const int Ls = stored_level_read_by(Lo);
      if (!d.reserve(c, base + F, Ls, cnt[Ls])) return LoopEnd::device_failed;
      if (!d.resume(Lo)) return LoopEnd::device_failed;
      n_overflows += 1;
      L0 = Lo;
      continue;
    }
    int empty = -1;
    for (int L = L0; L <= L0 + len; ++L)
      if (cnt[L] == 0) {
        empty = L;
        break;
      }
    if (empty > 0) {
      Lmax = empty - 1;
      return LoopEnd::ok;
    }
    L0 += len;
    batch = std::max(4, std::min(batch * 2, 64));
  }
}

}  // namespace tpg
