// CPU run of the library's one-pass level loop (csrc/sizing.h) against known
// level sizes: a simulated device applies the extension kernels' fit test
// and claims exact child counts, so the host loop's sizing, growth and replay
// decisions are the ones the library takes on the GPU for the same graph.
//
// stdin: first_batch held_rec held_msk rec0 msk0 growth stale_children (read size
//        of an overflowing level's children short by this many)
//        n_levels, then size[1] .. size[n_levels]
// stdout: status n_overflows Lmax reserves rec_cap mask_cap levels_equal
#include <cstdio>
#include <cstdint>
#include <vector>

#include "sizing.h"

using namespace tpg;

namespace {

struct SimDev {
  std::vector<int64_t> truth;  // size of every level (index = level)
  int64_t rec = 0, msk = 0;
  double growth = 1.0;         // buffers grow to at least this factor of their old size
  int64_t stale = 0;           // children left out of the size the host reads (a planted fault)
  std::vector<int64_t> count, off, report;
  bool ovf = false;
  int ovl = 0;
  int64_t reserves = 0;
  bool kept_too_much = false;

  int64_t rec_cap() const { return rec; }
  int64_t mask_cap() const { return msk; }
  int64_t size(int L) const { return L < (int)truth.size() ? truth[L] : 0; }
  bool reserve(const TreeCaps& c, int64_t keep_rec, int keep_level, int64_t keep_mask) {
    // what is kept must have been held
    if (keep_rec > rec || (keep_level > 0 && keep_mask > msk)) kept_too_much = true;
    if (c.rec > rec) rec = std::max<int64_t>(c.rec, (int64_t)(rec * growth));
    if (c.msk > msk) msk = std::max<int64_t>(c.msk, (int64_t)(msk * growth));
    reserves += 1;
    return true;
  }
  // launches L0 .. L0 + len - 1, each with the kernels' early exits
  bool run(int L0, int len, BatchReport& r) {
    for (int li = 0; li < len; ++li) {
      const int L = L0 + li;
      if (ovf) break;
      const int64_t F = count[L];
      if (F == 0) continue;
      const int64_t base = off[L - 1] + count[L - 1];
      if (!level_fits(L, base, F, rec, msk)) {
        ovf = true;
        ovl = L - 1;
        break;
      }
      off[L] = base;
      count[L + 1] = size(L + 1);
    }
    report = count;
    if (ovf) report[ovl + 1] = std::max<int64_t>(0, report[ovl + 1] - stale);
    r.overflow = ovf;
    r.overflow_level = ovl;
    r.count = report.data();
    return true;
  }
  bool resume(int Lo) {
    count[Lo + 1] = 0;
    ovf = false;
    ovl = 0;
    return true;
  }
};

}  // namespace

int main() {
  int first_batch = 4, n_levels = 0;
  long long held_rec, held_msk, rec0, msk0, stale;
  double growth;
  if (scanf("%d %lld %lld %lld %lld %lf %lld %d", &first_batch, &held_rec, &held_msk, &rec0, &msk0,
            &growth, &stale, &n_levels) != 8)
    return 2;
  const int max_levels = 4100;
  SimDev d;
  d.truth.assign(n_levels + 2, 0);
  for (int L = 1; L <= n_levels; ++L) {
    long long x;
    if (scanf("%lld", &x) != 1) return 2;
    d.truth[L] = x;
  }
  d.growth = growth;
  d.stale = stale;
  d.count.assign(max_levels + 2, 0);
  d.off.assign(max_levels + 2, 0);
  d.count[1] = d.truth[1];
  // the loop's first request, as the library makes it (n = the level-1 size)
  const TreeCaps first = onepass_first_caps(held_rec, held_msk, (int)d.truth[1], rec0, msk0);
  d.rec = first.rec;
  d.msk = first.msk;
  std::vector<int64_t> cnt(max_levels + 1, 0);
  cnt[1] = d.truth[1];
  int Lmax = 0;
  int64_t n_ovf = 0;
  LoopFailure why;
  const LoopEnd e = onepass_levels(d, first_batch, max_levels, cnt, Lmax, n_ovf, why);
  int equal = !d.kept_too_much;
  for (int L = 1; L <= n_levels && e == LoopEnd::ok; ++L)
    if (L <= Lmax ? cnt[L] != d.truth[L] : d.truth[L] != 0) equal = 0;
  if (e == LoopEnd::ok && Lmax < n_levels && d.truth[Lmax + 1] != 0) equal = 0;
  printf("%d %lld %d %lld %lld %lld %d\n", (int)e, (long long)n_ovf, Lmax, (long long)d.reserves,
         (long long)d.rec, (long long)d.msk, equal);
  return 0;
}
