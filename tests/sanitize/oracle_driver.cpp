// Drives every routine of the CPU oracle on small random digraphs and CFGs
// (threads included), for builds with AddressSanitizer +
// UndefinedBehaviorSanitizer and with ThreadSanitizer.  A sanitizer report
// aborts; a disagreement between the oracle's own routines returns 1.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

extern "C" {
typedef struct orc_paths {
  int64_t n_paths, n_vertices;
  int64_t* offsets;
  int32_t* vertices;
} orc_paths;
typedef struct orc_stats {
  int64_t n_candidates, n_cycles, n_extensions, n_pp, n_pp_local, max_len;
} orc_stats;
void orc_free_paths(orc_paths*);
int orc_prime_paths(int, const int64_t*, const int32_t*, int, orc_paths*, orc_stats*, int64_t*,
                    int64_t*);
int orc_prime_paths_local(int, const int64_t*, const int32_t*, int, int, int, orc_paths*,
                          orc_stats*);
int orc_count(int, const int64_t*, const int32_t*, int, int64_t, orc_stats*, int64_t*, int64_t*,
              int64_t*);
int orc_bruteforce_pp(int, const int64_t*, const int32_t*, orc_paths*, orc_paths*);
int orc_bfs(int, const int64_t*, const int32_t*, int, int, int32_t*, int32_t*, int32_t*, int32_t*);
int orc_bruteforce_lexmin_shortest(int, const int64_t*, const int32_t*, int, int, int32_t*, int);
int orc_test_paths(int, const int64_t*, const int32_t*, int, int, const orc_paths*, orc_paths*,
                   int64_t*);
int orc_test_paths_greedy(int, const int64_t*, const int32_t*, int, int, const orc_paths*,
                          orc_paths*);
void orc_digest(int64_t, const int64_t*, const int32_t*, uint64_t*);
int orc_set_digests(int, const int64_t*, const int32_t*, int, int, int, int, int64_t*, uint64_t*,
                    int64_t*, int64_t*, uint64_t*);
}

namespace {

uint64_t rng_state = 0x2545F4914F6CDD1Dull;
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
  std::vector<int32_t> ci{0};
};

// A spine 0 -> ... -> n-1 plus random arcs between inner vertices (a CFG:
// every vertex reachable from 0 and reaching n-1), or any random digraph.
Csr graph(int n, int extra, bool cfg) {
  std::vector<std::vector<int32_t>> out(n);
  if (cfg)
    for (int v = 0; v + 1 < n; ++v) out[v].push_back(v + 1);
  for (int k = 0; k < extra; ++k) {
    const int a = cfg ? (n > 2 ? 1 + below(n - 2) : 0) : below(n);
    const int b = cfg ? (n > 2 ? 1 + below(n - 2) : 0) : below(n);
    if (cfg && n <= 2) break;
    out[a].push_back(b);
  }
  Csr g;
  g.n = n;
  g.ci.clear();
  for (int v = 0; v < n; ++v) {
    for (int w : out[v]) g.ci.push_back(w);
    g.rp.push_back((int64_t)g.ci.size());
  }
  if (g.ci.empty()) g.ci.push_back(0);
  return g;
}

}  // namespace

int main() {
  int bad = 0;
  for (int it = 0; it < 400; ++it) {
    const bool cfg = it % 2 == 0;
    const int n = 2 + below(cfg ? 16 : 7);
    Csr g = graph(n, below(cfg ? n + 1 : 2 * n + 1), cfg);
    const int64_t* rp = g.rp.data();
    const int32_t* ci = g.ci.data();
    orc_paths pp{}, loc{}, bf{}, all{}, tp{}, gr{};
    orc_stats st{}, st2{}, st3{};
    std::vector<int64_t> lv(n + 2), cy(n + 2), per(n);
    orc_prime_paths(n, rp, ci, 1 + it % 4, &pp, &st, lv.data(), cy.data());
    orc_prime_paths_local(n, rp, ci, 0, n, 1 + it % 3, &loc, &st2);
    orc_count(n, rp, ci, 3, it % 5 == 0 ? 50 : 0, &st3, lv.data(), cy.data(), per.data());
    if (st.n_pp != st2.n_pp || st.n_pp != st.n_pp_local) bad = 1;
    if (n <= 7 && orc_bruteforce_pp(n, rp, ci, &bf, &all) == 0 && bf.n_paths != pp.n_paths) bad = 1;
    std::vector<int32_t> df(n), par(n), db(n), nx(n), buf(n + 1);
    orc_bfs(n, rp, ci, 0, n - 1, df.data(), par.data(), db.data(), nx.data());
    if (n <= 10) orc_bruteforce_lexmin_shortest(n, rp, ci, 0, n - 1, buf.data(), n + 1);
    int64_t nsp = 0;
    uint64_t d[2], pd[2], td[2];
    if (orc_test_paths(n, rp, ci, 0, n - 1, &pp, &tp, &nsp) == 0) {
      orc_test_paths_greedy(n, rp, ci, 0, n - 1, &pp, &gr);
      int64_t ntp = 0, nsp2 = 0;
      orc_set_digests(n, rp, ci, 0, n - 1, 1 + it % 4, 1 + it % 5, per.data(), pd, &ntp, &nsp2, td);
      orc_digest(tp.n_paths, tp.offsets, tp.vertices, d);
      if (ntp != tp.n_paths || d[0] != td[0] || d[1] != td[1] || nsp2 != nsp) bad = 1;
    }
    orc_digest(pp.n_paths, pp.offsets, pp.vertices, d);
    for (orc_paths* p : {&pp, &loc, &bf, &all, &tp, &gr}) orc_free_paths(p);
  }
  std::printf(bad ? "oracle routines disagree\n" : "oracle driver ok\n");
  return bad;
}
