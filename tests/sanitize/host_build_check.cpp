// Drives the library's host-side preprocessing (CSR validation, scale-free
// test, RCM, JaccardWithWindows, relabelling, BVSS and panel construction) on
// seeded graphs, for builds under AddressSanitizer + UndefinedBehaviorSanitizer
// or ThreadSanitizer (tests/test_sanitizers.py). It checks invariants that any
// correct build satisfies (permutations, one mask bit per directed edge, every
// slice present in the panel copy) and exits with status 0 only if all hold.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "host_build.h"

extern "C" {
void gg_free(void* h);
int64_t gg_n(const void* h);
int64_t gg_m(const void* h);
const int32_t* gg_row_ptr(const void* h);
const int32_t* gg_col(const void* h);
void* gg_rmat(int32_t scale, int32_t edgefactor, double a, double b, double c, uint64_t seed, int32_t permute,
              int32_t threads);
void* gg_grid(int32_t side, double p_delete, uint64_t seed, int32_t permute, int32_t threads);
void* gg_erdos_renyi(int64_t n, int64_t npairs, uint64_t seed, int32_t threads);
}

static int failures = 0;
#define EXPECT(cond, what)                                      \
  do {                                                          \
    if (!(cond)) {                                              \
      std::fprintf(stderr, "FAILED: %s (%s)\n", what, #cond);  \
      ++failures;                                               \
    }                                                           \
  } while (0)

static bool is_permutation(const std::vector<int32_t>& p, int64_t n) {
  if (static_cast<int64_t>(p.size()) != n) return false;
  std::vector<char> seen(n, 0);
  for (int32_t x : p) {
    if (x < 0 || x >= n || seen[x]) return false;
    seen[x] = 1;
  }
  return true;
}

static void check_graph(const char* name, int64_t n, const int32_t* rp, const int32_t* col) {
  const int64_t m = rp[n];
  std::string why;
  EXPECT(blest::validate_csr(n, m, rp, col, &why), name);
  if (m > 2) {  // an asymmetric copy must be rejected
    std::vector<int32_t> rp2(rp, rp + n + 1), col2(col, col + m);
    int64_t u = 0;
    while (rp2[u + 1] == rp2[u]) ++u;
    col2.erase(col2.begin() + rp2[u]);
    for (int64_t v = u + 1; v <= n; ++v) --rp2[v];
    EXPECT(!blest::validate_csr(n, m - 1, rp2.data(), col2.data(), &why), "asymmetric CSR rejected");
  }
  (void)blest::is_scale_free_like(n, rp);
  const std::vector<int32_t> rcm = blest::rcm_order(n, rp, col);
  EXPECT(is_permutation(rcm, n), "RCM order is a permutation");
  for (int sigma : {8, 16}) {
    const int64_t window = 1024;
    const std::vector<int32_t> jac = blest::jaccard_order(n, rp, col, sigma, window);
    EXPECT(is_permutation(jac, n), "Jaccard order is a permutation");
    bool inside = true;
    for (int64_t v = 0; v < n; ++v) inside &= jac[v] / window == v / window;
    EXPECT(inside, "Jaccard keeps every vertex in its window");
  }
  std::vector<int32_t> new_of_old, prp, pcol;
  blest::permute_csr(n, rp, col, rcm, new_of_old, prp, pcol);
  EXPECT(blest::validate_csr(n, m, prp.data(), pcol.data(), &why), "relabelled CSR is valid");
  for (int sigma : {8, 16, 32}) {
    for (int tau : {64, 128, 256}) {
      const bool wide = sigma != 8 || tau == 256;
      blest::Bvss b;
      EXPECT(blest::build_bvss(n, prp.data(), pcol.data(), sigma, tau, wide, &b), "build_bvss");
      int64_t bits = 0;
      if (wide)
        for (uint64_t w : b.slices64) bits += __builtin_popcountll(w & 0xffffffffULL);
      else
        for (uint32_t w : b.slices32) bits += __builtin_popcount(w & 0xffu);
      EXPECT(bits == m, "one mask bit per directed edge");
      EXPECT(static_cast<int64_t>(b.slice_ptr.back()) == b.nslices, "slice_ptr ends at the slice count");
      if (!wide) {
        for (int rb : {5, blest::panel_log2_rows(n, 256)}) {
          blest::Panels p;
          if (!blest::build_panels(n, b, rb, &p)) continue;
          int64_t nz = 0;
          for (uint32_t w : p.words) nz += (w & 0xffu) != 0;
          EXPECT(nz == b.nslices, "every slice appears once in the panel copy");
          EXPECT(static_cast<int64_t>(p.ptr.back()) == p.nchunks, "panel chunk offsets end at the chunk count");
        }
      }
    }
  }
}

int main() {
  struct G {
    const char* name;
    void* h;
  } graphs[] = {
      {"rmat14", gg_rmat(14, 16, 0.57, 0.19, 0.19, 91, 1, 8)},
      {"grid128", gg_grid(128, 0.1, 92, 1, 8)},
      {"er16k", gg_erdos_renyi(int64_t(1) << 14, int64_t(8) << 14, 93, 8)},
  };
  for (const G& g : graphs) {
    if (!g.h) {
      std::fprintf(stderr, "FAILED: generator %s\n", g.name);
      ++failures;
      continue;
    }
    check_graph(g.name, gg_n(g.h), gg_row_ptr(g.h), gg_col(g.h));
    gg_free(g.h);
  }
  std::printf("host_build_check: %d failures\n", failures);
  return failures == 0 ? 0 : 1;
}
