/* Drives the CPU oracle (oracle/oracle.c) with several worker threads on a
 * seeded R-MAT graph, for builds under AddressSanitizer + UndefinedBehavior-
 * Sanitizer or ThreadSanitizer (tests/test_sanitizers.py). It checks
 * identities that hold for any correct build (the certificate accepts every
 * BFS, per-source sums add up to the per-target sums of Eq. 4, msBFS rows
 * equal single-source BFS) and exits with status 0 only if all hold. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void gg_free(void *h);
int64_t gg_n(const void *h);
const int32_t *gg_row_ptr(const void *h);
const int32_t *gg_col(const void *h);
void *gg_rmat(int32_t scale, int32_t edgefactor, double a, double b, double c, uint64_t seed, int32_t permute,
              int32_t threads);
int32_t oracle_bfs(int64_t n, const int32_t *rp, const int32_t *col, int32_t src, int32_t *level);
int64_t oracle_components(int64_t n, const int32_t *rp, const int32_t *col, int32_t *label);
int32_t oracle_msbfs16(int64_t n, const int32_t *rp, const int32_t *col, const int32_t *srcs, int64_t k,
                       int16_t *out, int32_t threads);
int32_t oracle_closeness(int64_t n, const int32_t *rp, const int32_t *col, const int32_t *srcs, int64_t k,
                         int64_t *sums, int64_t *reach, double *cc, int32_t threads);
int32_t oracle_far(int64_t n, const int32_t *rp, const int32_t *col, const int32_t *srcs, int64_t k, int64_t *far,
                   int32_t threads);
int32_t oracle_certificate(int64_t n, const int32_t *rp, const int32_t *col, int32_t src, const int32_t *level,
                           int64_t *where);
int32_t oracle_bvss_count(int64_t n, const int32_t *rp, const int32_t *col, int32_t sigma, int32_t tau,
                          int64_t *nslices, int64_t *nvss);
int32_t oracle_bvss_fill(int64_t n, const int32_t *rp, const int32_t *col, int32_t sigma, int32_t tau,
                         int64_t *real_ptrs, int64_t *v2r, int64_t *slice_ptr, int32_t *rows, uint64_t *masks);

static int failures = 0;
#define EXPECT(cond, what)                                     \
  do {                                                         \
    if (!(cond)) {                                             \
      fprintf(stderr, "FAILED: %s (%s)\n", what, #cond);      \
      ++failures;                                              \
    }                                                          \
  } while (0)

int main(void) {
  void *g = gg_rmat(13, 16, 0.57, 0.19, 0.19, 94, 1, 8);
  if (!g) return 2;
  const int64_t n = gg_n(g);
  const int32_t *rp = gg_row_ptr(g), *col = gg_col(g);
  const int64_t k = 40;
  int32_t *srcs = malloc(sizeof(int32_t) * k);
  for (int64_t i = 0; i < k; ++i) srcs[i] = (int32_t)((i * 2654435761u) % (uint64_t)n);
  int32_t *lev = malloc(sizeof(int32_t) * n);
  int16_t *ms = malloc(sizeof(int16_t) * n * k);
  int64_t *sums = malloc(sizeof(int64_t) * k), *reach = malloc(sizeof(int64_t) * k), *far = malloc(sizeof(int64_t) * n);
  double *cc = malloc(sizeof(double) * k);
  int32_t *lab = malloc(sizeof(int32_t) * n);
  EXPECT(oracle_components(n, rp, col, lab) > 0, "components");
  EXPECT(oracle_msbfs16(n, rp, col, srcs, k, ms, 8) == 0, "msbfs16");
  for (int64_t i = 0; i < k; ++i) {
    int64_t where = 0;
    EXPECT(oracle_bfs(n, rp, col, srcs[i], lev) >= 0, "bfs");
    EXPECT(oracle_certificate(n, rp, col, srcs[i], lev, &where) == 0, "certificate accepts the BFS");
    int same = 1;
    for (int64_t v = 0; v < n; ++v) same &= ms[i * n + v] == lev[v];
    EXPECT(same, "msBFS row equals single-source BFS");
  }
  EXPECT(oracle_closeness(n, rp, col, srcs, k, sums, reach, cc, 8) == 0, "closeness");
  EXPECT(oracle_far(n, rp, col, srcs, k, far, 8) == 0, "far");
  int64_t s1 = 0, s2 = 0;
  for (int64_t i = 0; i < k; ++i) s1 += sums[i];
  for (int64_t v = 0; v < n; ++v) s2 += far[v];
  EXPECT(s1 == s2, "sum of per-source sums equals sum of per-target sums");
  int64_t nsl = 0, nvss = 0;
  EXPECT(oracle_bvss_count(n, rp, col, 8, 128, &nsl, &nvss) == 0, "bvss_count");
  const int64_t nsets = (n + 7) / 8;
  int64_t *real_ptrs = malloc(sizeof(int64_t) * (nsets + 1)), *v2r = malloc(sizeof(int64_t) * (nvss + 1));
  int64_t *slice_ptr = malloc(sizeof(int64_t) * (nsets + 1));
  int32_t *rows = malloc(sizeof(int32_t) * (nsl + 1));
  uint64_t *masks = malloc(sizeof(uint64_t) * (nsl + 1));
  EXPECT(oracle_bvss_fill(n, rp, col, 8, 128, real_ptrs, v2r, slice_ptr, rows, masks) == 0, "bvss_fill");
  int64_t bits = 0;
  for (int64_t i = 0; i < nsl; ++i) bits += __builtin_popcountll(masks[i]);
  EXPECT(bits == rp[n], "one mask bit per directed edge");
  free(srcs); free(lev); free(ms); free(sums); free(reach); free(far); free(cc); free(lab);
  free(real_ptrs); free(v2r); free(slice_ptr); free(rows); free(masks);
  gg_free(g);
  printf("oracle_check: %d failures\n", failures);
  return failures == 0 ? 0 : 1;
}
