/*
 * CPU oracle for BVSS breadth-first search -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this file's library. The GPU library never links or calls it, and
 * it shares no code, header or table with the GPU library.
 *
 * It computes, slowly and plainly, what the method reaches exactly:
 *
 *  - Single-source BFS levels (Background, Eq. 1 and the level definition
 *    that follows it): level[v] is the hop distance from src, level[src] = 0,
 *    and -1 stands for the paper's "infinity" (unreachable). Computed with a
 *    first-in first-out queue, the textbook definition of hop distance.
 *  - Multi-source BFS (Section "Multi-Source BFS", Alg. 5): one independent
 *    BFS per source, int16 levels, error if a distance exceeds 32767.
 *  - Closeness (Section "Closeness Centrality", Eq. 4 and Eq. 5): per-source
 *    distance sums and reachable counts in int64, and the per-target sums
 *    far[u] of Eq. 4 over a source set.
 *  - The BVSS structure (Section "Binarized Virtual Slice Sets"): slice set s
 *    covers columns [s*sigma, (s+1)*sigma); row i has a slice in set s iff it
 *    has a nonzero in those columns; mask bit b of that slice is set iff
 *    A[i][s*sigma+b] = 1, i.e. edge (s*sigma+b, i) exists; each slice set is
 *    split into virtual slice sets of at most tau slices; realPtrs and
 *    virtualToReal map between the two.
 *  - A complete O(m) distance certificate for a claimed level array.
 *
 * Everything is plain C with a dense scratch array; no blocking or fusion.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_ERR_ARG (-1)
#define ORACLE_ERR_OOM (-4)
#define ORACLE_ERR_OVERFLOW (-6)

/* FIFO-queue BFS from src. level has n entries; returns the number of levels
 * (max distance + 1) or a negative error. */
int32_t oracle_bfs(int64_t n, const int32_t *rp, const int32_t *col, int32_t src, int32_t *level) {
  if (n <= 0 || src < 0 || src >= n) return ORACLE_ERR_ARG;
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!queue) return ORACLE_ERR_OOM;
  for (int64_t v = 0; v < n; ++v) level[v] = -1;
  int64_t head = 0, tail = 0;
  level[src] = 0;
  queue[tail++] = src;
  int32_t maxlev = 0;
  while (head < tail) {
    int32_t u = queue[head++];
    for (int32_t p = rp[u]; p < rp[u + 1]; ++p) {
      int32_t v = col[p];
      if (level[v] == -1) {
        level[v] = level[u] + 1;
        if (level[v] > maxlev) maxlev = level[v];
        queue[tail++] = v;
      }
    }
  }
  free(queue);
  return maxlev + 1;
}

/* Connected components of the undirected graph: label[v] = index of v's
 * component, components numbered in order of their smallest vertex (a FIFO
 * BFS from each vertex not yet labelled, in vertex order). Returns the number
 * of components. Used to check reach counts: reach(s) = |component of s|. */
int64_t oracle_components(int64_t n, const int32_t *rp, const int32_t *col, int32_t *label) {
  if (n <= 0) return ORACLE_ERR_ARG;
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!queue) return ORACLE_ERR_OOM;
  for (int64_t v = 0; v < n; ++v) label[v] = -1;
  int64_t ncomp = 0;
  for (int64_t s = 0; s < n; ++s) {
    if (label[s] != -1) continue;
    int64_t head = 0, tail = 0;
    label[s] = (int32_t)ncomp;
    queue[tail++] = (int32_t)s;
    while (head < tail) {
      int32_t u = queue[head++];
      for (int32_t p = rp[u]; p < rp[u + 1]; ++p) {
        int32_t v = col[p];
        if (label[v] == -1) {
          label[v] = (int32_t)ncomp;
          queue[tail++] = v;
        }
      }
    }
    ++ncomp;
  }
  free(queue);
  return ncomp;
}

/* ---- multi-source work split over threads ---------------------------------- */

typedef struct {
  int64_t n;
  const int32_t *rp, *col, *srcs;
  int64_t k;
  int16_t *lev16;            /* k*n, source-major, or NULL */
  int64_t *sums, *reach;     /* k each, or NULL */
  int64_t *far;              /* n, per-thread partial (owned by the job), or NULL */
  int64_t next;              /* next source index to take */
  pthread_mutex_t lock;
  int32_t status;
} job_t;

typedef struct {
  job_t *job;
  int64_t *far_part;
} worker_t;

static void *worker(void *arg) {
  worker_t *w = (worker_t *)arg;
  job_t *j = w->job;
  int32_t *level = (int32_t *)malloc(sizeof(int32_t) * (size_t)j->n);
  if (!level) {
    pthread_mutex_lock(&j->lock);
    j->status = ORACLE_ERR_OOM;
    pthread_mutex_unlock(&j->lock);
    return NULL;
  }
  for (;;) {
    pthread_mutex_lock(&j->lock);
    int64_t c = j->next++;
    pthread_mutex_unlock(&j->lock);
    if (c >= j->k) break;
    int32_t r = oracle_bfs(j->n, j->rp, j->col, j->srcs[c], level);
    if (r < 0) {
      pthread_mutex_lock(&j->lock);
      j->status = r;
      pthread_mutex_unlock(&j->lock);
      continue;
    }
    int64_t sum = 0, reach = 0;
    for (int64_t v = 0; v < j->n; ++v) {
      int32_t d = level[v];
      if (j->lev16) {
        if (d > 32767) {
          pthread_mutex_lock(&j->lock);
          j->status = ORACLE_ERR_OVERFLOW;
          pthread_mutex_unlock(&j->lock);
          d = -1;
        }
        j->lev16[c * j->n + v] = (int16_t)d;
      }
      if (d >= 0) {
        sum += d;
        reach += 1;
        if (w->far_part) w->far_part[v] += d;
      }
    }
    if (j->sums) j->sums[c] = sum;
    if (j->reach) j->reach[c] = reach;
  }
  free(level);
  return NULL;
}

static int32_t run_job(job_t *j, int32_t threads) {
  if (threads < 1) threads = 1;
  if (threads > 256) threads = 256;
  pthread_t tid[256];
  worker_t ws[256];
  pthread_mutex_init(&j->lock, NULL);
  j->next = 0;
  j->status = ORACLE_OK;
  for (int t = 0; t < threads; ++t) {
    ws[t].job = j;
    ws[t].far_part = NULL;
    if (j->far) {
      ws[t].far_part = (int64_t *)calloc((size_t)j->n, sizeof(int64_t));
      if (!ws[t].far_part) {
        for (int q = 0; q < t; ++q) free(ws[q].far_part);
        pthread_mutex_destroy(&j->lock);
        return ORACLE_ERR_OOM;
      }
    }
  }
  for (int t = 0; t < threads; ++t) pthread_create(&tid[t], NULL, worker, &ws[t]);
  for (int t = 0; t < threads; ++t) pthread_join(tid[t], NULL);
  if (j->far) {
    for (int64_t v = 0; v < j->n; ++v) j->far[v] = 0;
    for (int t = 0; t < threads; ++t) {
      for (int64_t v = 0; v < j->n; ++v) j->far[v] += ws[t].far_part[v];
      free(ws[t].far_part);
    }
  }
  pthread_mutex_destroy(&j->lock);
  return j->status;
}

static int32_t check_sources(int64_t n, const int32_t *srcs, int64_t k) {
  if (n <= 0 || k < 0) return ORACLE_ERR_ARG;
  for (int64_t c = 0; c < k; ++c)
    if (srcs[c] < 0 || srcs[c] >= n) return ORACLE_ERR_ARG;
  return ORACLE_OK;
}

/* Multi-source BFS by repetition: lev16[c*n + v] = d(srcs[c], v) or -1. */
int32_t oracle_msbfs16(int64_t n, const int32_t *rp, const int32_t *col, const int32_t *srcs, int64_t k,
                       int16_t *lev16, int32_t threads) {
  int32_t r = check_sources(n, srcs, k);
  if (r) return r;
  job_t j;
  memset(&j, 0, sizeof j);
  j.n = n; j.rp = rp; j.col = col; j.srcs = srcs; j.k = k; j.lev16 = lev16;
  return run_job(&j, threads);
}

/* Per-source closeness inputs: sums[c] = sum of d(srcs[c], v) over reachable v,
 * reach[c] = number of reachable vertices (srcs[c] included), and
 * cc[c] = (reach-1)/sum in IEEE double (0 when sum is 0). */
int32_t oracle_closeness(int64_t n, const int32_t *rp, const int32_t *col, const int32_t *srcs, int64_t k,
                         int64_t *sums, int64_t *reach, double *cc, int32_t threads) {
  int32_t r = check_sources(n, srcs, k);
  if (r) return r;
  job_t j;
  memset(&j, 0, sizeof j);
  j.n = n; j.rp = rp; j.col = col; j.srcs = srcs; j.k = k; j.sums = sums; j.reach = reach;
  r = run_job(&j, threads);
  if (r) return r;
  if (cc)
    for (int64_t c = 0; c < k; ++c) cc[c] = sums[c] ? (double)(reach[c] - 1) / (double)sums[c] : 0.0;
  return ORACLE_OK;
}

/* Per-target sums of Eq. 4: far[u] = sum over sources s of d(s,u), finite pairs only. */
int32_t oracle_far(int64_t n, const int32_t *rp, const int32_t *col, const int32_t *srcs, int64_t k, int64_t *far,
                   int32_t threads) {
  int32_t r = check_sources(n, srcs, k);
  if (r) return r;
  job_t j;
  memset(&j, 0, sizeof j);
  j.n = n; j.rp = rp; j.col = col; j.srcs = srcs; j.k = k; j.far = far;
  return run_job(&j, threads);
}

/* Distance certificate for a claimed level array of a BFS from src on an
 * undirected graph. Returns 0 if every condition holds, otherwise a positive
 * code and the offending vertex in *where:
 *  1: level[src] != 0 or a level below -1
 *  2: an edge with exactly one end reached
 *  3: an edge whose reached ends differ by more than one level
 *  4: a reached v != src with no neighbour at level[v]-1
 * Together these imply level[] equals the true hop distance (a parent chain
 * gives a path of length level[v]; no edge allows a shorter one). */
int32_t oracle_certificate(int64_t n, const int32_t *rp, const int32_t *col, int32_t src, const int32_t *level,
                           int64_t *where) {
  *where = -1;
  if (src < 0 || src >= n) return ORACLE_ERR_ARG;
  if (level[src] != 0) { *where = src; return 1; }
  for (int64_t v = 0; v < n; ++v) {
    int32_t dv = level[v];
    if (dv < -1) { *where = v; return 1; }
    int has_parent = (v == src);
    for (int32_t p = rp[v]; p < rp[v + 1]; ++p) {
      int32_t du = level[col[p]];
      if ((du < 0) != (dv < 0)) { *where = v; return 2; }
      if (dv >= 0) {
        int32_t diff = du - dv;
        if (diff > 1 || diff < -1) { *where = v; return 3; }
        if (du == dv - 1) has_parent = 1;
      }
    }
    if (dv > 0 && !has_parent) { *where = v; return 4; }
  }
  return 0;
}

/* Certificate for a directed graph (rp/col: out-arcs u -> col[p]): level[]
 * is the hop distance from src along arcs iff
 *  1: level[src] = 0 and every level is >= -1;
 *  2: every arc u -> v with u reached has v reached;
 *  3: ... and level[v] <= level[u] + 1;
 *  4: every reached v != src has an in-arc from some u at level[v] - 1.
 * 4 gives a path of length level[v] from src, 3 forbids a shorter one, and 2
 * makes the reached set closed under arcs, so it is exactly what src reaches.
 * The in-arc test of 4 is collected on the way over the out-arcs. */
int32_t oracle_certificate_directed(int64_t n, const int32_t *rp, const int32_t *col, int32_t src,
                                    const int32_t *level, int64_t *where) {
  *where = -1;
  if (src < 0 || src >= n) return ORACLE_ERR_ARG;
  if (level[src] != 0) { *where = src; return 1; }
  uint8_t *parent = (uint8_t *)calloc((size_t)n, 1);
  if (!parent) return ORACLE_ERR_OOM;
  int32_t r = 0;
  for (int64_t u = 0; u < n && !r; ++u) {
    int32_t du = level[u];
    if (du < -1) { *where = u; r = 1; break; }
    if (du < 0) continue;
    for (int32_t p = rp[u]; p < rp[u + 1]; ++p) {
      int32_t v = col[p], dv = level[v];
      if (dv < 0) { *where = v; r = 2; break; }
      if (dv > du + 1) { *where = v; r = 3; break; }
      if (dv == du + 1) parent[v] = 1;
    }
  }
  for (int64_t v = 0; v < n && !r; ++v)
    if (level[v] > 0 && !parent[v]) { *where = v; r = 4; }
  free(parent);
  return r;
}

/* BVSS of the (symmetric) adjacency: counts first. */
int32_t oracle_bvss_count(int64_t n, const int32_t *rp, const int32_t *col, int32_t sigma, int32_t tau,
                          int64_t *nslices, int64_t *nvss) {
  if (n <= 0 || sigma < 1 || sigma > 64 || tau < 1) return ORACLE_ERR_ARG;
  int64_t ns = (n + sigma - 1) / sigma;
  uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
  int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!seen || !rows) { free(seen); free(rows); return ORACLE_ERR_OOM; }
  int64_t total = 0, vss = 0;
  for (int64_t s = 0; s < ns; ++s) {
    int64_t cnt = 0;
    for (int64_t j = s * sigma; j < (s + 1) * sigma && j < n; ++j)
      for (int32_t p = rp[j]; p < rp[j + 1]; ++p)
        if (!seen[col[p]]) { seen[col[p]] = 1; rows[cnt++] = col[p]; }
    for (int64_t q = 0; q < cnt; ++q) seen[rows[q]] = 0;
    total += cnt;
    vss += (cnt + tau - 1) / tau;
  }
  free(seen);
  free(rows);
  *nslices = total;
  *nvss = vss;
  return ORACLE_OK;
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* BVSS arrays: real_ptrs[N_s+1], v2r[N_v], and, per slice in slice-set then
 * ascending-row order, slice_row[] and slice_mask[] (bit b = column s*sigma+b).
 * slice_ptr[N_s+1] gives each slice set's slice range. */
int32_t oracle_bvss_fill(int64_t n, const int32_t *rp, const int32_t *col, int32_t sigma, int32_t tau,
                         int64_t *real_ptrs, int64_t *v2r, int64_t *slice_ptr, int32_t *slice_row,
                         uint64_t *slice_mask) {
  if (n <= 0 || sigma < 1 || sigma > 64 || tau < 1) return ORACLE_ERR_ARG;
  int64_t ns = (n + sigma - 1) / sigma;
  uint64_t *mask = (uint64_t *)calloc((size_t)n, sizeof(uint64_t));
  int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!mask || !rows) { free(mask); free(rows); return ORACLE_ERR_OOM; }
  int64_t out = 0, vss = 0;
  real_ptrs[0] = 0;
  slice_ptr[0] = 0;
  for (int64_t s = 0; s < ns; ++s) {
    int64_t cnt = 0;
    for (int64_t b = 0; b < sigma && s * sigma + b < n; ++b) {
      int64_t j = s * sigma + b;
      for (int32_t p = rp[j]; p < rp[j + 1]; ++p) {
        int32_t i = col[p];
        if (!mask[i]) rows[cnt++] = i;
        mask[i] |= (uint64_t)1 << b;
      }
    }
    qsort(rows, (size_t)cnt, sizeof(int32_t), cmp_i32);
    for (int64_t q = 0; q < cnt; ++q) {
      slice_row[out] = rows[q];
      slice_mask[out] = mask[rows[q]];
      mask[rows[q]] = 0;
      ++out;
    }
    int64_t nv = (cnt + tau - 1) / tau;
    for (int64_t q = 0; q < nv; ++q) v2r[vss + q] = s;
    vss += nv;
    real_ptrs[s + 1] = vss;
    slice_ptr[s + 1] = out;
  }
  free(mask);
  free(rows);
  return ORACLE_OK;
}
