/*
 * blest.h -- C ABI of the MI355X (gfx950) BVSS breadth-first-search library.
 *
 * The library implements the data-parallel hot path of "Graph Traversal on
 * Tensor Cores: A BFS Framework for Modern GPUs" (BLEST): level-synchronous
 * BFS written as a Boolean-semiring sparse-matrix / sparse-frontier product
 * (Background, Eq. 1 and Eq. 2) over Binarized Virtual Slice Sets (Section
 * BVSS), with lazy visited marking (Section "Lazy Vertex Updates", Alg. 3),
 * top-down / bottom-up switching (Section "Switching Mechanism", Eq. 3,
 * Alg. 4), multi-source BFS (Section "Multi-Source BFS", Alg. 5) and
 * closeness centrality (Section "Closeness Centrality", Eq. 4 and Eq. 5).
 *
 * Conventions for every entry point:
 *  - Graphs are undirected and simple: the CSR must be symmetric, rows sorted
 *    strictly ascending, no self loops. Vertex ids are int32.
 *  - "host" pointers are ordinary CPU memory, borrowed for the call only.
 *    "dev" pointers are device memory on the graph's device (e.g. torch
 *    tensors), owned by the caller.
 *  - `stream` is a hipStream_t (NULL = the null stream). Work is ordered on
 *    it. Unless a graph is built with opts.async = 1, each call waits for
 *    its stream before returning so that device-side errors are reported by
 *    the call itself.
 *  - Calls that use one graph must not overlap (the graph owns its working
 *    buffers); serialise them on one stream.
 *  - Every entry point returns a blest_status; on failure
 *    blest_last_error() holds a thread-local message. Output buffers are
 *    unspecified after a failure.
 */
#ifndef BLEST_H
#define BLEST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t blest_status;
#define BLEST_OK 0
#define BLEST_ERR_INVALID_ARG (-1)   /* NULL/size/option errors */
#define BLEST_ERR_INVALID_GRAPH (-2) /* CSR not symmetric/sorted/simple, n <= 0, m >= 2^31 */
#define BLEST_ERR_OUT_OF_RANGE (-3)  /* a source vertex outside [0, n) */
#define BLEST_ERR_OOM (-4)           /* host or device allocation failed */
#define BLEST_ERR_HIP (-5)           /* a HIP runtime call failed */
#define BLEST_ERR_OVERFLOW (-6)      /* an int16 level would exceed 32767 */
#define BLEST_ERR_UNSUPPORTED (-7)   /* option not supported (e.g. sigma) */
#define BLEST_ERR_TIMEOUT (-8)       /* a device-wide barrier exceeded its spin bound */
#define BLEST_ERR_NO_DEVICE (-9)     /* no usable gfx950 device */
#define BLEST_ERR_IO (-10)           /* a checkpoint file could not be read or written */

/* Short name of a status code (static string). */
const char* blest_status_str(blest_status s);
/* Detail of the last failure on the calling thread (static per thread). */
const char* blest_last_error(void);

typedef struct blest_graph blest_graph;

/* Host CSR of an undirected simple graph: row_ptr[n+1], col_idx[m]. */
typedef struct {
  int64_t n;
  int64_t m;
  const int32_t* row_ptr;
  const int32_t* col_idx;
} blest_csr;

/* Engine choice per BFS level (Section "Switching Mechanism"). */
#define BLEST_POLICY_HEURISTIC 0  /* Eq. 3: bottom-up iff #unvisited < eta*|Q|, else BVSS top-down */
#define BLEST_POLICY_BVSS 1       /* plain method: BVSS top-down every level */
#define BLEST_POLICY_PUSH 2       /* scalar top-down (push over CSR) every level */
#define BLEST_POLICY_BOTTOM_UP 3  /* bottom-up (Alg. 4) every level */
#define BLEST_POLICY_LEARNED 4    /* switch MLP (blest_set_switch_model); Eq. 3 fallback */
#define BLEST_POLICY_RANDOM 5     /* seeded random engine per level (engine-independence tests) */

/* Engine ids reported in blest_level_stat.engine. */
#define BLEST_ENGINE_BVSS 0
#define BLEST_ENGINE_PUSH 1
#define BLEST_ENGINE_BOTTOM_UP 2

#define BLEST_REORDER_NONE 0
#define BLEST_REORDER_RCM 1  /* Reverse Cuthill-McKee (Section "Boosting Cache Locality") */
#define BLEST_REORDER_AUTO 2 /* JaccardWithWindows if the degree distribution is scale-free-like (footnote
                                of that section), RCM otherwise (Section "Reordering the Graph") */
#define BLEST_REORDER_JACCARD 3 /* JaccardWithWindows (Section "Increasing Compression Ratio") */

typedef struct {
  int32_t sigma;        /* slice-set width in columns: 8 (default), 16 or 32 */
  int32_t tau;          /* max slices per virtual slice set: 64, 128 (default) or 256 */
  int32_t reorder;      /* BLEST_REORDER_* (default AUTO) */
  int32_t policy;       /* BLEST_POLICY_* (default HEURISTIC) */
  float eta;            /* Eq. 3 switching constant (default 10) */
  int32_t block_size;   /* threads per workgroup of the persistent kernel: 256, 512 (default) or 1024 */
  int32_t blocks_per_cu;/* persistent workgroups per compute unit, 0 = as many as fit */
  int32_t persistent;   /* 1 (default): one cooperative launch per BFS; 0: one launch per stage */
  int32_t wide_slices;  /* 1: 64-bit slices (row | mask) even where 32-bit packing fits */
  int32_t prefilter;    /* 1 (default): skip marking rows already visited */
  int32_t async;        /* 1: calls return without waiting for the stream (see blest_sync) */
  int32_t msbfs_width;  /* sources per multi-source batch: 64, 128, 256 or 512 (default 512) */
  uint64_t random_seed; /* seed of BLEST_POLICY_RANDOM */
  int32_t device;       /* HIP device ordinal, -1 = current device */
  int32_t single_block; /* 1 (default): levels whose Stage 1 can mark at most 4096 rows run on one
                           workgroup with workgroup barriers instead of device-wide ones */
  int32_t panel;        /* panel-blocked BVSS copy for dense top-down levels (sigma = 8, 32-bit
                           slices only): 0 = not built, 1 (default) = used when the queued slices
                           are at least an eighth of all slices, 2 = used at every BVSS level */
  int32_t panel_log2_rows; /* rows per panel = 2^this, in [5, 15]; 0 (default) = about one panel
                              per persistent workgroup */
  int32_t stage2_count_first; /* Stage 2 of a grid level either builds the frontier lists in the same
                                 pass as the visited update, or counts first and writes the lists
                                 only if the next level's engine reads them (one more device-wide
                                 barrier then). 0: same pass always; 1 (default): count first after a
                                 bottom-up or panel step or a frontier of mean degree >= 8; 2: count
                                 first always */
  int32_t msbfs_graph;  /* 1: multi-source BFS and closeness run as a hipGraph of per-phase kernels
                           (batch set-up, each level's engine and Stage 2, batch reduction),
                           replayed until done, instead of one persistent launch (default 0) */
  int32_t jaccard_window; /* window width W of BLEST_REORDER_JACCARD: a multiple of sigma greater
                             than sigma; 0 (default) = 1024 */
  int32_t update_scheme;  /* BLEST_UPDATE_*: how a single-source top-down level updates the vertices
                             it reaches (default AUTO) */
  int32_t directed;       /* 1: the CSR lists the out-arcs of a directed graph (A[i][j] = 1 iff arc
                             j -> i, Background); levels are distances along arcs. 0 (default): the
                             CSR must be symmetric */
  int32_t ms_ablation;    /* multi-source steps switched off, for the paper's ablation (Section
                             "Ablation Studies", MS-BFS): BLEST_MS_NO_GETVI | BLEST_MS_NO_DIRTY;
                             0 (default) = the full method. Results are unchanged */
  int32_t ms_mfma;        /* 1: the multi-source top-down neighbour check as an int8 matrix product on
                             the matrix cores (sigma = 8; an experiment against the bitwise check,
                             same results). 0 (default): bitwise */
  int32_t reserved;
} blest_opts;

/* Multi-source ablation flags (Section "Ablation Studies", MS-BFS: (A) drops
 * both, (AB) drops the tracking): NO_GETVI keeps the vertex words in vertex
 * order instead of the getVI remap (Section "Multi-Source BFS"); NO_DIRTY
 * drops the dynamic slice-set tracking (activeSets / dirtySets): every slice
 * set is finalised, all its words count as active and all its VSSs are queued
 * at every level. */
#define BLEST_MS_NO_GETVI 1
#define BLEST_MS_NO_DIRTY 2

/* Vertex update schemes of single-source BFS. LAZY: Alg. 3 (marks in Stage 1,
 * a Stage 2 pass builds the next frontier and queue; Section "Lazy Vertex
 * Updates"). EAGER: Alg. 2 (each hit sets the level and the next-frontier bit
 * at once; the first writer of a slice set enqueues its VSSs; one device-wide
 * barrier per level). AUTO: the paper's dispatch (Section "Ablation
 * Studies"): EAGER iff the built graph's update divergence U_div <= 25,000.
 * EAGER levels run the BVSS top-down engine or the bottom-up engine (a push
 * choice runs BVSS top-down); probe mode (blest_bfs_probe) always runs LAZY. */
#define BLEST_UPDATE_LAZY 0
#define BLEST_UPDATE_EAGER 1
#define BLEST_UPDATE_AUTO 2

/* Fills *opts with the defaults listed above. */
void blest_default_opts(blest_opts* opts);

/* Builds the BVSS of a CSR on the device (Section BVSS). The CSR is copied;
 * *out is owned by the caller until blest_free. opts may be NULL.
 * Directed graphs (opts.directed = 1): the slices of a set are the out-arcs
 * of its columns, the bottom-up engines read a transposed copy (in-arcs,
 * Alg. 4), and RCM or JaccardWithWindows orders the underlying undirected
 * graph. Every output (levels, multi-source levels, sums, reach, far) then
 * follows arcs from the sources.
 * Errors: INVALID_GRAPH (not symmetric unless directed, unsorted, self loops,
 * duplicates, n <= 0, m >= 2^31), UNSUPPORTED (sigma/tau), OOM, HIP, NO_DEVICE. */
blest_status blest_build(const blest_csr* csr, const blest_opts* opts, blest_graph** out);

/* Releases every host and device resource of g. NULL is a no-op. */
void blest_free(blest_graph* g);

/* Single-source BFS (Alg. 3 with the Eq. 3 switch and Alg. 4):
 * levels_dev[v] = hop distance from src, -1 if unreachable, in input vertex
 * ids. levels_dev: int32[n] device memory.
 * Errors: OUT_OF_RANGE (src), INVALID_ARG (NULL), TIMEOUT, HIP. */
blest_status blest_bfs(blest_graph* g, int32_t src, int32_t* levels_dev, void* stream);

/* Same result as blest_bfs, but at every level all three engines run from the
 * same state and are timed (device clock); the per-level log then holds the
 * three times (probe mode, used to label switch training data). */
blest_status blest_bfs_probe(blest_graph* g, int32_t src, int32_t* levels_dev, void* stream);

/* Multi-source BFS (Alg. 5): levels_dev[c*n + v] = d(srcs_host[c], v) as int16,
 * -1 if unreachable, source-major, input vertex ids. levels_dev: int16[k*n].
 * Sources may repeat; k = 0 is a no-op. Batches of opts.msbfs_width sources.
 * The graph keeps, from the first call on, a staging buffer of
 * n * (widest batch) int16 (plus an int32[n] id map for a relabelled graph)
 * through which each batch's levels reach levels_dev; blest_free releases it.
 * Errors: OUT_OF_RANGE, OVERFLOW (a distance > 32767; levels then unspecified),
 * INVALID_ARG, TIMEOUT, OOM, HIP. */
blest_status blest_msbfs(blest_graph* g, const int32_t* srcs_host, int32_t k, int16_t* levels_dev, void* stream);

/* blest_msbfs for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): same
 * arguments, same result, and no hipMalloc/hipFree or allocating library call.
 * The source list and the batch plan go to a static device array of
 * BLEST_MSBFS_NOALLOC_MAX_SOURCES + BLEST_MSBFS_NOALLOC_MAX_SOURCES / 16 int32
 * (278,528 bytes) that each device holds until the process ends; the graph's
 * multi-source working buffers must already exist, i.e. an earlier
 * blest_msbfs, blest_msbfs_batched, blest_closeness or blest_far call on this
 * graph used a batch width of at least opts.msbfs_width. Always one
 * persistent launch (opts.msbfs_graph is ignored); the call waits for the
 * stream twice while staging the sources and the plan (host memory is read
 * through a fixed buffer). Calls that overlap on one device race on that array
 * (as calls on one graph race on the graph): serialise them.
 * Errors: INVALID_ARG (k > BLEST_MSBFS_NOALLOC_MAX_SOURCES, NULL pointers),
 * UNSUPPORTED (the graph's multi-source buffers are not allocated yet), and
 * those of blest_msbfs. */
#define BLEST_MSBFS_NOALLOC_MAX_SOURCES 65536
blest_status blest_msbfs_noalloc(blest_graph* g, const int32_t* srcs_host, int32_t k, int16_t* levels_dev,
                                 void* stream);

/* Multi-source BFS with an explicit batch plan: the k sources are split, in
 * order, into consecutive batches of widths[0], widths[1], ... sources (each
 * 64, 128, 256 or 512; the last width repeats), all run in one persistent
 * launch. Output and errors as blest_msbfs. */
blest_status blest_msbfs_batched(blest_graph* g, const int32_t* srcs_host, int32_t k, const int32_t* widths_host,
                                 int32_t nwidths, int16_t* levels_dev, void* stream);

/* Closeness inputs per source (Eq. 4, Eq. 5, normalised per source):
 * sums_dev[c] = sum of d(srcs[c], v) over reachable v (int64),
 * reach_dev[c] = number of reachable vertices including srcs[c] (int64),
 * cc_dev[c] = (reach-1)/sum in IEEE double, 0 when sum = 0.
 * Any of the three output pointers may be NULL. */
blest_status blest_closeness(blest_graph* g, const int32_t* srcs_host, int64_t k, int64_t* sums_dev,
                             int64_t* reach_dev, double* cc_dev, void* stream);

/* Closeness with a checkpoint file, for runs long enough to be interrupted
 * (all sources of a large graph). Same outputs as blest_closeness. Sources
 * are processed in order, in chunks of up to 64 batches; after each chunk the
 * per-source sums and reach counts finished so far are written to `path`
 * (host file: a header with n, m, k and a hash of the source list, then the
 * finished sources' sums and reach; replaced atomically by rename). A call
 * that finds a matching file resumes after its finished sources and copies
 * their results to the outputs (cc recomputed as (reach-1)/sum). max_sources
 * > 0 stops after about that many new sources (whole chunks of at most that
 * size); 0 runs to the end. *done = sources finished in total (k when
 * complete); outputs are valid for [0, *done). The call waits for `stream`.
 * Errors: as blest_closeness; INVALID_ARG (NULL path or done, or a file
 * written for another graph or source list); IO (file cannot be read or
 * written). */
blest_status blest_closeness_resumable(blest_graph* g, const int32_t* srcs_host, int64_t k, int64_t* sums_dev,
                                       int64_t* reach_dev, double* cc_dev, const char* path, int64_t max_sources,
                                       int64_t* done, void* stream);

/* Per-target distance sums of Eq. 4 (Closeness Centrality): far_dev[v] =
 * sum over the k sources c that reach v of d(srcs[c], v), in input vertex ids;
 * far_dev: int64[n] device memory, overwritten. Paper's normalisation for a
 * connected graph with all vertices as sources: cc(v) = (n-1)/far(v) (Eq. 5).
 * Sources may repeat (each counts). Errors as blest_closeness. */
blest_status blest_far(blest_graph* g, const int32_t* srcs_host, int64_t k, int64_t* far_dev, void* stream);

/* Same result as blest_msbfs_batched, but every level runs both multi-source
 * engines (BVSS and bottom-up) from the same state and times each (device
 * clock), for switch training data (persistent launch; returns after the
 * stream syncs). Records via blest_msbfs_last_levels. */
blest_status blest_msbfs_probe(blest_graph* g, const int32_t* srcs_host, int32_t k, const int32_t* widths_host,
                               int32_t nwidths, int16_t* levels_dev, void* stream);

/* Per-level record of the last multi-source call (all batches in order). */
typedef struct {
  int32_t batch, level;
  int32_t engine;          /* BLEST_ENGINE_BVSS or _BOTTOM_UP (-1 in probe mode) */
  int32_t mlp_fallback;    /* learned policy: 1 if the pairs rule decided */
  int32_t width;           /* sources in the batch */
  int32_t live;            /* traversals whose frontier is non-empty at this level */
  int64_t new_pairs;       /* (vertex, traversal) pairs at this level */
  int64_t queue;           /* VSSs queued */
  int64_t queue_slices;
  int64_t unvisited_pairs;
  double t_engine_us[2];   /* probe mode: BVSS, bottom-up; else -1 */
  float feat[12];          /* the multi-source switch network's inputs */
} blest_ms_level_stat;

/* Copies up to cap records of the last multi-source call to buf (host);
 * *nrec = records written by the call. Errors: INVALID_ARG, HIP. */
blest_status blest_msbfs_last_levels(const blest_graph* g, blest_ms_level_stat* buf, int32_t cap, int32_t* nrec);

/* With opts.async = 1: waits for `stream` and reports device-side errors of the
 * calls enqueued since the last sync (TIMEOUT, OVERFLOW). */
blest_status blest_sync(blest_graph* g, void* stream);

/* Enables (on != 0) counting of the adjacency entries each level's engine
 * reads (blest_level_stat.work). Off by default: the count costs one device
 * atomic per workgroup before every Stage 1 barrier. Probe mode always counts. */
blest_status blest_set_log_work(blest_graph* g, int32_t on);

/* Changes the level-engine policy of an existing graph (BLEST_POLICY_*). */
blest_status blest_set_policy(blest_graph* g, int32_t policy, float eta, uint64_t random_seed);

typedef struct {
  int64_t n, m;
  int32_t sigma, tau;
  int32_t slice_bytes;   /* 4 (packed row<<8 | mask) or 8 (row<<32 | mask) */
  int32_t reordered;     /* 1 if RCM was applied, 3 if JaccardWithWindows, 0 if neither */
  int64_t n_slice_sets;  /* N_s = ceil(n / sigma) */
  int64_t n_vss;         /* N_v */
  int64_t n_slices;
  int64_t bvss_bytes;    /* device bytes of slices + slice-set offsets */
  int64_t csr_bytes;     /* device bytes of the CSR copy */
  int64_t work_bytes;    /* device bytes of BFS working buffers */
  int32_t grid_blocks;   /* persistent grid size */
  int32_t block_size;
  int32_t device;
  int32_t panel_log2_rows; /* rows per panel of the panel-blocked copy = 2^this; 0 if not built */
  int32_t update_scheme;   /* BLEST_UPDATE_LAZY or BLEST_UPDATE_EAGER: the scheme traversals use */
  int32_t directed;        /* 1 if built from a directed CSR */
  int32_t ms_graph_captures; /* multi-source graph mode (msbfs_graph = 1): hipGraphs built so far;
                                one per kernel variant, grid and LDS size, reused by later calls */
  int32_t reserved;
  double u_div;            /* update divergence of the built BVSS (after reordering); see
                              blest_update_divergence */
} blest_graph_stats;

/* Fills *out with structure sizes. Errors: INVALID_ARG. */
blest_status blest_graph_info(const blest_graph* g, blest_graph_stats* out);

/* JaccardWithWindows on the host (Alg. "JaccardWithWindows", Section
 * "Increasing Compression Ratio"): the relabelling BLEST_REORDER_JACCARD
 * applies before building the BVSS. Columns are grouped, window by window
 * (ids [wW, wW + W)), into slice sets of sigma columns: each set starts from
 * the window's highest-degree unassigned column and grows by the unassigned
 * column j sharing rows with the set's row union R that maximises
 * inter(j) / (|R| + deg(j) - inter(j)), or by the highest-degree one when no
 * column shares a row. Ties go to the smaller id; a last window narrower than
 * a multiple of sigma ends with a partial set. csr must be undirected and
 * simple (as for blest_build). new_of_old (host, n int32): the new id of every
 * vertex; each id stays inside its window. No device is used.
 * Errors: INVALID_ARG (NULL, sigma < 1, window not a multiple of sigma or not
 * greater than it), INVALID_GRAPH, OOM. */
blest_status blest_reorder_jaccard(const blest_csr* csr, int32_t sigma, int32_t window, int32_t* new_of_old);

/* Update divergence U_div (Section "Boosting Cache Locality") of the BVSS of
 * csr as given (no reordering) with slice-set width sigma and tau slices per
 * VSS: each VSS is a (tau/32) x ... matrix of 32 rows and theta = tau / 32
 * columns, slice j in column j mod theta; a column's divergence is the
 * population standard deviation of its slices' row ids, a VSS's divergence
 * the mean over its non-empty columns, U_div the mean over all VSSs (0 if
 * there are none). Host only, no device needed. Errors: INVALID_ARG,
 * INVALID_GRAPH, UNSUPPORTED (sigma/tau), OOM. */
blest_status blest_update_divergence(const blest_csr* csr, int32_t sigma, int32_t tau, double* u_div);

/* Per-level record of the last single-source BFS (Alg. 3, Stage 2 statistics). */
typedef struct {
  int32_t level;        /* frontier level l; the record describes the step l -> l+1 */
  int32_t engine;       /* BLEST_ENGINE_* that produced level l+1 (-1 for the last level) */
  int64_t frontier;     /* |F_l| vertices */
  int64_t queue;        /* |Q_l| virtual slice sets */
  int64_t queue_slices; /* slices in Q_l */
  int64_t frontier_edges;  /* m_f: sum of degrees of F_l */
  int64_t unvisited;    /* n - #visited through level l */
  int64_t unvisited_edges; /* m_u: sum of degrees of unvisited vertices */
  int64_t deg_ge_32;    /* frontier vertices with degree >= 32 */
  int64_t deg_ge_1024;  /* frontier vertices with degree >= 1024 */
  double t_step_us;     /* device time of the chosen engine's step plus finalisation */
  double t_stage1_us;   /* device time of the engine's step alone (Stage 1 and its barrier) */
  double t_engine_us[3];/* probe mode: time of each engine from the same state; else -1 */
  int32_t mlp_fallback; /* learned policy: 1 if Eq. 3 was used (input out of range) */
  int32_t bvss_panel;   /* 1 if the BVSS step read the panel-blocked copy (all slices, LDS marks) */
  int64_t work;         /* adjacency entries read by the step's engine: slices (BVSS),
                           CSR edges (push, bottom-up); probe mode: all three engines */
  double t_count_us;    /* grid levels: time from the step's start until Stage 2's statistics
                           were known (before any list emission); 0 for one-workgroup levels */
} blest_level_stat;

/* Copies up to cap records of the last BFS to buf (host); *nlevels = number
 * of frontier levels (max level + 1). Errors: INVALID_ARG. */
blest_status blest_last_level_stats(const blest_graph* g, blest_level_stat* buf, int32_t cap, int32_t* nlevels);

/* Copies the BVSS to host buffers (internal vertex ids; see perm):
 * real_ptrs[N_s+1], v2r[N_v] (virtualToReal), slice_ptr[N_s+1],
 * slice_row[n_slices], slice_mask[n_slices] (bit b = column s*sigma+b),
 * perm[n] (input id -> internal id). Any pointer may be NULL. */
blest_status blest_export_bvss(const blest_graph* g, int64_t* real_ptrs, int64_t* v2r, int64_t* slice_ptr,
                               int32_t* slice_row, uint64_t* slice_mask, int32_t* perm);

/* ---- learned switch (not in the paper; its Conclusion names a more robust
 * switching criterion as future work) ------------------------------------ */

#define BLEST_MLP_IN 12
#define BLEST_MLP_HIDDEN 64
#define BLEST_MLP_OUT 3
/* Flat parameter count: W1[64][12], b1[64], W2[64][64], b2[64], W3[3][64], b3[3]. */
#define BLEST_MLP_NPARAMS 5187

/* Installs switch-network weights (host arrays) used by BLEST_POLICY_LEARNED:
 * params[BLEST_MLP_NPARAMS]; mean[12], std[12] standardise the features.
 * g = NULL sets the default for graphs built afterwards.
 * Errors: INVALID_ARG (nparams mismatch, std <= 0). */
blest_status blest_set_switch_model(blest_graph* g, const float* params, int32_t nparams, const float* mean,
                                    const float* std);

/* Installs the multi-source switch network (same format; inputs listed at
 * blest_ms_level_stat.feat: log(1+new pairs), log(1+queued slices), shares of
 * new pairs, VSSs, slices and unvisited pairs, log batch width, log |Q| - log
 * unvisited pairs, log live traversals - log batch width, three zeros). Outputs 0 (BVSS) and 2 (bottom-up) are used;
 * any other choice falls back to the pairs rule. g = NULL: default for graphs
 * built afterwards. Errors as blest_set_switch_model. */
blest_status blest_set_ms_switch_model(blest_graph* g, const float* params, int32_t nparams, const float* mean,
                                       const float* std);

/* Minimum softmax probability of the network's choice for BLEST_POLICY_LEARNED
 * (default 0.5), for both networks of g (single- and multi-source); below it,
 * and for standardised inputs outside [-6, 6], the level falls back to Eq. 3
 * (the pairs rule for multi-source levels). A model installed later takes the
 * default again. g = NULL sets the default for later models.
 * Errors: INVALID_ARG (min_prob outside (0, 1]). */
blest_status blest_set_switch_confidence(blest_graph* g, float min_prob);

/* Per-level features (12 floats, the network's inputs before standardising)
 * of the last BFS's levels, to host: feat[nlev][12]. With F the frontier, Q its
 * VSSs, S their slices, m_f its edges, U the unvisited vertices, m_u their
 * edges, N_v / N_slices the BVSS totals, all logarithms base 2:
 * log(1+|F|), log(1+S), log(1+|F|) - log n, log(1+|Q|) - log(1+N_v),
 * log(1+S) - log(1+N_slices), log(1+m_f) - log(1+m), log(1+|U|) - log n,
 * log(1+m_u) - log(1+m), log(1+|Q|) - log(1+|U|) (Eq. 3's ratio), and three
 * reserved zeros. */
blest_status blest_last_level_features(const blest_graph* g, float* feat, int32_t cap, int32_t* nlevels);

/* Forward pass on the device: logits_dev[b][3] for x_dev[b][12] (already
 * standardised), params_dev[BLEST_MLP_NPARAMS]. fp32. */
blest_status blest_mlp_forward(const float* params_dev, const float* x_dev, int32_t batch, float* logits_dev,
                               void* stream);

/* Weighted mean softmax cross-entropy and its gradient on the device:
 * loss_dev[1], grad_dev[BLEST_MLP_NPARAMS]; y_dev int32 labels in {0,1,2};
 * w_dev per-sample weights (NULL = 1). fp32. */
blest_status blest_mlp_loss_grad(const float* params_dev, const float* x_dev, const int32_t* y_dev,
                                 const float* w_dev, int32_t batch, float* loss_dev, float* grad_dev, void* stream);

/* One bias-corrected Adam step (Kingma and Ba) at step t >= 1, in place on
 * params_dev, m_dev, v_dev (n floats each). */
blest_status blest_mlp_adam(float* params_dev, const float* grad_dev, float* m_dev, float* v_dev, int32_t n,
                            int32_t t, float lr, float beta1, float beta2, float eps, void* stream);

/* Full training loop on the device: `steps` Adam steps on minibatches of
 * `batch` samples drawn (counter-based, from `seed`) out of x_dev[nsamples][12],
 * y_dev, w_dev (NULL = 1); loss_log_dev[steps] receives each step's loss (may be
 * NULL). m_dev/v_dev are Adam state (zero them to start). */
blest_status blest_mlp_train(float* params_dev, float* m_dev, float* v_dev, const float* x_dev,
                             const int32_t* y_dev, const float* w_dev, int32_t nsamples, int32_t batch,
                             int32_t steps, float lr, uint64_t seed, float* loss_log_dev, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* BLEST_H */
