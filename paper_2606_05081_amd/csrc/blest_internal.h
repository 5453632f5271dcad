// Internal structures of the BVSS BFS library (host + device).
//
// Device data of one graph (internal vertex ids, after optional RCM):
//   rp[n+1], col[m]          CSR copy (int32), used by the push and pull engines
//   slice_ptr[N_s+1]         first slice of each slice set (uint32)
//   slices[n_slices]         one word per slice, ascending row within a set:
//                            32-bit  (row << 8)  | mask   when sigma = 8, n <= 2^24
//                            64-bit  (row << 32) | mask   otherwise
//   degmask[N_s]             sigma-bit mask of vertices with degree > 0
//   orig_id[n]               internal id -> input id (NULL when not reordered)
//   rp_in, col_in            in-arcs of a directed graph (Alg. 4 reads the CSR
//                            of the transpose); the same arrays as rp, col
//                            for an undirected graph
// A virtual slice set (VSS) is a run of at most tau consecutive slices of one
// slice set, so VSS k of set s covers slices [slice_ptr[s] + k*tau, ...). The
// queue holds one 16-byte descriptor per VSS (first slice, count, frontier
// bits of its set, set id) instead of padding every VSS to tau slices.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

#include "blest.h"

namespace blest {

// Entries past the last chunk base of the panel copy, so that a wave may read
// the bases of a whole batch of consecutive chunks with scalar loads.
constexpr int kPanelBasePad = 8;


constexpr int kStatFields = 12;     // accumulated by Stage 2, one 256-byte line each
constexpr int kStatSlots = 3;       // rotating per-level slots
constexpr int kPad = 32;            // 32 x 8 bytes = 256 bytes
constexpr int kMaxSwitchFeatures = 12;

enum StatField : int {
  F_FRONTIER = 0,  // new frontier vertices (also the frontier-list append cursor)
  F_QUEUE = 1,     // VSS descriptors enqueued (also the queue append cursor)
  F_QSLICES = 2,   // slices covered by those descriptors
  F_FEDGES = 3,    // sum of degrees of new frontier vertices
  F_DEG32 = 4,     // new frontier vertices with degree >= 32
  F_DEG1024 = 5,   // ... >= 1024
  F_LIGHT = 6,     // light-vertex list append cursor (push engine)
  F_HEAVY = 7,     // heavy-vertex edge-chunk list append cursor (push engine)
  F_CUMV = 8,      // vertices visited through this level
  F_CUME = 9,      // sum of degrees of those vertices
  F_WORK = 10,     // adjacency entries (slices or CSR edges) read by the engine that left this level
  F_LIVE = 11,     // multi-source: one 64-bit word per batch word, bit c set iff traversal c gained a vertex
};

// Push-engine work split: vertices of degree <= kLightMax are walked by one
// lane; larger ones are cut into chunks of kHeavyChunk edges walked by a wave.
constexpr int kLightMax = 32;
constexpr int kHeavyChunk = 256;

// Device control block. Fields that many workgroups update sit on their own
// 256-byte lines.
struct alignas(256) Ctl {
  unsigned long long acc[kStatSlots][kStatFields][kPad];
  unsigned int bar_count[kPad * 2];      // top-level arrivals (one per XCD leader, or per block)
  unsigned int bar_gen[kPad * 2];        // top-level generation
  unsigned int xcd_count[8][kPad];       // per-XCD arrivals
  unsigned int xcd_gen[8][kPad];         // per-XCD release flags
  unsigned int xcd_blocks[8][kPad];      // blocks of this launch resident on each XCD
  unsigned int xcd_active[kPad];         // number of XCDs with at least one block
  int error[kPad * 2];   // first device-side error (BLEST_ERR_*), 0 if none
  int done[kPad * 2];    // per-stage launch mode: 1 once the frontier is empty
  int overflow[kPad * 2];
  int single_level[kPad];          // first level after a single-workgroup episode
  unsigned int single_gen[kPad];   // number of finished single-workgroup episodes
  int single_progress[kPad];       // last level a running single-workgroup episode finished
  int nlevels[kPad * 2]; // frontier levels of the last traversal
  int ms_state[2][kPad];   // multi-source graph mode: {phase, batch, level} read by even/odd kernels
  int ms_nrec[kPad];       // multi-source level records written by the last call
};

// One record per level of a multi-source call (all batches in order).
struct MsLevelRec {
  int batch, level, engine, fallback, width, live;  // live: traversals with a non-empty frontier
  long long fresh, queue, qslices, unvisited;  // new pairs, VSSs, slices, unvisited pairs
  unsigned long long t_engine[2];              // probe mode: device ticks of BVSS and bottom-up
  float feat[kMaxSwitchFeatures];
};

// One record per frontier level, written by workgroup 0 of the persistent kernel.
struct LevelRec {
  long long frontier, queue, qslices, fedges, unvisited, unvisited_edges, deg32, deg1024;
  long long work;                 // adjacency entries read by the step's engine
  unsigned long long t_begin;     // device clock (100 MHz) when the step started
  unsigned long long t_mid;       // ... when Stage 1 ended (after its barrier)
  unsigned long long t_end;       // ... when its finalisation ended
  unsigned long long t_count;     // ... when Stage 2's statistics were known (grid levels)
  unsigned long long t_engine[3]; // probe mode: ticks of each engine
  int engine;
  int fallback;
  int panel;                      // BVSS step ran on the panel-blocked copy
  float feat[kMaxSwitchFeatures];
};

struct MlpDev {
  float params[BLEST_MLP_NPARAMS];
  float mean[BLEST_MLP_IN];
  float inv_std[BLEST_MLP_IN];
  float max_ratio;  // network used only if sum_k exp(z_k - z_max) <= max_ratio (= 1 / min confidence)
  int valid;
};

// Kernel arguments of one single-source traversal (passed by value).
struct BfsArgs {
  const int32_t* rp;
  const int32_t* col;
  const int32_t* rp_in;     // in-arcs, read by the bottom-up engines (rp/col for an undirected graph)
  const int32_t* col_in;
  const void* degmask_in;   // vertices with an in-arc (degmask for an undirected graph)
  const uint32_t* slice_ptr;
  const void* slices;
  const void* degmask;
  const int32_t* orig_id;
  int64_t n, m, nsets;
  int64_t nvss, nslices;  // totals of the BVSS (switch features)
  int32_t tau;
  // working state
  void* vis;       // sigma-bit visited word per slice set (V_curr)
  void* front;     // sigma-bit frontier words per slice set, three buffers fstride bytes apart: the lazy
                   // scheme uses the first two (by level parity), the eager scheme all three (level mod 3)
  long long fstride;  // bytes from the first frontier buffer to the second
  uint8_t* mark;   // one byte per vertex: lazily marked in Stage 1 (V_next)
  uint4* queue[3]; // VSS descriptors {first slice, count, frontier bits, set}; the eager
                   // scheme rotates all three, the lazy scheme uses the first two
  int32_t* flight[2];             // light frontier vertices
  unsigned long long* fheavy[2];  // heavy frontier edge chunks: (vertex << 32) | first edge offset
  Ctl* ctl;
  long long* part;  // per-workgroup partial Stage 2 counters (grid size x 8)
  LevelRec* log;
  int32_t log_cap;
  const MlpDev* mlp;
  int32_t* levels; // output, input ids
  int32_t src;     // internal id
  int32_t policy;
  float eta;
  uint64_t seed;
  int32_t probe;
  int32_t prefilter;
  int32_t count_work;  // accumulate F_WORK (adjacency entries read per level)
  int32_t single_block;  // run small levels on workgroup 0 alone
  // panel-blocked BVSS copy (sigma = 8, 32-bit slices); npanels = 0 if absent
  const uint32_t* pwords;  // nchunks * 64 slice words
  const uint32_t* pbase;   // first set of each chunk (+ kPanelBasePad entries of padding)
  const uint32_t* pptr;    // npanels + 1 chunk offsets
  int32_t npanels;
  int32_t panel_rb;        // log2 rows per panel
  int32_t panel_mode;      // 1: dense levels only, 2: every BVSS level
  long long panel_slots;   // nchunks * kPanelChunk
  int32_t count_first;     // two-phase Stage 2 after dense steps
  unsigned long long timeout_ticks;
};

// Device-resident graph and working buffers (owned by one blest_graph).
struct DevGraph {
  int device = 0;
  int directed = 0;           // rp/col hold out-arcs; rp_in/col_in the in-arcs
  int sigma = 8, tau = 128, wide = 0;
  int64_t n = 0, m = 0, nsets = 0, nvss = 0, nslices = 0, nheavy_cap = 0;
  int32_t* rp = nullptr;
  int32_t* col = nullptr;
  uint32_t* slice_ptr = nullptr;
  void* slices = nullptr;
  void* degmask = nullptr;
  int32_t* orig_id = nullptr;
  const int32_t* rp_in = nullptr;   // = rp, col, degmask unless directed
  const int32_t* col_in = nullptr;
  const void* degmask_in = nullptr;
  void* vis = nullptr;
  void* front = nullptr;  // three buffers, fstride bytes apart
  size_t fstride = 0;
  uint8_t* mark = nullptr;
  uint4* queue[3] = {nullptr, nullptr, nullptr};
  int32_t* flight[2] = {nullptr, nullptr};
  unsigned long long* fheavy[2] = {nullptr, nullptr};
  Ctl* ctl = nullptr;
  MlpDev* ms_mlp = nullptr;  // switch network of the multi-source kernels
  long long* part = nullptr;
  LevelRec* log = nullptr;
  int log_cap = 0;
  MlpDev* mlp = nullptr;
  int* host_flags = nullptr;  // pinned: done flag readback of the per-stage mode
  int block = 512, grid = 0, num_cu = 0, persistent = 1, prefilter = 1, count_work = 0, single_block = 1;
  uint32_t* pwords = nullptr;
  uint32_t* pbase = nullptr;
  uint32_t* pptr = nullptr;
  int64_t npanels = 0, nchunks = 0;
  int panel_rb = 0, panel_mode = 0;
  int count_first = 1;
  size_t mark_bytes = 0;
  double tick_us = 0.01;      // device clock period in microseconds
  int eager = 0;              // single-source traversals use the eager scheme (Alg. 2)
  int ms_ablation = 0;        // multi-source ablation flags (BLEST_MS_NO_*)
  int ms_mfma = 0;            // multi-source top-down check on MFMA (experiment)
  int grid_eager = 0;         // co-resident grid of the eager kernel
  double u_div = 0.0;         // update divergence of the BVSS
};

// Single-source traversal on the device (bfs.hip). Returns a HIP error;
// device-side errors are left in ctl->error.
hipError_t bfs_run(const DevGraph& g, BfsArgs a, hipStream_t st);
// Largest co-resident grid of the persistent kernel for this graph.
hipError_t bfs_grid_size(const DevGraph& g, int policy_learned, int blocks_per_cu, int* grid);
// Same for the eager-scheme kernel.
hipError_t bfs_grid_size_eager(const DevGraph& g, int blocks_per_cu, int* grid);
BfsArgs bfs_args(const DevGraph& g);

// Switch-network kernels (mlp.hip).
hipError_t mlp_forward_launch(const float* params, const float* x, int32_t batch, float* logits, hipStream_t st);
hipError_t mlp_loss_grad_launch(const float* params, const float* x, const int32_t* y, const float* w, int32_t batch,
                                float* loss, float* grad, hipStream_t st);
hipError_t mlp_adam_launch(float* params, const float* grad, float* m, float* v, int32_t n, int32_t t, float lr,
                           float beta1, float beta2, float eps, hipStream_t st);
hipError_t mlp_train_launch(float* params, float* m, float* v, const float* x, const int32_t* y, const float* w,
                            int32_t nsamples, int32_t batch, int32_t steps, float lr, uint64_t seed, float* loss_log,
                            float* grad, hipStream_t st);

}  // namespace blest
