// Multi-source BFS and closeness (msbfs.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "blest_internal.h"

namespace blest {

// Device buffers of the multi-source traversal, sized for the widest batch
// (kappa = 64 * wmax bits per vertex) on first use.
struct MsDev {
  int device = 0;
  int wmax = 0;
  int64_t nhat = 0;
  int64_t nsets = 0;
  unsigned long long* F = nullptr;   // frontier words, getVI-ordered, W per vertex
  unsigned long long* V = nullptr;   // visited words
  unsigned long long* N = nullptr;   // next words: visited bits plus this level's marks (atomic OR targets)
  unsigned long long* act = nullptr; // per slice set: sources active in it
  // int16 level output: a batch's levels are first written by internal id
  // (lstage[i * 64 W + c], the row of vertex i) and copied to the caller's
  // source-major rows once the batch is done; perm: input id -> internal id
  int16_t* lstage = nullptr;
  int64_t lstage_elems = 0;
  int32_t* perm = nullptr;
  uint8_t* dirty = nullptr;          // per slice set: marked in Stage 1
  uint4* queue[2] = {nullptr, nullptr};
  int32_t* srcs = nullptr;           // internal ids of all sources of a call
  int64_t srcs_cap = 0;
  long long* part = nullptr;         // per-block partial sums and reach
  int part_blocks = 0;
  void* batches = nullptr;           // batch descriptors
  int batches_cap = 0;
  int grid = 0, block = 512;
  MsLevelRec* log = nullptr;       // per-level records of the last call
  int log_cap = 0;
  hipStream_t gstream = nullptr;  // graph mode: capture/replay stream (non-blocking)
  hipEvent_t gev[2] = {nullptr, nullptr};
  // graph mode: the graph of phase kernels, built and instantiated once per
  // kernel variant, grid and LDS size; a call rewrites its kernel nodes'
  // arguments
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraphNode_t gnode[32] = {};
  const void* gfn = nullptr;
  int ggrid = 0;
  unsigned gshmem = 0;
  long long gcaptures = 0;  // graphs built so far
};

// Runs all k sources in one persistent launch, in consecutive batches whose
// widths (sources per batch: 64, 128, 256 or 512) are widths[0..nwidths-1],
// the last width repeating. levels16 (k*n, source-major, input ids) and/or
// sums/reach/cc may be NULL. Device-side errors (overflow, timeout) are left
// in g.ctl->error. Returns after the launch is enqueued.
// probe != 0: every level runs both engines from the same state and times
// each (persistent launch). Level records go to ms->log (ms_nrec in ctl).
// far (n entries, input ids, zeroed by the caller): per-target distance sums
// of Eq. 4, added to. graph != 0: the same work as a hipGraph of per-phase kernels (batch set-up,
// seeding, each level's engine and Stage 2, batch reduction) replayed until a
// device-side state machine reports the last batch done; the call then
// returns with the work finished.
hipError_t ms_run(const DevGraph& g, MsDev* ms, const int32_t* srcs_internal, int32_t k, const int32_t* widths,
                  int nwidths, int policy, float eta, uint64_t seed, int16_t* levels16, int64_t* sums,
                  int64_t* reach, double* cc, hipStream_t st, int graph = 0, int64_t* far = nullptr,
                  int probe = 0);
// True when every buffer a persistent multi-source launch of width 64 * W
// needs is already allocated for this graph.
bool ms_ready(const DevGraph& g, const MsDev* ms, int W);
// blest_msbfs without device allocation: the source list (mapped to internal
// ids through perm, a host array, when not NULL) and the batch plan of
// uniform `width` go to a static device array; always the persistent launch.
// hipErrorNotReady: the graph's multi-source buffers are not allocated yet;
// hipErrorInvalidValue: k above BLEST_MSBFS_NOALLOC_MAX_SOURCES or a bad width.
hipError_t ms_run_noalloc(const DevGraph& g, MsDev* ms, const int32_t* srcs, const int32_t* perm, int32_t k,
                          int width, int policy, float eta, uint64_t seed, int16_t* levels16, hipStream_t st);
void ms_release(MsDev* ms);   // frees the per-vertex arrays
void ms_free_all(MsDev* ms);  // frees everything
void ms_reset(MsDev* ms);     // clears marks after a device-side error

}  // namespace blest
