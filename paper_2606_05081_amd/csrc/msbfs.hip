// Multi-source BFS (Section "Multi-Source BFS", Alg. 5) and closeness
// centrality (Section "Closeness Centrality", Eq. 4 and Eq. 5) for gfx950.
//
// kappa = 64 * W concurrent traversals share one pass over the BVSS. Every
// vertex u owns W 64-bit words in each of F (frontier), V (visited) and N
// (marked during Stage 1), stored at getVI(u) = (u mod sigma) * rho +
// floor(u / sigma), rho = number of slice sets, so that consecutive slice
// sets touch consecutive words (the paper's coalescing remap).
//
// Stage 1, top-down over BVSS (E0): a wave takes one queued virtual slice set
// of set s, stages the sigma * W frontier words of s's vertices in LDS, and
// for each slice (row, mask) forms M = OR of the staged words selected by the
// mask bits -- bit c of M is set iff the row has a neighbour in the frontier
// of traversal c, which is what the paper's per-source ballot + binary MMA
// loop computes. Words whose sources are inactive in s (activeSets) are
// skipped; bits already visited are dropped; the rest is OR-ed into N with
// one no-return 64-bit atomic per word, and the row's set is marked dirty.
// Stage 1, bottom-up (E2): a lane owns a vertex with unvisited traversals and
// ORs its neighbours' frontier words until every unvisited bit is covered;
// it alone writes N[u], so no atomics. Only live traversals count (those
// whose frontier is non-empty, from Stage 2's OR of all new words): a
// traversal with an empty frontier can reach nothing more, and waiting for
// its bit (a source in a small component, or one that has finished) would
// turn every early exit into a full adjacency scan.
// Stage 2 visits dirty slice sets only: new = N & ~V, V |= new, F = new,
// activeSets[s] = OR of the set's new words, the set's VSSs are enqueued when
// nonzero, int16 levels are written, and per-source counts of newly reached
// vertices feed the closeness sums.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "device_common.h"
#include "mlp_infer.h"
#include "msbfs.h"

namespace blest {

namespace {

constexpr int kWMax = 8;  // up to 512 sources per batch

// LDS words per wave for the top-down engine: the frontier words of one slice
// set (sigma * W), and for sigma = 8 also two 16-entry nibble tables per word
// (32 * W).
template <int SIGMA>
constexpr int ms_lds_words() {
  return (SIGMA == 8 ? SIGMA + 32 : SIGMA) * kWMax;
}

struct MsBatch {
  int32_t offset;  // first source index of the batch in the call's source list
  int32_t count;   // sources in the batch (<= 64 * W)
  int32_t W;       // 64-bit words per vertex
  int32_t pad;
};

struct MsArgs {
  const int32_t* rp;
  const int32_t* col;
  const int32_t* rp_in;   // in-arcs (the bottom-up engine); rp/col for an undirected graph
  const int32_t* col_in;
  const uint32_t* slice_ptr;
  const void* slices;
  const int32_t* orig_id;
  int64_t n, m, nsets;
  int32_t tau;
  unsigned long long* F;
  unsigned long long* V;
  unsigned long long* N;
  unsigned long long* act;
  uint8_t* dirty;
  uint4* queue[2];
  const int32_t* srcs;
  const MsBatch* batches;
  int32_t nbatches;
  int16_t* levels16;  // k * n or NULL
  int16_t* lstage;    // the batch's levels by internal id (n * 64 W), or NULL: Stage 2 writes levels16 directly
  const int32_t* perm;  // input id -> internal id, or NULL when not relabelled
  int64_t* sums;      // k or NULL
  int64_t* reach;     // k or NULL
  double* cc;         // k or NULL
  int64_t* far;       // n (input ids) or NULL: per-target sums of Eq. 4, accumulated
  long long* part;    // per block: kappa sums then kappa reach counts
  Ctl* ctl;
  int32_t policy;
  float eta;
  uint64_t seed;
  int64_t nvss, nslices;  // BVSS totals (switch features)
  const MlpDev* mlp;      // multi-source switch network (policy LEARNED), or NULL
  int32_t probe;          // 1: every level runs both engines from the same state and times each
  MsLevelRec* log;        // one record per level of the call, or NULL
  int32_t log_cap;
  unsigned long long timeout_ticks;
  int32_t ablation;       // BLEST_MS_NO_GETVI | BLEST_MS_NO_DIRTY (the paper's ablation steps), else 0
};

__device__ __forceinline__ long long get_vi(long long u, long long rho, int sigma) {
  return (u % sigma) * rho + u / sigma;
}

// Ablation flags: ABL >= 0 is a compile-time value (the full method's kernel
// uses 0, so the flags cost it nothing); ABL = -1 reads them from the arguments.
template <int ABL>
__device__ __forceinline__ int ms_abl(const MsArgs& a) {
  if constexpr (ABL >= 0)
    return ABL;
  else
    return a.ablation;
}

// Word index of vertex u: getVI order, or u itself in the ablation without it.
template <int ABL>
__device__ __forceinline__ long long ms_vi(const MsArgs& a, long long u, long long rho, int sigma) {
  return (ms_abl<ABL>(a) & BLEST_MS_NO_GETVI) ? u : get_vi(u, rho, sigma);
}

__device__ __forceinline__ unsigned long long batch_mask(int count, int w) {
  const int lo = w * 64;
  if (count >= lo + 64) return ~0ULL;
  if (count <= lo) return 0ULL;
  return (1ULL << (count - lo)) - 1ULL;
}

__device__ __forceinline__ unsigned long long mix64_ms(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Sets count int16 values to -1: elementwise up to 16-byte alignment, then
// 16-byte stores, then the tail.
// Switch inputs of a multi-source level, counted in (vertex, traversal) pairs
// (base-2 logarithms): new pairs and queued slices (absolute), then shares:
// new pairs / all pairs, VSSs / N_v, queued slices / all slices, unvisited
// pairs / all pairs, the batch width, the ratio of the pairs rule
// (log |Q| - log unvisited pairs), live traversals / batch width; three
// reserved zeros.
__device__ __forceinline__ void ms_features(float (&f)[kMaxSwitchFeatures], const MsArgs& a, long long fresh,
                                            long long qlen, long long qslices, long long unv, int count,
                                            int live) {
  const float pairs = log2f(static_cast<float>(count) * static_cast<float>(a.n));
  const float lu = log2f(1.0f + static_cast<float>(unv));
  f[0] = log2f(1.0f + static_cast<float>(fresh));
  f[1] = log2f(1.0f + static_cast<float>(qslices));
  f[2] = f[0] - pairs;
  f[3] = log2f(1.0f + static_cast<float>(qlen)) - log2f(1.0f + static_cast<float>(a.nvss));
  f[4] = f[1] - log2f(1.0f + static_cast<float>(a.nslices));
  f[5] = lu - pairs;
  f[6] = log2f(static_cast<float>(count));
  f[7] = log2f(1.0f + static_cast<float>(qlen)) - lu;
  f[8] = log2f(static_cast<float>(max(live, 1))) - f[6];
#pragma unroll
  for (int k = 9; k < kMaxSwitchFeatures; ++k) f[k] = 0.0f;
}

// Live traversals of a stat slot (Stage 2 ORs the new words into F_LIVE;
// words beyond the batch width stay zero). One 64-byte read, no dependent loads.
__device__ __forceinline__ int ms_live_count(const Ctl* ctl, int slot) {
  const unsigned long long* p = &ctl->acc[slot][F_LIVE][0];
  int c = 0;
#pragma unroll
  for (int w = 0; w < kWMax; ++w) c += __popcll(p[w]);
  return c;
}

// Block 0 clears one stat slot: element 0 of every field and the F_LIVE words.
__device__ __forceinline__ void ms_clear_slot(Ctl* ctl, int slot) {
  for (int t = threadIdx.x; t < kStatFields + kWMax; t += blockDim.x) {
    if (t < kStatFields)
      ctl->acc[slot][t][0] = 0ULL;
    else
      ctl->acc[slot][F_LIVE][t - kStatFields] = 0ULL;
  }
}

// Engine of a multi-source level (uniform across the grid: every input is).
// Eq. 3 counted in (vertex, traversal) pairs: the bottom-up engine reads W
// frontier words per scanned edge and rarely stops early while many
// traversals are open, so it is chosen only once fewer than eta * |Q| pairs
// remain unvisited. LEARNED: the switch network (output 0 = BVSS, 2 =
// bottom-up; anything else, or low confidence, falls back to the pairs rule).
// Contains __syncthreads() when s_mlp is set.
__device__ int ms_choose(const MsArgs& a, const float (&feat)[kMaxSwitchFeatures], long long qlen, long long unv,
                         int level, int bi, const float* s_mlp, int* fallback) {
  __shared__ int s_choice;
  *fallback = 0;
  const int rule = (static_cast<double>(unv) < static_cast<double>(a.eta) * static_cast<double>(qlen))
                       ? BLEST_ENGINE_BOTTOM_UP
                       : BLEST_ENGINE_BVSS;
  switch (a.policy) {
    case BLEST_POLICY_BVSS:
    case BLEST_POLICY_PUSH:
      return BLEST_ENGINE_BVSS;
    case BLEST_POLICY_BOTTOM_UP:
      return BLEST_ENGINE_BOTTOM_UP;
    case BLEST_POLICY_RANDOM:
      return (mix64_ms(a.seed + 0x9E3779B97F4A7C15ULL * static_cast<unsigned long long>(level + 1 + 977 * bi)) & 1ULL)
                 ? BLEST_ENGINE_BOTTOM_UP
                 : BLEST_ENGINE_BVSS;
    case BLEST_POLICY_LEARNED:
      if (s_mlp != nullptr) {
        if (threadIdx.x < 64) {
          const int c = mlp_choose_wave(s_mlp, feat);
          if (threadIdx.x == 0) s_choice = c;
        }
        __syncthreads();
        const int c = s_choice;
        __syncthreads();
        if (c == BLEST_ENGINE_BVSS || c == BLEST_ENGINE_BOTTOM_UP) return c;
      }
      *fallback = 1;
      return rule;
    default:
      return rule;
  }
}

__device__ void fill_minus_one(int16_t* p, long long count, long long gtid, long long nthreads) {
  const long long mis = (16 - (reinterpret_cast<uintptr_t>(p) & 15)) & 15;
  const long long head = min(count, mis / 2);
  for (long long i = gtid; i < head; i += nthreads) p[i] = -1;
  const long long nvec = (count - head) / 8;
  ulonglong2* v = reinterpret_cast<ulonglong2*>(p + head);
  for (long long i = gtid; i < nvec; i += nthreads) v[i] = make_ulonglong2(~0ULL, ~0ULL);
  for (long long i = head + nvec * 8 + gtid; i < count; i += nthreads) p[i] = -1;
}

// ---------------------------------------------------------------- Stage 1

template <int SIGMA, class SliceT, int K, int ABL>
__device__ void ms_engine_bvss_k(const MsArgs& a, const uint4* __restrict__ q, long long qlen, int W,
                                 long long gwave, long long nwaves, unsigned long long* lds_f) {
  const SliceT* __restrict__ sl = static_cast<const SliceT*>(a.slices);
  const long long rho = a.nsets;
  const int lane = lane_id();
  for (long long i = gwave; i < qlen; i += nwaves) {
    const uint4 d = q[i];
    const uint32_t start = d.x, cnt = d.y;
    const long long s = d.w;
    // Stage the frontier words of the set's sigma vertices (vertex s*SIGMA+b
    // sits at b*rho + s in getVI order).
    for (int j = lane; j < SIGMA * W; j += 64) {
      const int b = j / W, w = j % W;
      lds_f[j] = a.F[ms_vi<ABL>(a, s * SIGMA + b, rho, SIGMA) * W + w];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    SliceT sv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t j = static_cast<uint32_t>(lane) + 64u * k;
      sv[k] = (j < cnt) ? sl[start + j] : SliceT(0);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t mask = static_cast<uint32_t>(sv[k] & ((SliceT(1) << SIGMA) - 1));
      if (!mask) continue;
      const long long row = static_cast<long long>(sv[k] >> SliceFmt<SliceT>::kRowShift);
      const long long vi = ms_vi<ABL>(a, row, rho, SIGMA);
      bool any = false;
      for (int w = 0; w < W; ++w) {
        if (!a.act[s * W + w]) continue;
        unsigned long long mw = 0;
        uint32_t t = mask;
        while (t) {
          const int b = __builtin_ctz(t);
          t &= t - 1;
          mw |= lds_f[b * W + w];
        }
        if (!mw) continue;
        mw &= ~a.V[vi * W + w];
        if (mw) {
          __hip_atomic_fetch_or(&a.N[vi * W + w], mw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          any = true;
        }
      }
      if (any) a.dirty[row / SIGMA] = 1;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

__device__ __forceinline__ unsigned long long readlane64(unsigned long long x, int l) {
  const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(x), l);
  const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(x >> 32), l);
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}

// The sigma = 8 form of the engine above, shaped for memory latency. Per VSS
// the slices, the set's frontier words and its activity words are loaded
// together. The frontier words are staged in LDS and expanded into two
// 16-entry tables per word w: lo[i] = OR of the words of the vertices in bit
// subset i of bits 0..3, hi[i] the same for bits 4..7, so a slice's
// neighbour word for w is lo[mask & 15] | hi[mask >> 4] (two LDS reads, where
// the bit loop took up to eight dependent ones). Then, two words at a time
// (one 16-byte load per vertex), the next words of all the lane's K slices
// are loaded at once before any is used, and an atomic OR is issued only for
// bits not yet in them. As in Alg. 5's V_next, a next word holds the visited
// bits plus this level's marks, so this one load filters both; it only grows
// during Stage 1, so a bit seen set needs no OR, and a stale read only costs
// an OR that changes nothing. On this GPU the device-scope ORs, performed at
// the memory side, are what bounds the step. LDS layout per wave: F at [b * W + w], tables at
// [8 W + (h * 16 + i) * W + w].
// (Not inlined: it gets its own register allocation instead of adding to the
// persistent kernel's; its pointers are converted to the global address space.)
template <class SliceT, int K, int ABL>
__device__ __attribute__((noinline)) void ms_engine_bvss8(const MsArgs& a, const uint4* q_in, long long qlen, int W,
                                                          long long gwave, long long nwaves,
                                                          unsigned long long* lds_in) {
  constexpr int SIGMA = 8;
  const gptr<const SliceT> sl = to_global(static_cast<const SliceT*>(a.slices));
  const gptr<const uint4> q = to_global(q_in);
  const gptr<const unsigned long long> F = to_global(static_cast<const unsigned long long*>(a.F));
  const gptr<const unsigned long long> act = to_global(static_cast<const unsigned long long*>(a.act));
  const gptr<unsigned long long> N = to_global(a.N);
  const gptr<uint8_t> dirty = to_global(a.dirty);
  const lptr<unsigned long long> lds = to_lds(lds_in);
  const long long rho = a.nsets;
  const int lane = lane_id();
  const lptr<unsigned long long> tab = lds + SIGMA * W;
  for (long long i = gwave; i < qlen; i += nwaves) {
    const uint4 d = q[i];
    const uint32_t start = d.x, cnt = d.y;
    const long long s = d.w;
    SliceT sv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t j = static_cast<uint32_t>(lane) + 64u * k;
      sv[k] = (j < cnt) ? sl[start + j] : SliceT(0);
    }
    unsigned long long fw = 0ULL, aw = 0ULL;
    if (lane < SIGMA * W) fw = F[ms_vi<ABL>(a, s * SIGMA + lane / W, rho, SIGMA) * W + lane % W];
    if (lane < W) aw = act[s * W + lane];
    if (lane < SIGMA * W) lds[lane] = fw;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int e = lane; e < 32 * W; e += 64) {
      const int w = e % W, t = e / W;
      const int h = t >> 4, sub = t & 15;
      unsigned long long x = 0ULL;
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if ((sub >> b) & 1) x |= lds[(4 * h + b) * W + w];
      tab[e] = x;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    long long vi[K];
    uint32_t m8[K];
    bool any[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      m8[k] = static_cast<uint32_t>(sv[k] & SliceT(0xff));
      vi[k] = ms_vi<ABL>(a, static_cast<long long>(sv[k] >> SliceFmt<SliceT>::kRowShift), rho, SIGMA);
      any[k] = false;
    }
    if (W == 1) {
      if (readlane64(aw, 0)) {
        unsigned long long mw[K], v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) mw[k] = m8[k] ? (tab[m8[k] & 15u] | tab[16u + (m8[k] >> 4)]) : 0ULL;
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = mw[k] ? N[vi[k]] : ~0ULL;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const unsigned long long m = mw[k] & ~v[k];
          if (m) {
            __hip_atomic_fetch_or(&N[vi[k]], m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            any[k] = true;
          }
        }
      }
    } else {
      // W is even: words w and w + 1 of a vertex are one aligned 16-byte
      // load (N is 16-byte aligned and vi * W + w is even)
      for (int w = 0; w < W; w += 2) {
        if (!(readlane64(aw, w) | readlane64(aw, w + 1))) continue;
        unsigned long long m0[K], m1[K];
        u64x2 v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          m0[k] = m8[k] ? (tab[(m8[k] & 15u) * W + w] | tab[(16u + (m8[k] >> 4)) * W + w]) : 0ULL;
          m1[k] = m8[k] ? (tab[(m8[k] & 15u) * W + w + 1] | tab[(16u + (m8[k] >> 4)) * W + w + 1]) : 0ULL;
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
          v[k] = (m0[k] | m1[k]) ? *(gptr<const u64x2>)(N + vi[k] * W + w) : u64x2{~0ULL, ~0ULL};
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const unsigned long long x0 = m0[k] & ~v[k].x, x1 = m1[k] & ~v[k].y;
          if (x0) __hip_atomic_fetch_or(&N[vi[k] * W + w], x0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (x1) __hip_atomic_fetch_or(&N[vi[k] * W + w + 1], x1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          any[k] = any[k] || (x0 | x1) != 0ULL;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (any[k]) dirty[(sv[k] >> SliceFmt<SliceT>::kRowShift) / SIGMA] = 1;
    __builtin_amdgcn_wave_barrier();
  }
}

// The same neighbour check as an int8 matrix product on the matrix cores (an
// experiment kept behind opts.ms_mfma; sigma = 8 only). For 16 slices of a VSS
// and 16 traversals c, C = A B with A[i][b] = bit b of slice i's mask and
// B[b][c] = bit c of vertex b's frontier word: C[i][c] > 0 iff row i has a
// neighbour in traversal c's frontier, the count Eq. 2 tests (popc(a & x) > 0).
// One v_mfma_i32_16x16x32_i8 per (16 slices, 16 traversals): K = 32 holds the
// 8 mask bits and 24 zeros; lane l supplies A[l % 16][8 (l / 16) .. + 7] and
// B[8 (l / 16) .. + 7][l % 16], so only lanes 0..15 carry nonzero operands,
// and receives C[4 (l / 16) + r][l % 16] in its r-th result.
typedef int ms_v4i __attribute__((ext_vector_type(4)));

template <class SliceT, int ABL>
__device__ void ms_engine_mfma(const MsArgs& a, const uint4* __restrict__ q, long long qlen, int W, long long gwave,
                               long long nwaves, unsigned long long* lds_f) {
  constexpr int SIGMA = 8;
  const SliceT* __restrict__ sl = static_cast<const SliceT*>(a.slices);
  const long long rho = a.nsets;
  const int lane = lane_id();
  const int c16 = lane & 15;
  const bool carrier = lane < 16;
  for (long long i = gwave; i < qlen; i += nwaves) {
    const uint4 d = q[i];
    const uint32_t start = d.x, cnt = d.y;
    const long long s = d.w;
    for (int j = lane; j < SIGMA * W; j += 64) {
      const int b = j / W, w = j % W;
      lds_f[j] = a.F[ms_vi<ABL>(a, s * SIGMA + b, rho, SIGMA) * W + w];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t t0 = 0; t0 < cnt; t0 += 16) {
      SliceT sw = 0;
      if (carrier && t0 + c16 < cnt) sw = sl[start + t0 + c16];
      const uint32_t mask = static_cast<uint32_t>(sw & SliceT(0xff));
      long afrag = 0;
#pragma unroll
      for (int b = 0; b < 8; ++b) afrag |= static_cast<long>((mask >> b) & 1u) << (8 * b);
      unsigned long long hw[kWMax];
#pragma unroll
      for (int w = 0; w < kWMax; ++w) hw[w] = 0ULL;
      for (int w = 0; w < W; ++w) {
        if (!a.act[s * W + w]) continue;
#pragma unroll
        for (int j4 = 0; j4 < 4; ++j4) {
          long bfrag = 0;
          if (carrier) {
#pragma unroll
            for (int b = 0; b < 8; ++b)
              bfrag |= static_cast<long>((lds_f[b * W + w] >> (16 * j4 + c16)) & 1ULL) << (8 * b);
          }
          ms_v4i c = {0, 0, 0, 0};
          c = __builtin_amdgcn_mfma_i32_16x16x32_i8(afrag, bfrag, c, 0, 0, 0);
          // row i = 4 q + r of the tile holds its 16 bits at [16 q, 16 q + 16) of ballot r
          unsigned long long bal[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) bal[r] = __ballot(c[r] > 0);
          const int rq = c16 >> 2, rr = c16 & 3;
          const unsigned long long br = rr == 0 ? bal[0] : rr == 1 ? bal[1] : rr == 2 ? bal[2] : bal[3];
          hw[w] |= ((br >> (16 * rq)) & 0xffffULL) << (16 * j4);
        }
      }
      if (carrier && mask) {
        const long long row = static_cast<long long>(sw >> SliceFmt<SliceT>::kRowShift);
        const long long vi = ms_vi<ABL>(a, row, rho, SIGMA);
        bool any = false;
        for (int w = 0; w < W; ++w) {
          unsigned long long mw = hw[w];
          if (!mw) continue;
          mw &= ~a.V[vi * W + w];
          if (mw) {
            __hip_atomic_fetch_or(&a.N[vi * W + w], mw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            any = true;
          }
        }
        if (any) a.dirty[row / SIGMA] = 1;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

template <int SIGMA, class SliceT, bool MF, int ABL>
__device__ void ms_engine_bvss(const MsArgs& a, const uint4* q, long long qlen, int W, long long gwave,
                               long long nwaves, unsigned long long* lds_f) {
  if constexpr (MF && SIGMA == 8) {
    ms_engine_mfma<SliceT, ABL>(a, q, qlen, W, gwave, nwaves, lds_f);
    return;
  }
  if constexpr (SIGMA == 8) {
    switch (a.tau) {
      case 64:
        ms_engine_bvss8<SliceT, 1, ABL>(a, q, qlen, W, gwave, nwaves, lds_f);
        break;
      case 128:
        ms_engine_bvss8<SliceT, 2, ABL>(a, q, qlen, W, gwave, nwaves, lds_f);
        break;
      case 192:
        ms_engine_bvss8<SliceT, 3, ABL>(a, q, qlen, W, gwave, nwaves, lds_f);
        break;
      default:
        ms_engine_bvss8<SliceT, 4, ABL>(a, q, qlen, W, gwave, nwaves, lds_f);
        break;
    }
    return;
  }
  switch (a.tau) {
    case 64:
      ms_engine_bvss_k<SIGMA, SliceT, 1, ABL>(a, q, qlen, W, gwave, nwaves, lds_f);
      break;
    case 128:
      ms_engine_bvss_k<SIGMA, SliceT, 2, ABL>(a, q, qlen, W, gwave, nwaves, lds_f);
      break;
    case 192:
      ms_engine_bvss_k<SIGMA, SliceT, 3, ABL>(a, q, qlen, W, gwave, nwaves, lds_f);
      break;
    default:
      ms_engine_bvss_k<SIGMA, SliceT, 4, ABL>(a, q, qlen, W, gwave, nwaves, lds_f);
      break;
  }
}

template <int SIGMA, int ABL>
__device__ void ms_engine_pull(const MsArgs& a, int W, int count, const unsigned long long* live, long long gtid,
                               long long nthreads) {
  const long long rho = a.nsets;
  unsigned long long bm[kWMax];
#pragma unroll
  for (int w = 0; w < kWMax; ++w) bm[w] = (w < W) ? (batch_mask(count, w) & live[w]) : 0ULL;
  for (long long u = gtid; u < a.n; u += nthreads) {
    const int p0 = a.rp_in[u], p1 = a.rp_in[u + 1];
    if (p0 == p1) continue;
    const long long vi = ms_vi<ABL>(a, u, rho, SIGMA);
    unsigned long long vis[kWMax], unv[kWMax], acc[kWMax];
    bool open = false;
#pragma unroll
    for (int w = 0; w < kWMax; ++w) {
      vis[w] = (w < W) ? a.V[vi * W + w] : ~0ULL;
      unv[w] = ~vis[w] & bm[w];
      acc[w] = 0ULL;
      open |= unv[w] != 0ULL;
    }
    if (!open) continue;
    // Four in-neighbours at a time: their column indices and frontier words
    // are loaded before any is tested (the test may end the scan, so one at a
    // time every load waited for the previous one); up to three loads past
    // the covering neighbour are wasted.
    for (int p = p0; p < p1; p += 4) {
      long long iv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) iv[j] = p + j < p1 ? ms_vi<ABL>(a, a.col_in[p + j], rho, SIGMA) : -1;
      bool covered = true;
#pragma unroll
      for (int w = 0; w < kWMax; ++w) {
        if (w < W && unv[w]) {
          unsigned long long f[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) f[j] = iv[j] >= 0 ? a.F[iv[j] * W + w] : 0ULL;
          acc[w] |= f[0] | f[1] | f[2] | f[3];
          covered &= (acc[w] & unv[w]) == unv[w];
        }
      }
      if (covered) break;
    }
    bool any = false;
#pragma unroll
    for (int w = 0; w < kWMax; ++w) {
      const unsigned long long x = acc[w] & unv[w];
      if (w < W && x) {
        a.N[vi * W + w] = vis[w] | x;  // N = visited words plus this level's marks
        any = true;
      }
    }
    if (any) a.dirty[u / SIGMA] = 1;
  }
}

// ---------------------------------------------------------------- Stage 2

struct MsExpandRec {
  unsigned long long out;
  uint32_t n, s0, ns, s;
};
// Copies a finished batch's staged levels to the caller's rows:
// levels16[(offset + c) * n + v] = level of input vertex v in traversal c, -1
// if the traversal did not reach it. Thread t handles input ids v = t, t +
// nthreads, ...: for each traversal the wave's 64 stores are consecutive, and
// each lane reads its vertex's staging row 16 bytes at a time. Visited bits
// come from V (getVI order), so unreached pairs need no staged value.
template <int SIGMA, int ABL>
__device__ __attribute__((noinline)) void ms_copy_levels(const MsArgs& a, const MsBatch& bt, long long gtid,
                                                         long long nthreads) {
  const int W = bt.W;
  const long long K = 64LL * W;
  const long long n = a.n;
  const long long rho = a.nsets;
  const int count = bt.count;
  int16_t* out = a.levels16 + static_cast<long long>(bt.offset) * n;
  for (long long v = gtid; v < n; v += nthreads) {
    const long long i = a.perm ? a.perm[v] : v;
    const long long vi = ms_vi<ABL>(a, i, rho, SIGMA);
    const uint4* row = reinterpret_cast<const uint4*>(a.lstage + i * K);
    for (int w = 0; w < W && 64 * w < count; ++w) {
      const unsigned long long vis = a.V[vi * W + w];
      for (int j = 0; j < 8 && 64 * w + 8 * j < count; ++j) {
        const uint32_t bits = static_cast<uint32_t>(vis >> (8 * j)) & 0xffu;
        uint4 q = make_uint4(0u, 0u, 0u, 0u);
        if (bits) q = row[8 * w + j];
        const uint32_t h[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int c = 64 * w + 8 * j + e;
          if (c >= count) break;
          const int16_t lv = static_cast<int16_t>((h[e / 2] >> (16 * (e % 2))) & 0xffffu);
          out[static_cast<long long>(c) * n + v] = ((bits >> e) & 1u) ? lv : static_cast<int16_t>(-1);
        }
      }
    }
  }
}

constexpr int kMsExpandMin = 8;
constexpr int kMsMaxExpand = 128;

template <int SIGMA, int BLOCK, int ABL>
__device__ void ms_finalize(const MsArgs& a, const MsBatch& bt, int new_level, int slot_out, int sel_out,
                            long long cum_in, int* lds_cnt, bool count_sources) {
  __shared__ int lds32[BLOCK / 64];
  __shared__ long long lds64[3 * (BLOCK / 64)];
  __shared__ unsigned long long qbase;
  __shared__ MsExpandRec rec[kMsMaxExpand];
  __shared__ int nrec;
  __shared__ unsigned long long lds_live[kWMax];  // OR of this block's new words
  if (threadIdx.x == 0) nrec = 0;
  if (threadIdx.x < kWMax) lds_live[threadIdx.x] = 0ULL;
  const int W = bt.W;
  const long long rho = a.nsets;
  const uint32_t tau = static_cast<uint32_t>(a.tau);
  unsigned long long* acc = &a.ctl->acc[slot_out][0][0];
  uint4* __restrict__ queue = a.queue[sel_out];
  const int lane = lane_id();
  long long st[3] = {0, 0, 0};  // new pairs, queued slices, (unused)
  const bool overflow = a.levels16 != nullptr && new_level > 32767;
  for (long long base = static_cast<long long>(blockIdx.x) * BLOCK; base < a.nsets;
       base += static_cast<long long>(gridDim.x) * BLOCK) {
    const long long s = base + threadIdx.x;
    // Without dynamic slice-set tracking (an ablation step) every set is
    // finalised at every level, all its words count as active and all its
    // VSSs are queued.
    const bool track = !(ms_abl<ABL>(a) & BLEST_MS_NO_DIRTY);
    const bool mine = s < a.nsets && (!track || a.dirty[s]);
    int nq = 0;
    uint32_t s0 = 0, ns = 0;
    if (__syncthreads_or(mine)) {
      if (mine) a.dirty[s] = 0;
      const bool wave_any = __ballot(mine) != 0ULL;
      unsigned long long A_any = 0ULL;
      int far_cnt[SIGMA];  // per vertex of the set: traversals that reached it at this level
#pragma unroll
      for (int b = 0; b < SIGMA; ++b) far_cnt[b] = 0;
      if (wave_any) {
        for (int w = 0; w < W; ++w) {
          unsigned long long dw[SIGMA];
          unsigned long long Aw = 0ULL;
          // N holds the visited words plus this level's marks (Alg. 5's
          // V_next); the new bits are its difference from V. All the set's
          // N and V words for word w are loaded before any store (the stores
          // below would otherwise order each vertex's loads after the
          // previous vertex's stores).
          long long idx[SIGMA];
          unsigned long long nx[SIGMA], old[SIGMA];
#pragma unroll
          for (int b = 0; b < SIGMA; ++b) {
            idx[b] = ms_vi<ABL>(a, s * SIGMA + b, rho, SIGMA) * W + w;
            nx[b] = mine ? a.N[idx[b]] : 0ULL;
            old[b] = mine ? a.V[idx[b]] : 0ULL;
          }
#pragma unroll
          for (int b = 0; b < SIGMA; ++b) {
            dw[b] = 0ULL;
            if (mine) {
              const unsigned long long dd = nx[b] & ~old[b];
              if (dd) a.V[idx[b]] = nx[b];
              a.F[idx[b]] = dd;
              dw[b] = dd;
              Aw |= dd;
              far_cnt[b] += __popcll(dd);
            }
          }
          if (mine) a.act[s * W + w] = track ? Aw : ~0ULL;
          A_any |= Aw;
          if (Aw & ~lds_live[w])
            __hip_atomic_fetch_or(&lds_live[w], Aw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          // int16 levels. Staged: each new (vertex, traversal) pair goes to
          // the vertex's staging row. The wave writes them together: for each
          // of its lanes' sets with new bits (lane l holds set s - lane + l),
          // lane c stores traversal 64 w + c of each of the set's vertices,
          // so one store covers 128 contiguous bytes of a row. Direct (no
          // staging buffer): for each traversal c with new vertices in this
          // set, the set's vertices in c's output row (scattered when
          // relabelled).
          if (a.lstage && !overflow) {
            const long long K = 64LL * W;
            unsigned long long todo = __ballot(Aw != 0ULL);
            while (todo) {
              const int l = __builtin_ctzll(todo);
              todo &= todo - 1;
              int16_t* rows = a.lstage + (s - lane + l) * SIGMA * K + 64 * w + lane;
#pragma unroll
              for (int b = 0; b < SIGMA; ++b) {
                const unsigned long long d = readlane64(dw[b], l);
                if ((d >> lane) & 1ULL) rows[b * K] = static_cast<int16_t>(new_level);
              }
            }
          } else if (a.levels16 && Aw && !overflow) {
            unsigned long long t = Aw;
            while (t) {
              const int c = __builtin_ctzll(t);
              t &= t - 1;
              const long long row = static_cast<long long>(bt.offset) + w * 64 + c;
              int16_t* out = a.levels16 + row * a.n;
#pragma unroll
              for (int b = 0; b < SIGMA; ++b)
                if ((dw[b] >> c) & 1ULL) {
                  const long long u = s * SIGMA + b;
                  out[a.orig_id ? a.orig_id[u] : u] = static_cast<int16_t>(new_level);
                }
            }
          }
          if (Aw && overflow) __hip_atomic_store(&a.ctl->error[0], static_cast<int>(BLEST_ERR_OVERFLOW),
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          // Per-source counts of new vertices: lane c accumulates traversal
          // w*64+c by a ballot over the wave's lanes (vertical popcount).
          int cnt_c = 0;  // lane c: new vertices of traversal w*64+c in this wave
#pragma unroll
          for (int b = 0; b < SIGMA; ++b) {
            st[0] += __popcll(dw[b]);
            if (count_sources && __ballot(dw[b] != 0ULL)) {
              for (int c = 0; c < 64; ++c) {
                const int pc = __popcll(__ballot((dw[b] >> c) & 1ULL));
                if (lane == c) cnt_c += pc;
              }
            }
          }
          if (cnt_c) atomicAdd(&lds_cnt[w * 64 + lane], cnt_c);
        }
      }
      if (a.far && mine && A_any && new_level > 0) {
        // Eq. 4: far[u] += level * (traversals reaching u at this level); the
        // thread owns set s, so no other thread updates these vertices
#pragma unroll
        for (int b = 0; b < SIGMA; ++b)
          if (far_cnt[b]) {
            const long long u = s * SIGMA + b;
            a.far[a.orig_id ? a.orig_id[u] : u] += static_cast<int64_t>(new_level) * far_cnt[b];
          }
      }
      if (mine && (A_any || !track)) {
        s0 = a.slice_ptr[s];
        ns = a.slice_ptr[s + 1] - s0;
        nq = static_cast<int>((ns + tau - 1) / tau);
        st[1] += ns;
      }
      // enqueue the VSSs of every set that gained a vertex in some traversal
      int v1[1] = {nq}, ex1[1], tot1[1];
      block_exclusive_scan<BLOCK, 1>(v1, ex1, tot1, lds32);
      if (threadIdx.x == 0) qbase = tot1[0] ? fetch_add_u64(acc + F_QUEUE * kPad, tot1[0]) : 0ULL;
      __syncthreads();
      long long oq = static_cast<long long>(qbase) + ex1[0];
      if (nq > kMsExpandMin) {
        const int r = atomicAdd(&nrec, 1);
        if (r < kMsMaxExpand) {
          rec[r] = MsExpandRec{static_cast<unsigned long long>(oq), static_cast<uint32_t>(nq), s0, ns,
                               static_cast<uint32_t>(s)};
          nq = 0;
        }
      }
      for (int k2 = 0; k2 < nq; ++k2) {
        const uint32_t off = static_cast<uint32_t>(k2) * tau;
        queue[oq + k2] = make_uint4(s0 + off, min(tau, ns - off), 0u, static_cast<uint32_t>(s));
      }
      __syncthreads();
      const int nr = min(nrec, kMsMaxExpand);
      for (int r = 0; r < nr; ++r) {
        const MsExpandRec e = rec[r];
        for (uint32_t i = threadIdx.x; i < e.n; i += BLOCK) {
          const uint32_t off = i * tau;
          queue[e.out + i] = make_uint4(e.s0 + off, min(tau, e.ns - off), 0u, e.s);
        }
      }
      __syncthreads();
      if (threadIdx.x == 0) nrec = 0;
      __syncthreads();
    }
  }
  block_sum64<BLOCK, 3>(st, lds64);
  __syncthreads();
  if (threadIdx.x < W) {
    const unsigned long long v = lds_live[threadIdx.x];
    if (v) __hip_atomic_fetch_or(acc + F_LIVE * kPad + threadIdx.x, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (threadIdx.x == 0) {
    if (st[0]) {
      add_u64(acc + F_FRONTIER * kPad, st[0]);
      add_u64(acc + F_CUMV * kPad, st[0]);
    }
    if (st[1]) add_u64(acc + F_QSLICES * kPad, st[1]);
    if (blockIdx.x == 0 && cum_in) add_u64(acc + F_CUMV * kPad, cum_in);
  }
  if (count_sources) {
    __syncthreads();
    // block-private partial sums across levels: sum += level * count, reach += count
    long long* part = a.part + static_cast<long long>(blockIdx.x) * (2 * 64 * kWMax);
    for (int c = threadIdx.x; c < 64 * W; c += BLOCK) {
      const int x = lds_cnt[c];
      if (x) {
        part[c] += static_cast<long long>(new_level) * x;
        part[64 * kWMax + c] += x;
        lds_cnt[c] = 0;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------- kernel

// MODE 0: the full method with the bitwise check; 1: the check on the matrix
// cores; 10 + f: the bitwise check with ablation flags f (each a kernel of its
// own, so no variant's branches or registers weigh on another).
template <int SIGMA, class SliceT, int BLOCK, int MODE = 0>
__global__ void __launch_bounds__(BLOCK) k_ms_persistent(MsArgs a) {
  constexpr bool MF = MODE == 1;
  constexpr int ABL = MODE >= 10 ? MODE - 10 : 0;
  extern __shared__ float s_mlp[];
  __shared__ unsigned long long lds_f[(BLOCK / 64) * ms_lds_words<SIGMA>()];
  __shared__ int lds_cnt[64 * kWMax];
  const bool learned = a.policy == BLEST_POLICY_LEARNED && a.mlp != nullptr && a.mlp->valid;
  if (learned) mlp_to_lds(a.mlp, s_mlp);
  const long long nthreads = static_cast<long long>(gridDim.x) * BLOCK;
  const long long gtid = static_cast<long long>(blockIdx.x) * BLOCK + threadIdx.x;
  const int wave = wave_in_block();
  const long long gwave = static_cast<long long>(blockIdx.x) * (BLOCK / 64) + wave;
  const long long nwaves = static_cast<long long>(gridDim.x) * (BLOCK / 64);
  unsigned long long* my_f = lds_f + wave * ms_lds_words<SIGMA>();
  const long long rho = a.nsets;
  const long long nhat = a.nsets * SIGMA;
  const bool count_sources = a.sums != nullptr || a.reach != nullptr || a.cc != nullptr;
  for (int c = threadIdx.x; c < 64 * kWMax; c += BLOCK) lds_cnt[c] = 0;
  BarrierCtx bc;
  if (!barrier_register(a.ctl, &bc, a.timeout_ticks)) return;
  int total_levels = 0;
  int nrec = 0;  // level records written so far (the same count in every workgroup)
  for (int bi = 0; bi < a.nbatches; ++bi) {
    const MsBatch bt = a.batches[bi];
    const int W = bt.W;
    // clear the batch's state and its level rows
    for (long long i = gtid; i < nhat * W; i += nthreads) {
      a.F[i] = 0ULL;
      a.V[i] = 0ULL;
      a.N[i] = 0ULL;
    }
    if (a.levels16 && !a.lstage) fill_minus_one(a.levels16 + static_cast<long long>(bt.offset) * a.n,
                                                static_cast<long long>(bt.count) * a.n, gtid, nthreads);
    if (count_sources) {
      long long* part = a.part + static_cast<long long>(blockIdx.x) * (2 * 64 * kWMax);
      for (int c = threadIdx.x; c < 2 * 64 * kWMax; c += BLOCK) part[c] = 0;
    }
    if (blockIdx.x == 0)
      for (int t = 0; t < kStatSlots; ++t) ms_clear_slot(a.ctl, t);
    if (!grid_barrier(a.ctl, bc)) return;
    // seed: mark each source in its own traversal's bit
    for (long long c = gtid; c < bt.count; c += nthreads) {
      const long long u = a.srcs[bt.offset + c];
      const long long vi = ms_vi<ABL>(a, u, rho, SIGMA);
      __hip_atomic_fetch_or(&a.N[vi * W + c / 64], 1ULL << (c % 64), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      a.dirty[u / SIGMA] = 1;
    }
    if (!grid_barrier(a.ctl, bc)) return;
    ms_finalize<SIGMA, BLOCK, ABL>(a, bt, 0, 0, 0, 0, lds_cnt, count_sources);
    if (!grid_barrier(a.ctl, bc)) return;
    const long long pairs_total = static_cast<long long>(bt.count) * a.n;
    for (int level = 0;; ++level) {
      const int slot = level % kStatSlots;
      const unsigned long long* accr = &a.ctl->acc[slot][0][0];
      const long long fresh = static_cast<long long>(accr[F_FRONTIER * kPad]);
      if (fresh == 0) break;
      const long long qlen = static_cast<long long>(accr[F_QUEUE * kPad]);
      const long long qslices = static_cast<long long>(accr[F_QSLICES * kPad]);
      const long long cumv = static_cast<long long>(accr[F_CUMV * kPad]);
      const int live = ms_live_count(a.ctl, slot);
      const unsigned long long* live_w = accr + F_LIVE * kPad;
      float feat[kMaxSwitchFeatures];
      ms_features(feat, a, fresh, qlen, qslices, pairs_total - cumv, bt.count, live);
      int fallback = 0;
      const int engine = ms_choose(a, feat, qlen, pairs_total - cumv, level, bi, learned ? s_mlp : nullptr, &fallback);
      if (blockIdx.x == 0) ms_clear_slot(a.ctl, (level + 1) % kStatSlots);
      MsLevelRec* rec = (a.log && nrec < a.log_cap) ? a.log + nrec : nullptr;
      if (blockIdx.x == 0 && threadIdx.x == 0 && rec) {
        rec->batch = bi;
        rec->level = level;
        rec->engine = a.probe ? -1 : engine;
        rec->fallback = fallback;
        rec->width = bt.count;
        rec->live = live;
        rec->fresh = fresh;
        rec->queue = qlen;
        rec->qslices = qslices;
        rec->unvisited = pairs_total - cumv;
        rec->t_engine[0] = rec->t_engine[1] = 0ULL;
        for (int k = 0; k < kMaxSwitchFeatures; ++k) rec->feat[k] = feat[k];
      }
      ++nrec;
      if (a.probe) {
        // both engines from the same state: their marks are the same set
        const unsigned long long t0 = dev_ticks();
        ms_engine_bvss<SIGMA, SliceT, MF, ABL>(a, a.queue[level & 1], qlen, W, gwave, nwaves, my_f);
        if (!grid_barrier(a.ctl, bc)) return;
        const unsigned long long t1 = dev_ticks();
        ms_engine_pull<SIGMA, ABL>(a, W, bt.count, live_w, gtid, nthreads);
        if (!grid_barrier(a.ctl, bc)) return;
        if (blockIdx.x == 0 && threadIdx.x == 0 && rec) {
          rec->t_engine[0] = t1 - t0;
          rec->t_engine[1] = dev_ticks() - t1;
        }
      } else {
        if (engine == BLEST_ENGINE_BVSS)
          ms_engine_bvss<SIGMA, SliceT, MF, ABL>(a, a.queue[level & 1], qlen, W, gwave, nwaves, my_f);
        else
          ms_engine_pull<SIGMA, ABL>(a, W, bt.count, live_w, gtid, nthreads);
        if (!grid_barrier(a.ctl, bc)) return;
      }
      ms_finalize<SIGMA, BLOCK, ABL>(a, bt, level + 1, (level + 1) % kStatSlots, (level & 1) ^ 1, cumv, lds_cnt,
                                count_sources);
      if (!grid_barrier(a.ctl, bc)) return;
      total_levels = max(total_levels, level + 1);
    }
    if (a.lstage && a.ctl->error[0] == 0) ms_copy_levels<SIGMA, ABL>(a, bt, gtid, nthreads);
    if (count_sources) {
      // reduce the block partials of this batch
      for (long long c = gtid; c < bt.count; c += nthreads) {
        long long su = 0, re = 0;
        for (unsigned blk = 0; blk < gridDim.x; ++blk) {
          const long long* part = a.part + static_cast<long long>(blk) * (2 * 64 * kWMax);
          su += part[c];
          re += part[64 * kWMax + c];
        }
        const long long row = bt.offset + c;
        if (a.sums) a.sums[row] = su;
        if (a.reach) a.reach[row] = re;
        if (a.cc) a.cc[row] = su ? static_cast<double>(re - 1) / static_cast<double>(su) : 0.0;
      }
    }
    if (!grid_barrier(a.ctl, bc)) return;
  }
  if (blockIdx.x == 0) {
    if (threadIdx.x < 8) a.ctl->xcd_blocks[threadIdx.x][0] = 0u;
    if (threadIdx.x == 8) a.ctl->xcd_active[0] = 0u;
    if (threadIdx.x == 0) a.ctl->nlevels[0] = total_levels;
    if (threadIdx.x == 0) a.ctl->ms_nrec[0] = nrec;
  }
}

// ------------------------------------------------ hipGraph-captured levels
//
// The same traversal as k_ms_persistent, cut into one kernel per grid-wide
// phase so that a fixed sequence of launches can be captured in a hipGraph
// and replayed: the kernel's work is chosen by a state {phase, batch, level}
// in the control block. Kernel i of a graph reads state slot i % 2 and
// workgroup 0 writes the next state to the other slot (the next kernel starts
// only after every workgroup of this one has finished, so no workgroup reads a
// slot while it is being written). After the last batch the phase is
// MS_DONE and the remaining kernels of a replay do nothing.
enum MsPhase : int { MS_INIT = 0, MS_SEED = 1, MS_FIN0 = 2, MS_ENGINE = 3, MS_FIN = 4, MS_END = 5, MS_DONE = 6 };
constexpr int kMsGraphKernels = 32;  // kernels per graph (even)
static_assert(sizeof(MsDev::gnode) / sizeof(hipGraphNode_t) == kMsGraphKernels, "one node handle per kernel");

template <int SIGMA, class SliceT, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_ms_phase(MsArgs a, int parity) {
  constexpr int ABL = -1;
  extern __shared__ float s_mlp[];
  __shared__ unsigned long long lds_f[(BLOCK / 64) * ms_lds_words<SIGMA>()];
  __shared__ int lds_cnt[64 * kWMax];
  const int phase = a.ctl->ms_state[parity][0];
  const int bi = a.ctl->ms_state[parity][1];
  const int level = a.ctl->ms_state[parity][2];
  const int nrec = a.ctl->ms_state[parity][3];
  int next[4] = {MS_DONE, bi, level, nrec};
  if (phase != MS_DONE) {
    const long long nthreads = static_cast<long long>(gridDim.x) * BLOCK;
    const long long gtid = static_cast<long long>(blockIdx.x) * BLOCK + threadIdx.x;
    const int wave = wave_in_block();
    const long long gwave = static_cast<long long>(blockIdx.x) * (BLOCK / 64) + wave;
    const long long nwaves = static_cast<long long>(gridDim.x) * (BLOCK / 64);
    unsigned long long* my_f = lds_f + wave * ms_lds_words<SIGMA>();
    const long long rho = a.nsets;
    const long long nhat = a.nsets * SIGMA;
    const bool count_sources = a.sums != nullptr || a.reach != nullptr || a.cc != nullptr;
    for (int q = threadIdx.x; q < 64 * kWMax; q += BLOCK) lds_cnt[q] = 0;
    __syncthreads();
    const MsBatch bt = a.batches[bi];
    const int W = bt.W;
    switch (phase) {
      case MS_INIT:
        for (long long i = gtid; i < nhat * W; i += nthreads) {
          a.F[i] = 0ULL;
          a.V[i] = 0ULL;
          a.N[i] = 0ULL;
        }
        if (a.levels16 && !a.lstage) fill_minus_one(a.levels16 + static_cast<long long>(bt.offset) * a.n,
                                                    static_cast<long long>(bt.count) * a.n, gtid, nthreads);
        if (count_sources) {
          long long* part = a.part + static_cast<long long>(blockIdx.x) * (2 * 64 * kWMax);
          for (int q = threadIdx.x; q < 2 * 64 * kWMax; q += BLOCK) part[q] = 0;
        }
        if (blockIdx.x == 0)
          for (int t = 0; t < kStatSlots; ++t) ms_clear_slot(a.ctl, t);
        next[0] = MS_SEED;
        break;
      case MS_SEED:
        for (long long q = gtid; q < bt.count; q += nthreads) {
          const long long u = a.srcs[bt.offset + q];
          const long long vi = ms_vi<ABL>(a, u, rho, SIGMA);
          __hip_atomic_fetch_or(&a.N[vi * W + q / 64], 1ULL << (q % 64), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          a.dirty[u / SIGMA] = 1;
        }
        next[0] = MS_FIN0;
        break;
      case MS_FIN0:
        ms_finalize<SIGMA, BLOCK, ABL>(a, bt, 0, 0, 0, 0, lds_cnt, count_sources);
        next[0] = MS_ENGINE;
        next[2] = 0;
        break;
      case MS_ENGINE: {
        const unsigned long long* accr = &a.ctl->acc[level % kStatSlots][0][0];
        const long long fresh = static_cast<long long>(accr[F_FRONTIER * kPad]);
        if (fresh == 0) {
          next[0] = MS_END;
          break;
        }
        const long long qlen = static_cast<long long>(accr[F_QUEUE * kPad]);
        const long long qslices = static_cast<long long>(accr[F_QSLICES * kPad]);
        const long long cumv = static_cast<long long>(accr[F_CUMV * kPad]);
        const long long unv = static_cast<long long>(bt.count) * a.n - cumv;
        const bool learned = a.policy == BLEST_POLICY_LEARNED && a.mlp != nullptr && a.mlp->valid;
        if (learned) {
          mlp_to_lds(a.mlp, s_mlp);
          __syncthreads();
        }
        const int live = ms_live_count(a.ctl, level % kStatSlots);
        float feat[kMaxSwitchFeatures];
        ms_features(feat, a, fresh, qlen, qslices, unv, bt.count, live);
        int fallback = 0;
        const int engine = ms_choose(a, feat, qlen, unv, level, bi, learned ? s_mlp : nullptr, &fallback);
        if (blockIdx.x == 0) {
          ms_clear_slot(a.ctl, (level + 1) % kStatSlots);
          if (threadIdx.x == 0 && a.log && nrec < a.log_cap) {
            MsLevelRec* rec = a.log + nrec;
            rec->batch = bi;
            rec->level = level;
            rec->engine = engine;
            rec->fallback = fallback;
            rec->width = bt.count;
            rec->live = live;
            rec->fresh = fresh;
            rec->queue = qlen;
            rec->qslices = qslices;
            rec->unvisited = unv;
            rec->t_engine[0] = rec->t_engine[1] = 0ULL;
            for (int k = 0; k < kMaxSwitchFeatures; ++k) rec->feat[k] = feat[k];
          }
        }
        next[3] = nrec + 1;
        if (engine == BLEST_ENGINE_BVSS)
          ms_engine_bvss<SIGMA, SliceT, false, ABL>(a, a.queue[level & 1], qlen, W, gwave, nwaves, my_f);
        else
          ms_engine_pull<SIGMA, ABL>(a, W, bt.count, accr + F_LIVE * kPad, gtid, nthreads);
        next[0] = MS_FIN;
        break;
      }
      case MS_FIN: {
        const long long cumv = static_cast<long long>(a.ctl->acc[level % kStatSlots][F_CUMV][0]);
        ms_finalize<SIGMA, BLOCK, ABL>(a, bt, level + 1, (level + 1) % kStatSlots, (level & 1) ^ 1, cumv, lds_cnt,
                                  count_sources);
        next[0] = MS_ENGINE;
        next[2] = level + 1;
        break;
      }
      default:  // MS_END
        if (a.lstage && a.ctl->error[0] == 0) ms_copy_levels<SIGMA, ABL>(a, bt, gtid, nthreads);
        if (count_sources) {
          for (long long q = gtid; q < bt.count; q += nthreads) {
            long long su = 0, re = 0;
            for (unsigned blk = 0; blk < gridDim.x; ++blk) {
              const long long* part = a.part + static_cast<long long>(blk) * (2 * 64 * kWMax);
              su += part[q];
              re += part[64 * kWMax + q];
            }
            const long long row = bt.offset + q;
            if (a.sums) a.sums[row] = su;
            if (a.reach) a.reach[row] = re;
            if (a.cc) a.cc[row] = su ? static_cast<double>(re - 1) / static_cast<double>(su) : 0.0;
          }
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
          if (level > a.ctl->nlevels[0]) a.ctl->nlevels[0] = level;
          a.ctl->ms_nrec[0] = nrec;
        }
        next[0] = bi + 1 < a.nbatches ? MS_INIT : MS_DONE;
        next[1] = bi + 1;
        next[2] = 0;
        break;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (int i = 0; i < 4; ++i) a.ctl->ms_state[parity ^ 1][i] = next[i];
}

__global__ void k_ms_start(Ctl* ctl) {
  if (threadIdx.x == 0) {
    ctl->ms_state[0][0] = MS_INIT;
    ctl->ms_state[0][1] = 0;
    ctl->ms_state[0][2] = 0;
    ctl->ms_state[0][3] = 0;
    ctl->nlevels[0] = 0;
    ctl->ms_nrec[0] = 0;
  }
}

template <int SIGMA, class SliceT>
const void* ms_phase_fn() {
  return reinterpret_cast<const void*>(&k_ms_phase<SIGMA, SliceT, 512>);
}

template <int SIGMA, class SliceT, int BLOCK>
const void* ms_fn() {
  return reinterpret_cast<const void*>(&k_ms_persistent<SIGMA, SliceT, BLOCK>);
}

template <int SIGMA, class SliceT>
const void* ms_fn_block(int block) {
  switch (block) {
    case 256:
      return ms_fn<SIGMA, SliceT, 256>();
    case 1024:
      return ms_fn<SIGMA, SliceT, 1024>();
    default:
      return ms_fn<SIGMA, SliceT, 512>();
  }
}

// The multi-source kernel keeps sigma words per slice set live in Stage 2;
// 512-thread blocks leave it enough registers to avoid spilling at sigma 8.
constexpr int kMsBlock = 512;
constexpr int kMsLogCap = 1 << 16;  // level records per call

const void* ms_kernel(const DevGraph& g) {
  // the matrix-core check and the ablation steps are kernels of their own, so
  // their registers and branches never weigh on the full method's kernel
  if (g.ms_mfma && g.sigma == 8)
    return g.wide ? reinterpret_cast<const void*>(&k_ms_persistent<8, uint64_t, kMsBlock, 1>)
                  : reinterpret_cast<const void*>(&k_ms_persistent<8, uint32_t, kMsBlock, 1>);
  if (g.ms_ablation && g.sigma == 8) {
    if (g.wide)
      return g.ms_ablation == 1   ? reinterpret_cast<const void*>(&k_ms_persistent<8, uint64_t, kMsBlock, 11>)
             : g.ms_ablation == 2 ? reinterpret_cast<const void*>(&k_ms_persistent<8, uint64_t, kMsBlock, 12>)
                                  : reinterpret_cast<const void*>(&k_ms_persistent<8, uint64_t, kMsBlock, 13>);
    return g.ms_ablation == 1   ? reinterpret_cast<const void*>(&k_ms_persistent<8, uint32_t, kMsBlock, 11>)
           : g.ms_ablation == 2 ? reinterpret_cast<const void*>(&k_ms_persistent<8, uint32_t, kMsBlock, 12>)
                                : reinterpret_cast<const void*>(&k_ms_persistent<8, uint32_t, kMsBlock, 13>);
  }
  if (g.sigma == 8 && !g.wide) return ms_fn_block<8, uint32_t>(kMsBlock);
  if (g.sigma == 8) return ms_fn_block<8, uint64_t>(kMsBlock);
  if (g.sigma == 16) return ms_fn_block<16, uint64_t>(kMsBlock);
  return ms_fn_block<32, uint64_t>(kMsBlock);
}

void ms_graph_destroy(MsDev* ms) {
  if (ms->gexec) (void)hipGraphExecDestroy(ms->gexec);
  if (ms->graph) (void)hipGraphDestroy(ms->graph);
  ms->gexec = nullptr;
  ms->graph = nullptr;
  ms->gfn = nullptr;
  for (auto& nd : ms->gnode) nd = nullptr;
}

hipError_t ensure(const DevGraph& g, MsDev* ms, int wmax, int32_t k, int nbatches) {
  const int64_t nhat = g.nsets * g.sigma;
  if (ms->wmax < wmax || ms->nhat != nhat) {
    ms_release(ms);
    const size_t words = static_cast<size_t>(nhat) * wmax;
    hipError_t e;
    if ((e = hipMalloc(&ms->F, words * 8)) != hipSuccess) return e;
    if ((e = hipMalloc(&ms->V, words * 8)) != hipSuccess) return e;
    if ((e = hipMalloc(&ms->N, words * 8)) != hipSuccess) return e;
    if ((e = hipMalloc(&ms->act, static_cast<size_t>(g.nsets) * wmax * 8)) != hipSuccess) return e;
    if ((e = hipMalloc(&ms->dirty, static_cast<size_t>(g.nsets))) != hipSuccess) return e;
    for (int i = 0; i < 2; ++i)
      if ((e = hipMalloc(&ms->queue[i], sizeof(uint4) * static_cast<size_t>(std::max<int64_t>(g.nvss, 1)))) !=
          hipSuccess)
        return e;
    if ((e = hipMemset(ms->N, 0, words * 8)) != hipSuccess) return e;
    if ((e = hipMemset(ms->dirty, 0, static_cast<size_t>(g.nsets))) != hipSuccess) return e;
    ms->wmax = wmax;
    ms->nhat = nhat;
    ms->nsets = g.nsets;
  }
  if (ms->srcs_cap < k) {
    if (ms->srcs) (void)hipFree(ms->srcs);
    ms->srcs = nullptr;
    hipError_t e = hipMalloc(&ms->srcs, sizeof(int32_t) * static_cast<size_t>(k));
    if (e != hipSuccess) return e;
    ms->srcs_cap = k;
  }
  if (ms->batches_cap < nbatches) {
    if (ms->batches) (void)hipFree(ms->batches);
    ms->batches = nullptr;
    hipError_t e = hipMalloc(&ms->batches, sizeof(MsBatch) * static_cast<size_t>(nbatches));
    if (e != hipSuccess) return e;
    ms->batches_cap = nbatches;
  }
  if (ms->grid == 0) {
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ms_kernel(g), kMsBlock,
                                                                 kLdsMlpFloats * sizeof(float));
    if (e != hipSuccess) return e;
    if (nb < 1) return hipErrorInvalidConfiguration;
    nb = std::min(nb, 2);
    ms->grid = nb * g.num_cu;
    ms->block = kMsBlock;
  }
  if (!ms->log) {
    hipError_t e = hipMalloc(&ms->log, sizeof(MsLevelRec) * static_cast<size_t>(kMsLogCap));
    if (e != hipSuccess) return e;
    ms->log_cap = kMsLogCap;
  }
  if (ms->part_blocks < ms->grid) {
    if (ms->part) (void)hipFree(ms->part);
    ms->part = nullptr;
    hipError_t e = hipMalloc(&ms->part, sizeof(long long) * 2 * 64 * kWMax * static_cast<size_t>(ms->grid));
    if (e != hipSuccess) return e;
    ms->part_blocks = ms->grid;
  }
  return hipSuccess;
}

// Kernel arguments of one multi-source call whose source list and batch plan
// are already on the device (srcs_dev, batches_dev).
MsArgs ms_args(const DevGraph& g, const MsDev* ms, const int32_t* srcs_dev, const MsBatch* batches_dev, int nplan,
               int policy, float eta, uint64_t seed, int16_t* levels16, int64_t* sums, int64_t* reach, double* cc,
               int64_t* far, int probe) {
  MsArgs a{};
  a.rp = g.rp;
  a.col = g.col;
  a.rp_in = g.rp_in;
  a.col_in = g.col_in;
  a.slice_ptr = g.slice_ptr;
  a.slices = g.slices;
  a.orig_id = g.orig_id;
  a.n = g.n;
  a.m = g.m;
  a.nsets = g.nsets;
  a.tau = g.tau;
  a.F = ms->F;
  a.V = ms->V;
  a.N = ms->N;
  a.act = ms->act;
  a.dirty = ms->dirty;
  a.queue[0] = ms->queue[0];
  a.queue[1] = ms->queue[1];
  a.srcs = srcs_dev;
  a.batches = batches_dev;
  a.nbatches = nplan;
  a.levels16 = levels16;
  a.lstage = levels16 ? ms->lstage : nullptr;
  a.perm = ms->perm;
  a.sums = sums;
  a.reach = reach;
  a.cc = cc;
  a.far = far;
  a.nvss = g.nvss;
  a.nslices = g.nslices;
  a.mlp = g.ms_mlp;
  a.probe = probe;
  a.log = ms->log;
  a.log_cap = ms->log_cap;
  a.part = ms->part;
  a.ctl = g.ctl;
  a.policy = policy;
  a.eta = eta;
  a.seed = seed;
  a.timeout_ticks = 3000000000ULL;  // 30 s
  a.ablation = g.ms_ablation;
  return a;
}

}  // namespace

__global__ void k_ms_perm(const int32_t* __restrict__ orig_id, int64_t n, int32_t* __restrict__ perm) {
  for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    perm[orig_id[i]] = static_cast<int32_t>(i);
}

// Staging rows for the int16 level output of batches up to 64 * wmax wide,
// and (for a relabelled graph) the input -> internal id map they are read
// back through.
hipError_t ensure_levels(const DevGraph& g, MsDev* ms, int wmax, hipStream_t st) {
  const int64_t need = g.n * 64 * static_cast<int64_t>(wmax);
  hipError_t e;
  if (ms->lstage_elems < need) {
    if (ms->lstage) (void)hipFree(ms->lstage);
    ms->lstage = nullptr;
    ms->lstage_elems = 0;
    if ((e = hipMalloc(&ms->lstage, sizeof(int16_t) * static_cast<size_t>(need))) != hipSuccess) return e;
    ms->lstage_elems = need;
  }
  if (g.orig_id && !ms->perm) {
    if ((e = hipMalloc(&ms->perm, sizeof(int32_t) * static_cast<size_t>(std::max<int64_t>(g.n, 1)))) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_ms_perm, dim3(static_cast<unsigned>(std::min<int64_t>((g.n + 255) / 256, 4096))),
                       dim3(256), 0, st, g.orig_id, g.n, ms->perm);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t ms_run(const DevGraph& g, MsDev* ms, const int32_t* srcs, int32_t k, const int32_t* widths, int nwidths,
                  int policy, float eta, uint64_t seed, int16_t* levels16, int64_t* sums, int64_t* reach, double* cc,
                  hipStream_t st, int graph, int64_t* far, int probe) {
  if (k <= 0) return hipSuccess;
  std::vector<MsBatch> plan;
  int32_t off = 0;
  for (int i = 0; off < k; ++i) {
    const int width = widths[nwidths > 0 ? std::min(i, nwidths - 1) : 0];
    const int W = width / 64;
    plan.push_back(MsBatch{off, std::min(64 * W, k - off), W, 0});
    off += 64 * W;
  }
  const int nplan = static_cast<int>(plan.size());
  int wmax = 1;
  for (int i = 0; i < nplan; ++i) wmax = std::max(wmax, plan[i].W);
  hipError_t e = ensure(g, ms, wmax, k, nplan);
  if (e != hipSuccess) return e;
  if (levels16 && (e = ensure_levels(g, ms, wmax, st)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(ms->srcs, srcs, sizeof(int32_t) * k, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(ms->batches, plan.data(), sizeof(MsBatch) * nplan, hipMemcpyHostToDevice, st)) !=
      hipSuccess)
    return e;
  // the copies read pageable host memory; wait so `plan` may go out of scope
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  MsArgs a = ms_args(g, ms, ms->srcs, static_cast<const MsBatch*>(ms->batches), nplan, policy, eta, seed, levels16,
                     sums, reach, cc, far, probe);
  const unsigned shmem = policy == BLEST_POLICY_LEARNED ? kLdsMlpFloats * sizeof(float) : 0u;
  if (!graph || probe) {
    void* args[] = {static_cast<void*>(&a)};
    return hipLaunchCooperativeKernel(ms_kernel(g), dim3(ms->grid), dim3(ms->block), args, shmem, st);
  }
  // Graph mode: kMsGraphKernels phase kernels, then copies of the state and
  // error words to pinned host memory, built once as a hipGraph for a stream
  // of our own (the caller's may be the null stream) and replayed until the
  // state says MS_DONE. One instantiated graph serves every call with the
  // same kernel, grid and LDS size: a call only rewrites the kernel nodes'
  // arguments. The replays are ordered after the caller's stream by an event.
  if (!ms->gstream) {
    if ((e = hipStreamCreateWithFlags(&ms->gstream, hipStreamNonBlocking)) != hipSuccess) return e;
    for (int i = 0; i < 2; ++i)
      if ((e = hipEventCreateWithFlags(&ms->gev[i], hipEventDisableTiming)) != hipSuccess) return e;
  }
  const void* fn = (g.sigma == 8 && !g.wide) ? ms_phase_fn<8, uint32_t>()
                   : g.sigma == 8            ? ms_phase_fn<8, uint64_t>()
                   : g.sigma == 16           ? ms_phase_fn<16, uint64_t>()
                                             : ms_phase_fn<32, uint64_t>();
  hipStream_t gs = ms->gstream;
  int* flags = g.host_flags;
  int par[kMsGraphKernels];
  void* kargs[kMsGraphKernels][2];
  hipKernelNodeParams kp[kMsGraphKernels];
  for (int i = 0; i < kMsGraphKernels; ++i) {
    par[i] = i & 1;
    kargs[i][0] = static_cast<void*>(&a);
    kargs[i][1] = static_cast<void*>(&par[i]);
    kp[i] = hipKernelNodeParams{};
    kp[i].func = const_cast<void*>(fn);
    kp[i].gridDim = dim3(ms->grid);
    kp[i].blockDim = dim3(kMsBlock);
    kp[i].sharedMemBytes = shmem;
    kp[i].kernelParams = kargs[i];
    kp[i].extra = nullptr;
  }
  if (ms->gexec && (ms->gfn != fn || ms->ggrid != ms->grid || ms->gshmem != shmem)) {
    ms_graph_destroy(ms);
  }
  if (!ms->gexec) {
    if ((e = hipGraphCreate(&ms->graph, 0)) != hipSuccess) return e;
    hipGraphNode_t prev = nullptr;
    for (int i = 0; i < kMsGraphKernels && e == hipSuccess; ++i) {
      e = hipGraphAddKernelNode(&ms->gnode[i], ms->graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp[i]);
      prev = ms->gnode[i];
    }
    hipGraphNode_t cp[2] = {nullptr, nullptr};
    if (e == hipSuccess)
      e = hipGraphAddMemcpyNode1D(&cp[0], ms->graph, &prev, 1, flags + 2, &g.ctl->ms_state[0][0], sizeof(int),
                                  hipMemcpyDeviceToHost);
    if (e == hipSuccess)
      e = hipGraphAddMemcpyNode1D(&cp[1], ms->graph, &cp[0], 1, flags + 3, &g.ctl->error[0], sizeof(int),
                                  hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipGraphInstantiate(&ms->gexec, ms->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      ms_graph_destroy(ms);
      return e;
    }
    ms->gfn = fn;
    ms->ggrid = ms->grid;
    ms->gshmem = shmem;
    ++ms->gcaptures;
  } else {
    for (int i = 0; i < kMsGraphKernels; ++i)
      if ((e = hipGraphExecKernelNodeSetParams(ms->gexec, ms->gnode[i], &kp[i])) != hipSuccess) return e;
  }
  if ((e = hipEventRecord(ms->gev[0], st)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(gs, ms->gev[0], 0)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_ms_start, dim3(1), dim3(64), 0, gs, g.ctl);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // every batch has at most 3 + 2 * 32768 + 1 phases (levels are int16)
  const long long max_replays = static_cast<long long>(nplan) * (2LL * 32768 + 4) / kMsGraphKernels + 2;
  for (long long r = 0; e == hipSuccess; ++r) {
    if (r >= max_replays) {
      e = hipErrorLaunchTimeOut;
      break;
    }
    if ((e = hipGraphLaunch(ms->gexec, gs)) != hipSuccess) break;
    if ((e = hipStreamSynchronize(gs)) != hipSuccess) break;
    if (flags[2] == MS_DONE || flags[3] != 0) break;
  }
  if (e != hipSuccess) return e;
  if ((e = hipEventRecord(ms->gev[1], gs)) != hipSuccess) return e;
  return hipStreamWaitEvent(st, ms->gev[1], 0);
}

void ms_release(MsDev* ms) {
  for (void* p : {static_cast<void*>(ms->F), static_cast<void*>(ms->V), static_cast<void*>(ms->N),
                  static_cast<void*>(ms->act), static_cast<void*>(ms->dirty), static_cast<void*>(ms->queue[0]),
                  static_cast<void*>(ms->queue[1])})
    if (p) (void)hipFree(p);
  ms->F = ms->V = ms->N = ms->act = nullptr;
  ms->dirty = nullptr;
  ms->queue[0] = ms->queue[1] = nullptr;
  ms->wmax = 0;
  ms->nhat = 0;
  if (ms->lstage) (void)hipFree(ms->lstage);
  if (ms->perm) (void)hipFree(ms->perm);
  ms->lstage = nullptr;
  ms->lstage_elems = 0;
  ms->perm = nullptr;
}

void ms_free_all(MsDev* ms) {
  ms_release(ms);
  ms_graph_destroy(ms);
  if (ms->gstream) (void)hipStreamDestroy(ms->gstream);
  for (int i = 0; i < 2; ++i)
    if (ms->gev[i]) (void)hipEventDestroy(ms->gev[i]);
  ms->gstream = nullptr;
  ms->gev[0] = ms->gev[1] = nullptr;
  if (ms->srcs) (void)hipFree(ms->srcs);
  if (ms->part) (void)hipFree(ms->part);
  if (ms->batches) (void)hipFree(ms->batches);
  if (ms->log) (void)hipFree(ms->log);
  ms->log = nullptr;
  ms->log_cap = 0;
  ms->srcs = nullptr;
  ms->part = nullptr;
  ms->batches = nullptr;
  ms->srcs_cap = 0;
  ms->part_blocks = 0;
  ms->batches_cap = 0;
  ms->grid = 0;
}

void ms_reset(MsDev* ms) {
  // After a device-side error N and dirty may hold stale marks.
  if (ms->N && ms->nhat) (void)hipMemset(ms->N, 0, static_cast<size_t>(ms->nhat) * ms->wmax * 8);
  if (ms->dirty && ms->nsets) (void)hipMemset(ms->dirty, 0, static_cast<size_t>(ms->nsets));
}

// ----------------------------------------------------------- no-alloc entry
// blest_msbfs_noalloc keeps the source list and the batch plan of a call in
// this array instead of in buffers the library allocates: the first
// BLEST_MSBFS_NOALLOC_MAX_SOURCES entries hold internal source ids, then one
// 4-int batch descriptor per batch (at most one per 64 sources). Each device
// holds its own copy until the process ends; host code reaches it only
// through the address hipGetSymbolAddress gives for the current device.
constexpr int kNoAllocMaxSources = BLEST_MSBFS_NOALLOC_MAX_SOURCES;
constexpr int kNoAllocMaxBatches = kNoAllocMaxSources / 64;
static_assert(sizeof(MsBatch) == 4 * sizeof(int32_t), "batch descriptor layout");
static __device__ __align__(256) int32_t scratch[kNoAllocMaxSources + 4 * kNoAllocMaxBatches];

namespace {

constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
int32_t* g_noalloc_ptr[kNoAllocDevices] = {};

// This device's copy of `scratch`, looked up once per device (the caller
// has made `device` current).
hipError_t noalloc_scratch(int device, int32_t** out) {
  if (device < 0 || device >= kNoAllocDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_noalloc_ptr[device] = static_cast<int32_t*>(p);
  }
  *out = g_noalloc_ptr[device];
  return hipSuccess;
}

}  // namespace

bool ms_ready(const DevGraph& g, const MsDev* ms, int W) {
  return ms->wmax >= W && ms->nhat == g.nsets * g.sigma && ms->F && ms->V && ms->N && ms->act && ms->dirty &&
         ms->queue[0] && ms->queue[1] && ms->grid > 0 && ms->log && ms->part && ms->part_blocks >= ms->grid;
}

hipError_t ms_run_noalloc(const DevGraph& g, MsDev* ms, const int32_t* srcs, const int32_t* perm, int32_t k,
                          int width, int policy, float eta, uint64_t seed, int16_t* levels16, hipStream_t st) {
  if (k <= 0) return hipSuccess;
  if (k > kNoAllocMaxSources || width % 64 != 0 || width < 64 || width > 64 * kWMax) return hipErrorInvalidValue;
  const int W = width / 64;
  if (!ms_ready(g, ms, W)) return hipErrorNotReady;
  int32_t* base = nullptr;
  hipError_t e = noalloc_scratch(g.device, &base);
  if (e != hipSuccess) return e;
  int32_t* dsrcs = base;
  MsBatch* dplan = reinterpret_cast<MsBatch*>(base + kNoAllocMaxSources);
  // Internal source ids through a fixed host staging buffer; the copies read
  // pageable memory, so each is waited for before the buffer is refilled.
  constexpr int kStage = 4096;
  int32_t stage[kStage];
  for (int32_t off = 0; off < k; off += kStage) {
    const int32_t c = std::min<int32_t>(kStage, k - off);
    for (int32_t i = 0; i < c; ++i) stage[i] = perm ? perm[srcs[off + i]] : srcs[off + i];
    if ((e = hipMemcpyAsync(dsrcs + off, stage, sizeof(int32_t) * c, hipMemcpyHostToDevice, st)) != hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  }
  const int per = 64 * W;
  const int nplan = (k + per - 1) / per;
  MsBatch plan[kNoAllocMaxBatches];
  for (int i = 0; i < nplan; ++i) plan[i] = MsBatch{i * per, std::min(per, k - i * per), W, 0};
  if ((e = hipMemcpyAsync(dplan, plan, sizeof(MsBatch) * nplan, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  MsArgs a = ms_args(g, ms, dsrcs, dplan, nplan, policy, eta, seed, levels16, nullptr, nullptr, nullptr, nullptr, 0);
  // no staging buffer here (the entry point allocates nothing): Stage 2
  // writes the caller's rows directly
  a.lstage = nullptr;
  const unsigned shmem = policy == BLEST_POLICY_LEARNED ? kLdsMlpFloats * sizeof(float) : 0u;
  void* args[] = {static_cast<void*>(&a)};
  return hipLaunchCooperativeKernel(ms_kernel(g), dim3(ms->grid), dim3(ms->block), args, shmem, st);
}

}  // namespace blest
