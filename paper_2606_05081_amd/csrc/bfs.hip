// Single-source BVSS breadth-first search for gfx950.
//
// One traversal step turns frontier level l into level l+1 in two stages
// (Section "Lazy Vertex Updates", Alg. 3):
//   Stage 1 marks every vertex that has a neighbour in the frontier, with a
//           plain byte store of 1 into mark[] (idempotent, so no atomics).
//           Three interchangeable engines do this:
//             E0 BVSS top-down: one wave per queued virtual slice set; each
//                lane tests (mask & alpha) != 0 for its slices, alpha being
//                the frontier bits of the set (Eq. 1 / Eq. 2, popc(a&x) > 0
//                written as a bitwise AND).
//             E1 push: frontier vertices walk their CSR rows.
//             E2 bottom-up (Alg. 4): each unvisited vertex scans its row and
//                stops at the first frontier neighbour.
//   Stage 2 sweeps the marks of every slice set, keeps the bits not yet
//           visited (the XOR of V_next and V_curr), writes their level,
//           updates visited/frontier words, enqueues every VSS of each set
//           that gained a vertex and accumulates the per-level statistics.
// The engine of each step is chosen on the device (Eq. 3 heuristic, learned
// network, fixed or random) identically by every workgroup. All levels run in
// one cooperative persistent launch separated by a device-wide barrier
// (Section "Switching Mechanism", last paragraph); a per-stage launch mode is
// kept for comparison.
#include "device_common.h"
#include "mlp_infer.h"

namespace blest {

// Frontier buffer of a level parity (level l reads buffer l & 1; its Stage 2
// writes the other one, so an engine never reads words being rewritten).
__device__ __forceinline__ void* front_buf(const BfsArgs& a, int sel) {
  return static_cast<char*>(a.front) + (sel ? a.fstride : 0LL);
}

// Per-workgroup Stage 2 partial counters: frontier, queued slices, frontier
// edges, deg >= 32, deg >= 1024, light, heavy and queue entries.
constexpr int kParts = 8;

// Row pointers rp[s*SIGMA .. s*SIGMA + SIGMA] of a slice set's vertices with
// 16-byte loads. rp is padded on the device to N_s*SIGMA + 1 entries (the
// tail repeats m), and s*SIGMA*4 is a multiple of 16, so the loads are aligned
// and in bounds.
template <int SIGMA>
__device__ __forceinline__ void load_set_rp(gptr<const int32_t> rp, long long s, int (&r)[SIGMA + 1]) {
  const gptr<const int4> p = (gptr<const int4>)(rp + s * SIGMA);
#pragma unroll
  for (int i = 0; i < SIGMA / 4; ++i) {
    const int4 q = p[i];
    r[4 * i + 0] = q.x;
    r[4 * i + 1] = q.y;
    r[4 * i + 2] = q.z;
    r[4 * i + 3] = q.w;
  }
  r[SIGMA] = rp[s * SIGMA + SIGMA];
}

// ------------------------------------------------------------- decisions

struct LevelView {
  long long frontier, queue, qslices, fedges, deg32, deg1024, light, heavy, cumv, cume;
};

__device__ __forceinline__ LevelView read_level(const Ctl* ctl, int slot) {
  const gptr<const unsigned long long> acc = to_global(&ctl->acc[slot][0][0]);
  LevelView v;
  v.frontier = static_cast<long long>(acc[F_FRONTIER * kPad]);
  v.queue = static_cast<long long>(acc[F_QUEUE * kPad]);
  v.qslices = static_cast<long long>(acc[F_QSLICES * kPad]);
  v.fedges = static_cast<long long>(acc[F_FEDGES * kPad]);
  v.deg32 = static_cast<long long>(acc[F_DEG32 * kPad]);
  v.deg1024 = static_cast<long long>(acc[F_DEG1024 * kPad]);
  v.light = static_cast<long long>(acc[F_LIGHT * kPad]);
  v.heavy = static_cast<long long>(acc[F_HEAVY * kPad]);
  v.cumv = static_cast<long long>(acc[F_CUMV * kPad]);
  v.cume = static_cast<long long>(acc[F_CUME * kPad]);
  return v;
}

// Same, with agent-scope loads (used inside a single-workgroup episode, where
// the counters were just updated by device atomics without a barrier).
__device__ __forceinline__ LevelView read_level_atomic(const Ctl* ctl, int slot) {
  const gptr<const unsigned long long> acc = to_global(&ctl->acc[slot][0][0]);
  LevelView v;
  v.frontier = static_cast<long long>(ld_relaxed_u64(acc + F_FRONTIER * kPad));
  v.queue = static_cast<long long>(ld_relaxed_u64(acc + F_QUEUE * kPad));
  v.qslices = static_cast<long long>(ld_relaxed_u64(acc + F_QSLICES * kPad));
  v.fedges = static_cast<long long>(ld_relaxed_u64(acc + F_FEDGES * kPad));
  v.deg32 = static_cast<long long>(ld_relaxed_u64(acc + F_DEG32 * kPad));
  v.deg1024 = static_cast<long long>(ld_relaxed_u64(acc + F_DEG1024 * kPad));
  v.light = static_cast<long long>(ld_relaxed_u64(acc + F_LIGHT * kPad));
  v.heavy = static_cast<long long>(ld_relaxed_u64(acc + F_HEAVY * kPad));
  v.cumv = static_cast<long long>(ld_relaxed_u64(acc + F_CUMV * kPad));
  v.cume = static_cast<long long>(ld_relaxed_u64(acc + F_CUME * kPad));
  return v;
}

// The 12 switch features of a level (network inputs before standardising).
__device__ __forceinline__ void level_features(float (&f)[kMaxSwitchFeatures], const LevelView& v, const BfsArgs& a,
                                               int level, long long prev_frontier) {
  (void)level;
  const long long unv = a.n - v.cumv, unv_e = a.m - v.cume;
  const float lf = log2f(1.0f + static_cast<float>(v.frontier));
  const float lqs = log2f(1.0f + static_cast<float>(v.qslices));
  const float ln = log2f(static_cast<float>(a.n));
  const float lm = log2f(1.0f + static_cast<float>(a.m));
  (void)lm;
  f[0] = lf;
  f[1] = lqs;
  f[2] = lf - ln;
  f[3] = log2f(1.0f + static_cast<float>(v.queue)) - log2f(1.0f + static_cast<float>(a.nvss));
  f[4] = lqs - log2f(1.0f + static_cast<float>(a.nslices));
  f[5] = log2f(1.0f + static_cast<float>(v.fedges)) - lm;
  f[6] = log2f(1.0f + static_cast<float>(unv)) - ln;
  f[7] = log2f(1.0f + static_cast<float>(unv_e)) - lm;
  // Eq. 3's own quantities, as a log ratio
  f[8] = log2f(1.0f + static_cast<float>(v.queue)) - log2f(1.0f + static_cast<float>(unv));
  // Reserved (zero). The frontier degree histogram and the growth ratio were
  // inputs once; on R-MAT + grid training data they let the network learn
  // family shortcuts that failed on Erdos-Renyi graphs.
  (void)prev_frontier;
  f[9] = 0.0f;
  f[10] = 0.0f;
  f[11] = 0.0f;
}

// Eq. 3: bottom-up iff #unvisited < eta * |Q_curr| (|Q| counts VSSs).
__device__ __forceinline__ int heuristic_engine(long long unvisited, long long queue, float eta) {
  return (static_cast<double>(unvisited) < static_cast<double>(eta) * static_cast<double>(queue))
             ? BLEST_ENGINE_BOTTOM_UP
             : BLEST_ENGINE_BVSS;
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Uniform engine choice for the step out of `level`. Contains __syncthreads().
__device__ __forceinline__ int choose_engine_inl(const BfsArgs& a, const LevelView& v,
                                                 const float (&feat)[kMaxSwitchFeatures], int level,
                                                 const float* s_mlp, int* fallback) {
  __shared__ int s_choice;
  const long long unvisited = a.n - v.cumv;
  *fallback = 0;
  switch (a.policy) {
    case BLEST_POLICY_BVSS:
      return BLEST_ENGINE_BVSS;
    case BLEST_POLICY_PUSH:
      return BLEST_ENGINE_PUSH;
    case BLEST_POLICY_BOTTOM_UP:
      return BLEST_ENGINE_BOTTOM_UP;
    case BLEST_POLICY_RANDOM:
      return static_cast<int>(mix64(a.seed + 0x9E3779B97F4A7C15ULL * static_cast<unsigned long long>(level + 1)) % 3ULL);
    case BLEST_POLICY_LEARNED:
      if (s_mlp != nullptr) {
        if (threadIdx.x < 64) {
          int c = mlp_choose_wave(s_mlp, feat);
          if (threadIdx.x == 0) s_choice = c;
        }
        __syncthreads();
        int c = s_choice;
        __syncthreads();
        if (c >= 0) return c;
      }
      *fallback = 1;
      return heuristic_engine(unvisited, v.queue, a.eta);
    default:
      return heuristic_engine(unvisited, v.queue, a.eta);
  }
}

// The same as an out-of-line call (the lazy kernel, where inlining it would
// only add to the register pressure).
__device__ int choose_engine(const BfsArgs& a, const LevelView& v, const float (&feat)[kMaxSwitchFeatures],
                             int level, const float* s_mlp, int* fallback) {
  return choose_engine_inl(a, v, feat, level, s_mlp, fallback);
}

// ------------------------------------------------------------ Stage 1

constexpr int kSingleHash = 8192;              // LDS hash-set slots (power of two)
constexpr long long kSingleMaxMarks = 4096;    // keeps the hash set at most half full
// LDS layout of a single-workgroup level: hs[kSingleHash] hash slots, then
// the list of recorded sets hs[kSingleHash + 1 + i] with its length at
// hs[kSingleHash].
constexpr int kSingleLds = kSingleHash + 1 + kSingleMaxMarks;

__device__ __forceinline__ void record_set(lptr<int> hs, long long s, Ctl* ctl) {
  uint32_t h = (static_cast<uint32_t>(s) * 2654435761u) >> (32 - 13);
  for (int probe = 0; probe < kSingleHash; ++probe) {
    int old = -1;
    __hip_atomic_compare_exchange_strong(hs + h, &old, static_cast<int>(s), __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
    if (old == -1) {
      const int idx = __hip_atomic_fetch_add(hs + kSingleHash, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      hs[kSingleHash + 1 + idx] = static_cast<int>(s);
      return;
    }
    if (old == static_cast<int>(s)) return;
    h = (h + 1) & (kSingleHash - 1);
  }
  __hip_atomic_store(&ctl->error[0], static_cast<int>(BLEST_ERR_INVALID_ARG), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}


// E0: BVSS top-down with pull mechanics and lazy marking. A wave takes G
// consecutive queue entries at a time and issues all their slice loads before
// testing any, so each lane keeps G * K independent loads in flight
// (K = tau / 64 slices per lane per VSS).
template <int SIGMA, class SliceT, int K, bool REC>
__device__ long long engine_bvss_k(const BfsArgs& a, const uint4* __restrict__ q, long long qlen, long long gwave,
                                   long long nwaves, lptr<int> hs) {
  long long work = 0;
  using M = typename MaskOf<SIGMA>::T;
  constexpr int G = 4;
  const gptr<const uint4> qg = to_global(q);
  gptr<const SliceT> __restrict__ sl = to_global(static_cast<const SliceT*>(a.slices));
  gptr<const M> __restrict__ vis = to_global(static_cast<const M*>(a.vis));
  gptr<uint8_t> __restrict__ mark = to_global(a.mark);
  const uint32_t lane = static_cast<uint32_t>(lane_id());
  const bool pre = a.prefilter != 0;
  for (long long base = gwave * G; base < qlen; base += nwaves * G) {
    uint4 dl = make_uint4(0u, 0u, 0u, 0u);
    if (lane < G && base + lane < qlen) dl = qg[base + lane];
    uint32_t st[G], cn[G];
    SliceT al[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      st[g] = __builtin_amdgcn_readlane(dl.x, g);
      cn[g] = __builtin_amdgcn_readlane(dl.y, g);
      al[g] = static_cast<SliceT>(static_cast<uint32_t>(__builtin_amdgcn_readlane(dl.z, g)));
    }
    SliceT w[G][K];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint32_t j = lane + 64u * k;
        work += j < cn[g];
        w[g][k] = (j < cn[g]) ? sl[st[g] + j] : SliceT(0);
      }
    if (pre) {
      M vv[G][K];
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const uint32_t row = static_cast<uint32_t>(w[g][k] >> SliceFmt<SliceT>::kRowShift);
          vv[g][k] = (w[g][k] & al[g]) ? vis[row / SIGMA] : M(~M(0));
        }
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const uint32_t row = static_cast<uint32_t>(w[g][k] >> SliceFmt<SliceT>::kRowShift);
          if (!((vv[g][k] >> (row % SIGMA)) & 1u)) {
            mark[row] = 1;
            if (REC) record_set(hs, row / SIGMA, a.ctl);
          }
        }
    } else {
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int k = 0; k < K; ++k)
          if (w[g][k] & al[g]) {
            const uint32_t row = static_cast<uint32_t>(w[g][k] >> SliceFmt<SliceT>::kRowShift);
            mark[row] = 1;
            if (REC) record_set(hs, row / SIGMA, a.ctl);
          }
    }
  }
  return work;
}

template <int SIGMA, class SliceT, bool REC>
__device__ long long engine_bvss(const BfsArgs& a, const uint4* __restrict__ q, long long qlen, long long gwave,
                                 long long nwaves, lptr<int> hs) {
  switch (a.tau) {
    case 64:
      return engine_bvss_k<SIGMA, SliceT, 1, REC>(a, q, qlen, gwave, nwaves, hs);
    case 128:
      return engine_bvss_k<SIGMA, SliceT, 2, REC>(a, q, qlen, gwave, nwaves, hs);
    case 192:
      return engine_bvss_k<SIGMA, SliceT, 3, REC>(a, q, qlen, gwave, nwaves, hs);
    default:
      return engine_bvss_k<SIGMA, SliceT, 4, REC>(a, q, qlen, gwave, nwaves, hs);
  }
}

// E0 on the panel-blocked copy, for dense levels. Workgroup b owns panels
// b, b + G, ... (2^rb consecutive rows each) and reads every chunk of its
// panel: 256 slice words, one 16-byte load per lane, plus the chunk's
// 512-byte window of frontier words (one 8-byte load per lane); a lane finds
// the frontier word of each of its slices' sets in the window by two wave
// shuffles. A slice hits when its mask meets that word, and the hit row's
// byte in an LDS byte map is set with a plain store (lazy marking is
// idempotent, so no atomic is needed). Loads of the next batch of chunks are
// issued before the current batch is tested. After the panel, the byte map
// minus the visited words gives the panel's new vertices; the workgroup owns
// those rows, so each new vertex is handled once and no visited word is read
// per hit. Either they are written to the mark bytes (32 rows per pair of
// 16-byte stores) for Stage 2, or (fused, new_level >= 0) the workgroup does
// Stage 2 for its rows itself: it updates the visited words, writes every
// next-frontier word of the panel (buffer sel ^ 1), writes the levels and
// stores its Stage 2 partial counters, so the grid needs no separate Stage 2
// sweep and no second barrier for the level.
// pm: LDS scratch of at least 2^rb bytes, left filled with ones (the
// single-workgroup hash set shares it).
constexpr int kPanelChunk = 256;      // slices per chunk (host layout)
constexpr int kPanelUnroll = 8;       // chunks per wave per batch
static_assert(kPanelUnroll <= kPanelBasePad, "batch bases are read past the last chunk");
constexpr int kPanelMaxBytes = 1 << 15;  // LDS byte map of one panel (rb <= 15)
static_assert(kSingleHash * 4 >= kPanelMaxBytes, "the panel byte map lives in the hash-set slots");
constexpr long long kPanelDenom = 8;  // dense: queued slices >= panel slots / 8

__device__ __forceinline__ bool use_panel(const BfsArgs& a, const LevelView& v) {
  if (a.npanels <= 0) return false;
  if (a.panel_mode == 2) return true;
  return v.qslices > kSingleMaxMarks && kPanelDenom * v.qslices >= a.panel_slots;
}

struct PanelPtrs {
  gptr<const uint4> words;    // 64 uint4 per chunk
  gptr<const uint2> front8;   // 8 frontier bytes per element
  cptr<const uint32_t> base;  // first set of each chunk (read-only: scalar loads)
};

// Loads chunk c (clamped to the panel's last chunk `cl`, so every load is in
// bounds; the caller skips chunks past the end): this lane's 4 slice words and
// its 8 bytes of the chunk's frontier window.
__device__ __forceinline__ void panel_load(const PanelPtrs& pp, uint32_t c, uint32_t cl, uint32_t lane, uint32_t b,
                                           uint4& w, uint2& f) {
  w = pp.words[static_cast<size_t>(min(c, cl)) * (kPanelChunk / 4) + lane];
  f = pp.front8[(b >> 3) + lane];
}

// Tests the 4 slices of one lane of one chunk; the frontier byte of a slice's
// set is taken from the lane holding it in the chunk's window.
__device__ __forceinline__ void panel_test4(const uint4& w, uint32_t b7, const uint2& f, uint32_t dmask, int rshift,
                                            lptr<uint32_t> pm) {
  const uint32_t s[4] = {w.x, w.y, w.z, w.w};
  uint32_t d[4], lo[4], hi[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    d[q] = ((s[q] >> 8) & dmask) + b7;
    const int src = static_cast<int>(d[q] >> 3);
    lo[q] = static_cast<uint32_t>(__shfl(static_cast<int>(f.x), src, 64));
    hi[q] = static_cast<uint32_t>(__shfl(static_cast<int>(f.y), src, 64));
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t al = (((d[q] >> 2) & 1u) ? hi[q] : lo[q]) >> (8u * (d[q] & 3u));
    if (s[q] & al & 0xffu) reinterpret_cast<lptr<uint8_t>>(pm)[s[q] >> rshift] = 1;
  }
}

// One batch of kPanelUnroll chunks in registers: each chunk's base set, this
// lane's 4 slice words and its 8 bytes of the chunk's frontier window; bit u
// of `valid` (wave-uniform) is set if chunk u lies in the panel.
struct PanelBatch {
  uint32_t b[kPanelUnroll];
  uint4 w[kPanelUnroll];
  uint2 f[kPanelUnroll];
  uint32_t valid;
};

// Bases of the chunks min(c, cl) .. min(c, cl) + U - 1 by scalar loads (c and
// cl wave-uniform; cl = the panel's last chunk). The base array is padded
// with kPanelBasePad zeros, so these loads stay in bounds and a base read
// past the last chunk is set 0, whose window is in bounds too.
__device__ __forceinline__ void panel_bases(const PanelPtrs& pp, uint32_t c, uint32_t cl,
                                            uint32_t (&x)[kPanelUnroll]) {
  const cptr<const uint32_t> b = pp.base + min(c, cl);
#pragma unroll
  for (int u = 0; u < kPanelUnroll; ++u) x[u] = b[u];
}

// Issues the slice and window loads of the batch starting at chunk c, whose
// bases panel_bases read into x. A chunk past cl loads chunk cl's words
// (in bounds) and is left out of the test by `valid`.
__device__ __forceinline__ void panel_issue(const PanelPtrs& pp, PanelBatch& B, uint32_t c, uint32_t cl,
                                            uint32_t lane, const uint32_t (&x)[kPanelUnroll]) {
  B.valid = c > cl ? 0u : (cl - c >= kPanelUnroll - 1 ? (1u << kPanelUnroll) - 1u : (2u << (cl - c)) - 1u);
#pragma unroll
  for (int u = 0; u < kPanelUnroll; ++u) {
    B.b[u] = x[u];
    panel_load(pp, c + u, cl, lane, x[u], B.w[u], B.f[u]);
  }
}

// Tests the chunks of a batch as straight-line code: a chunk outside the
// panel gets an all-zero frontier window, so it hits nothing. With no branch
// in the test, every path to the next batch's loads has waited for exactly
// this batch's loads and no later ones.
__device__ __forceinline__ void panel_test_batch(const PanelBatch& B, uint32_t dmask, int rshift, lptr<uint32_t> pm) {
#pragma unroll
  for (int u = 0; u < kPanelUnroll; ++u) {
    const bool in = (B.valid >> u) & 1u;
    const uint2 f = make_uint2(in ? B.f[u].x : 0u, in ? B.f[u].y : 0u);
    panel_test4(B.w[u], B.b[u] & 7u, f, dmask, rshift, pm);
  }
}

// Stage 2 for one 32-row group (four slice sets, sigma = 8) whose new
// vertices are x: level writes and the counters of finalize_count. The 33
// row pointers and 5 slice pointers of the group are loaded at once (rp and
// slice_ptr are padded on the device so these loads stay in bounds).
__device__ __forceinline__ void panel_count_group(const BfsArgs& a, long long g, uint32_t x, int new_level,
                                                  long long (&st)[kParts]) {
  const gptr<const int32_t> rp = to_global(a.rp);
  const gptr<const uint32_t> sp = to_global(a.slice_ptr);
  const gptr<int32_t> levels = to_global(a.levels);
  const gptr<const int32_t> orig_id = to_global(a.orig_id);
  const uint32_t tau = static_cast<uint32_t>(a.tau);
  const gptr<const int4> r4 = (gptr<const int4>)(rp + 32 * g);
  int r[33];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int4 q = r4[i];
    r[4 * i + 0] = q.x;
    r[4 * i + 1] = q.y;
    r[4 * i + 2] = q.z;
    r[4 * i + 3] = q.w;
  }
  r[32] = rp[32 * g + 32];
  const uint4 s4 = *(gptr<const uint4>)(sp + 4 * g);
  const uint32_t spt[5] = {s4.x, s4.y, s4.z, s4.w, sp[4 * g + 4]};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t xb = (x >> (8 * k)) & 0xffu;
    if (!xb) continue;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      if (!((xb >> b) & 1u)) continue;
      const long long u = 32 * g + 8 * k + b;
      const int d = r[8 * k + b + 1] - r[8 * k + b];
      st[0] += 1;
      st[2] += d;
      st[3] += d >= 32;
      st[4] += d >= 1024;
      if (d > kLightMax)
        st[6] += (d + kHeavyChunk - 1) / kHeavyChunk;
      else
        st[5] += 1;
      levels[orig_id ? orig_id[u] : u] = new_level;
    }
    const uint32_t ns = spt[k + 1] - spt[k];
    st[1] += ns;
    st[7] += (ns + tau - 1) / tau;
  }
}

template <int BLOCK>
__device__ __attribute__((noinline)) long long engine_panel(const BfsArgs& a, lptr<uint32_t> pm, int sel,
                                                            int new_level) {
  constexpr int U = kPanelUnroll;
  constexpr uint32_t NW = BLOCK / 64;
  constexpr uint32_t STEP = NW * U;
  const int rb = a.panel_rb;
  const int npanels = a.npanels;
  const uint32_t W = 1u << (rb - 5);  // 32-row groups per panel
  const lptr<u32x4> pm16 = reinterpret_cast<lptr<u32x4>>(pm);
  const lptr<const unsigned long long> pm64 = reinterpret_cast<lptr<const unsigned long long>>(pm);
  const uint32_t dmask = (1u << (24 - rb)) - 1u;
  const int rshift = 32 - rb;
  PanelPtrs pp;
  pp.words = to_global(reinterpret_cast<const uint4*>(a.pwords));
  pp.front8 = to_global(static_cast<const uint2*>(front_buf(a, sel)));
  pp.base = to_const_uniform(static_cast<const uint32_t*>(a.pbase));
  const gptr<const uint32_t> pptr = to_global(static_cast<const uint32_t*>(a.pptr));
  const gptr<uint32_t> vis32 = to_global(static_cast<uint32_t*>(a.vis));
  const gptr<uint32_t> next32 = to_global(static_cast<uint32_t*>(front_buf(a, sel ^ 1)));
  const gptr<uint4> mark16 = to_global(reinterpret_cast<uint4*>(a.mark));
  const bool fused = new_level >= 0;
  // fused: the workgroup's Stage 2 counters, summed per panel (kept out of
  // registers during the chunk loop)
  __shared__ unsigned long long s_part[kParts];
  if (threadIdx.x < kParts) s_part[threadIdx.x] = 0ULL;
  const uint32_t lane = static_cast<uint32_t>(lane_id());
  const uint32_t wv = static_cast<uint32_t>(wave_in_block());
  long long work = 0;
  for (int p = blockIdx.x; p < npanels; p += gridDim.x) {
    for (uint32_t j = threadIdx.x; j < 2 * W; j += BLOCK) pm16[j] = u32x4{0u, 0u, 0u, 0u};
    __syncthreads();
    // the chunk range is wave-uniform: scalar registers and scalar branches
    const uint32_t c0 = __builtin_amdgcn_readfirstlane(pptr[p]);
    const uint32_t c1 = __builtin_amdgcn_readfirstlane(pptr[p + 1]);
    const uint32_t cl = c1 - 1;  // used only when the panel has a chunk (c < c1)
    uint32_t c = c0 + __builtin_amdgcn_readfirstlane(wv) * U;
    if (c < c1) {
      // Software pipeline over batches of U chunks in two register sets used
      // in turn: batch k+1 is issued into one set before batch k is tested
      // from the other, so the test waits only for batch k's loads. (A copy
      // from a "next" set into a "current" one would wait for the batch in
      // flight.) The bases of a batch are one vector load, issued a batch
      // ahead and before the slice and window loads it precedes.
      // A counted loop with its exit at the bottom and loads issued
      // unconditionally (past the end they read the clamped last chunk), so
      // the wait before each test is the same on every path: the batch
      // tested has landed while the one issued after it is still in flight.
      // The wave's batches start at c, c + STEP, ...; nb of them hold chunks.
      const uint32_t nb = (c1 - c + STEP - 1) / STEP;
      PanelBatch A, B;
      uint32_t bn[U];
      work += static_cast<long long>(kPanelChunk) * ((nb - 1) * U + min(U, c1 - c - (nb - 1) * STEP));
      // (the scheduling barriers keep each batch's loads together and in
      // this order, so the wait counts below are the same on every path)
      panel_bases(pp, c, cl, bn);
      __builtin_amdgcn_sched_barrier(0);
      panel_issue(pp, A, c, cl, lane, bn);
      panel_bases(pp, c + STEP, cl, bn);
      __builtin_amdgcn_sched_barrier(0);
      panel_issue(pp, B, c + STEP, cl, lane, bn);
      panel_bases(pp, c + 2 * STEP, cl, bn);
      __builtin_amdgcn_sched_barrier(0);
      uint32_t k = 0;
      for (; k + 2 < nb; k += 2) {
        panel_test_batch(A, dmask, rshift, pm);
        __builtin_amdgcn_sched_barrier(0);
        panel_issue(pp, A, c + (k + 2) * STEP, cl, lane, bn);
        panel_bases(pp, c + (k + 3) * STEP, cl, bn);
        __builtin_amdgcn_sched_barrier(0);
        panel_test_batch(B, dmask, rshift, pm);
        __builtin_amdgcn_sched_barrier(0);
        panel_issue(pp, B, c + (k + 3) * STEP, cl, lane, bn);
        panel_bases(pp, c + (k + 4) * STEP, cl, bn);
        __builtin_amdgcn_sched_barrier(0);
      }
      panel_test_batch(A, dmask, rshift, pm);
      if (k + 1 < nb) panel_test_batch(B, dmask, rshift, pm);
    }
    __syncthreads();
    const size_t wb = static_cast<size_t>(p) * W;
    long long st[kParts] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t j = threadIdx.x; j < W; j += BLOCK) {
      const uint32_t m = gather8(pm64[4 * j]) | (gather8(pm64[4 * j + 1]) << 8) | (gather8(pm64[4 * j + 2]) << 16) |
                         (gather8(pm64[4 * j + 3]) << 24);
      if (fused) {
        uint32_t x = 0;
        if (m) {
          const uint32_t old = vis32[wb + j];
          x = m & ~old;
          if (x) vis32[wb + j] = old | x;
        }
        next32[wb + j] = x;
        if (x) panel_count_group(a, static_cast<long long>(wb + j), x, new_level, st);
        continue;
      }
      if (!m) continue;
      const uint32_t x = m & ~vis32[wb + j];
      if (!x) continue;
      uint32_t q[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t nib = (x >> (4 * k)) & 0xfu;
        q[k] = (nib & 1u) | ((nib & 2u) << 7) | ((nib & 4u) << 14) | ((nib & 8u) << 21);
      }
      mark16[2 * (wb + j)] = make_uint4(q[0], q[1], q[2], q[3]);
      mark16[2 * (wb + j) + 1] = make_uint4(q[4], q[5], q[6], q[7]);
    }
    if (fused) {
#pragma unroll
      for (int f = 0; f < kParts; ++f) {
        const long long t = wave_sum(st[f]);
        if (lane == 0 && t)
          __hip_atomic_fetch_add(&s_part[f], static_cast<unsigned long long>(t), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
    __syncthreads();
  }
  for (uint32_t j = threadIdx.x; j < 8 * W; j += BLOCK) pm[j] = 0xffffffffu;
  if (fused) {
    // every workgroup stores its partials (zero if it owns no panel)
    __syncthreads();
    if (threadIdx.x < kParts)
      to_global(a.part)[static_cast<long long>(blockIdx.x) * kParts + threadIdx.x] =
          static_cast<long long>(s_part[threadIdx.x]);
  }
  return lane == 0 ? work : 0;
}

// E1: push over the CSR rows of the frontier vertices.
template <int SIGMA, bool REC>
__device__ __attribute__((noinline)) long long engine_push(const BfsArgs& a, int sel, long long nlight, long long nheavy, long long gtid,
                                 long long nthreads, long long gwave, long long nwaves, lptr<int> hs) {
  long long work = 0;
  using M = typename MaskOf<SIGMA>::T;
  gptr<const M> __restrict__ vis = to_global(static_cast<const M*>(a.vis));
  gptr<const int32_t> __restrict__ rp = to_global(a.rp);
  gptr<const int32_t> __restrict__ col = to_global(a.col);
  gptr<uint8_t> __restrict__ mark = to_global(a.mark);
  const int lane = lane_id();
  gptr<const unsigned long long> __restrict__ heavy = to_global(a.fheavy[sel]);
  for (long long i = gwave; i < nheavy; i += nwaves) {
    const unsigned long long e = heavy[i];
    const int u = static_cast<int>(e >> 32);
    const int b = rp[u] + static_cast<int>(e & 0xffffffffULL);
    const int end = min(rp[u + 1], b + kHeavyChunk);
    for (int p = b + lane; p < end; p += 64) {
      const int v = col[p];
      ++work;
      if (!((vis[v / SIGMA] >> (v % SIGMA)) & 1u)) {
        mark[v] = 1;
        if (REC) record_set(hs, v / SIGMA, a.ctl);
      }
    }
  }
  // Light vertices, 64 per wave step: the wave walks the concatenation of
  // their rows, 64 edges at a time; each lane finds the vertex owning its edge
  // by a binary search over the wave's prefix sums of the degrees, so every
  // lane has an edge (not a vertex's serial chain of loads) in flight.
  gptr<const int32_t> __restrict__ light = to_global(a.flight[sel]);
  (void)gtid;
  (void)nthreads;
  for (long long base = gwave * 64; base < nlight; base += nwaves * 64) {
    const long long i = base + lane;
    int p0 = 0, d = 0;
    if (i < nlight) {
      const int u = light[i];
      p0 = rp[u];
      d = rp[u + 1] - p0;
    }
    const int incl = wave_inclusive_scan(d);
    const int total = __shfl(incl, 63, 64);
    work += lane == 0 ? total : 0;
    for (int e0 = 0; e0 < total; e0 += 64) {
      const int e = e0 + lane;
      int lo = 0;
#pragma unroll
      for (int stp = 32; stp >= 1; stp >>= 1)
        if (__shfl(incl, lo + stp - 1, 64) <= e) lo += stp;
      const int owner = lo & 63;
      const int start = __shfl(incl, owner, 64) - __shfl(d, owner, 64);
      const int op0 = __shfl(p0, owner, 64);
      if (e < total) {
        const int v = col[op0 + (e - start)];
        if (!((vis[v / SIGMA] >> (v % SIGMA)) & 1u)) {
          mark[v] = 1;
          if (REC) record_set(hs, v / SIGMA, a.ctl);
        }
      }
    }
  }
  return work;
}

// E2: bottom-up (Alg. 4). A lane owns one vertex; an unvisited vertex of
// degree <= kPullLight scans its row alone and stops at the first frontier
// neighbour. Longer rows are scanned by the whole wave, 64 neighbours per
// step, stopping at the first step that finds one.
constexpr int kPullLight = 32;

template <int SIGMA>
__device__ __attribute__((noinline)) long long engine_pull(const BfsArgs& a, int sel, long long gtid,
                                                           long long nthreads) {
  long long work = 0;
  using M = typename MaskOf<SIGMA>::T;
  gptr<const M> __restrict__ vis = to_global(static_cast<const M*>(a.vis));
  gptr<const M> __restrict__ front = to_global(static_cast<const M*>(front_buf(a, sel)));
  gptr<const M> __restrict__ degm = to_global(static_cast<const M*>(a.degmask_in));
  gptr<const int32_t> __restrict__ rp = to_global(a.rp_in);
  gptr<const int32_t> __restrict__ col = to_global(a.col_in);
  gptr<uint8_t> __restrict__ mark = to_global(a.mark);
  const long long nv = a.nsets * SIGMA;
  const int lane = lane_id();
  // 64-vertex chunks: round k gives the waves chunks k*nw .. k*nw + nw - 1,
  // rotated by k, so chunks with heavy rows that recur with a fixed stride
  // (a relabelling that puts each window's hubs first) spread over all waves
  const long long nw = nthreads / 64, gw = (gtid - lane) / 64;
  const long long nchunks = (nv + 63) / 64;
  for (long long k = 0; k * nw < nchunks; ++k) {
    const long long chunk = k * nw + (gw + k) % nw;
    if (chunk >= nchunks) continue;
    const long long ubase = chunk * 64;
    const long long u = ubase + lane;
    bool cand = false;
    int p = 0, e = 0;
    if (u < nv) {
      const long long s = u / SIGMA;
      const M unv = static_cast<M>(~vis[s] & degm[s]);
      cand = (unv >> (u % SIGMA)) & 1u;
    }
    if (cand) {
      p = rp[u];
      e = rp[u + 1];
    }
    const bool heavy = cand && (e - p > kPullLight);
    if (cand && !heavy) {
      // four independent neighbour loads per step shorten the dependent chain
      const int p0 = p;
      bool found = false;
      for (; p < e && !found; p += 4) {
        // one 16-byte load of 4 neighbours (col is padded by 4 entries, so
        // the load stays in bounds at the end of the array)
        int q[4];
        __builtin_memcpy(q, reinterpret_cast<const int32_t*>(col + p), sizeof(q));
        const int v0 = q[0];
        const int v1 = p + 1 < e ? q[1] : v0;
        const int v2 = p + 2 < e ? q[2] : v0;
        const int v3 = p + 3 < e ? q[3] : v0;
        found = ((front[v0 / SIGMA] >> (v0 % SIGMA)) & 1u) | ((front[v1 / SIGMA] >> (v1 % SIGMA)) & 1u) |
                ((front[v2 / SIGMA] >> (v2 % SIGMA)) & 1u) | ((front[v3 / SIGMA] >> (v3 % SIGMA)) & 1u);
      }
      if (found) mark[u] = 1;
      work += min(p, e) - p0;
    }
    unsigned long long hb = __ballot(heavy);
    while (hb) {
      const int l = __builtin_ctzll(hb);
      hb &= hb - 1;
      const int hp = __builtin_amdgcn_readlane(p, l), he = __builtin_amdgcn_readlane(e, l);
      for (int qq = hp; qq < he; qq += 64) {
        const int i = qq + lane;
        bool f = false;
        if (i < he) {
          const int v = col[i];
          f = (front[v / SIGMA] >> (v % SIGMA)) & 1u;
          ++work;
        }
        if (__ballot(f)) {
          if (lane == 0) mark[ubase + l] = 1;
          break;
        }
      }
    }
  }
  return work;
}

// Runs one engine and adds the adjacency entries it read to the level's
// F_WORK counter (one atomic per block).
// hs != nullptr: single-workgroup level, marked slice sets are recorded in hs
// (only the BVSS and push engines run there). pm: LDS scratch for the
// panel-blocked BVSS step (nullptr: that step is not available).
// fuse_level >= 0: a panel step also does Stage 2 for that new level.
template <int SIGMA, class SliceT, int BLOCK>
__device__ __forceinline__ void run_engine(const BfsArgs& a, int engine, int sel, int slot, const LevelView& v,
                                           long long gtid, long long nthreads, long long gwave, long long nwaves,
                                           lptr<int> hs, lptr<uint32_t> pm, int fuse_level = -1) {
  __shared__ long long lds_work[BLOCK / 64];
  long long work[1];
  constexpr bool kPanelFmt = SIGMA == 8 && sizeof(SliceT) == 4;
  if (kPanelFmt && engine == BLEST_ENGINE_BVSS && !hs && pm && use_panel(a, v))
    work[0] = engine_panel<BLOCK>(a, pm, sel, fuse_level);
  else if (engine == BLEST_ENGINE_BVSS)
    work[0] = hs ? engine_bvss<SIGMA, SliceT, true>(a, a.queue[sel], v.queue, gwave, nwaves, hs)
                 : engine_bvss<SIGMA, SliceT, false>(a, a.queue[sel], v.queue, gwave, nwaves, nullptr);
  else if (engine == BLEST_ENGINE_PUSH)
    work[0] = hs ? engine_push<SIGMA, true>(a, sel, v.light, v.heavy, gtid, nthreads, gwave, nwaves, hs)
                 : engine_push<SIGMA, false>(a, sel, v.light, v.heavy, gtid, nthreads, gwave, nwaves, nullptr);
  else
    work[0] = engine_pull<SIGMA>(a, sel, gtid, nthreads);
  if (a.count_work || a.probe) {
    block_sum64<BLOCK, 1>(work, lds_work);
    if (threadIdx.x == 0 && work[0]) add_u64(&a.ctl->acc[slot][F_WORK][0], static_cast<unsigned long long>(work[0]));
  }
}

// ------------------------------------------------------------ Stage 2




// Stage 2 over windows of 2*BLOCK slice sets; set_at(win, k) gives the set
// handled by this thread in slot k of window win, or -1. MODE:
//  FIN_ATOMIC  marks -> visited/frontier/levels, and the lists, with output
//              space reserved per window by one device atomic per list;
//  FIN_LOCAL   the same with the block-local cursors `local` (one workgroup
//              alone: no atomics; the caller stores the totals);
//  FIN_COUNT   marks -> visited/frontier/levels and counts only: every set's
//              frontier word is rewritten (0 if it gained nothing) and the
//              list sizes are added to st[5..7]; no list is written;
//  FIN_EMIT    no state change: the frontier words written by FIN_COUNT give
//              the new vertices, and the lists asked for (want_push,
//              want_queue) are written from the cursors `local`, which the
//              caller presets to this block's offsets.
// st[] accumulates frontier, queued slices, frontier edges, degree >= 32,
// degree >= 1024 and (FIN_COUNT) light, heavy and queue entries. Queue
// descriptors and heavy edge chunks are written wave-cooperatively: each lane
// finds the run that owns its output index by a binary search over the wave's
// prefix sums, so a hub set with thousands of VSSs costs a few wave steps.
enum FinMode : int { FIN_ATOMIC = 0, FIN_LOCAL = 1, FIN_COUNT = 2, FIN_EMIT = 3 };

// Slice sets per thread in one window of the Stage 2 sweep (a window is
// BLOCK * kFinSpt consecutive sets); their loads are issued together.
constexpr int kFinSpt = 4;

template <int SIGMA, int BLOCK, int MODE, class SetAt>
__device__ void finalize_windows(const BfsArgs& a, int new_level, gptr<unsigned long long> acc, int sel_out,
                                 long long win0, long long nwin, long long wstep, SetAt set_at, long long (&st)[8],
                                 unsigned long long* local, bool want_push = true, bool want_queue = true) {
  using M = typename MaskOf<SIGMA>::T;
  constexpr int SPT = kFinSpt;
  constexpr bool UPDATE = MODE != FIN_EMIT;
  __shared__ int lds32[3 * (BLOCK / 64)];
  __shared__ unsigned long long bases[3];
  gptr<M> __restrict__ vis = to_global(static_cast<M*>(a.vis));
  gptr<M> __restrict__ front = to_global(static_cast<M*>(front_buf(a, sel_out)));
  gptr<uint8_t> __restrict__ mark = to_global(a.mark);
  gptr<const int32_t> __restrict__ rp = to_global(a.rp);
  gptr<const uint32_t> __restrict__ sp = to_global(a.slice_ptr);
  const uint32_t tau = static_cast<uint32_t>(a.tau);
  gptr<int32_t> __restrict__ light = to_global(a.flight[sel_out]);
  gptr<unsigned long long> __restrict__ heavy = to_global(a.fheavy[sel_out]);
  gptr<uint4> __restrict__ queue = to_global(a.queue[sel_out]);
  gptr<int32_t> __restrict__ levels = to_global(a.levels);
  const gptr<const int32_t> __restrict__ orig_id = to_global(a.orig_id);
  const int lane = lane_id();
  const bool need_rp = UPDATE || want_push;
  const bool need_sp = UPDATE || want_queue;
  for (long long win = win0; win < nwin; win += wstep) {
    // The SPT sets of a thread are finalised in phases, each issuing the
    // loads of all SPT sets before any is used (marks; visited words; row and
    // slice pointers; input ids), so a window costs four dependent memory
    // round trips rather than four per set.
    M nw[SPT];
    long long sset[SPT];
    int nl[SPT], nh[SPT], nq[SPT];
    M got[SPT];
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
      const long long s = set_at(win, k);
      sset[k] = s;
      nw[k] = 0;
      nl[k] = nh[k] = nq[k] = 0;
      got[k] = 0;
      if (s >= 0) {
        if constexpr (UPDATE)
          got[k] = load_marks<SIGMA>(mark + s * SIGMA);
        else
          got[k] = front[s];
      }
    }
    if constexpr (UPDATE) {
      M old[SPT];
#pragma unroll
      for (int k = 0; k < SPT; ++k) old[k] = got[k] ? vis[sset[k]] : M(0);
#pragma unroll
      for (int k = 0; k < SPT; ++k) {
        const long long s = sset[k];
        if (s < 0) continue;
        const M x = static_cast<M>(got[k] & ~old[k]);
        if (got[k]) clear_marks<SIGMA>(mark + s * SIGMA);
        if (x) vis[s] = static_cast<M>(old[k] | x);
        if (MODE == FIN_COUNT)
          front[s] = x;
        else if (x)
          front[s] = x;
        nw[k] = x;
      }
    } else {
#pragma unroll
      for (int k = 0; k < SPT; ++k) nw[k] = got[k];
    }
    uint32_t p0[SPT], p1[SPT];
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
      p0[k] = p1[k] = 0;
      if (nw[k] && need_sp) {
        p0[k] = sp[sset[k]];
        p1[k] = sp[sset[k] + 1];
      }
    }
    if constexpr (SIGMA == 8) {
      // eight vertices per set: every set's row pointers and input ids fit
      // in registers at once
      int r[SPT][SIGMA + 1];
#pragma unroll
      for (int k = 0; k < SPT; ++k)
        if (nw[k] && need_rp) load_set_rp<SIGMA>(rp, sset[k], r[k]);
      if constexpr (UPDATE) {
        int32_t id[SPT][SIGMA];
#pragma unroll
        for (int k = 0; k < SPT; ++k)
#pragma unroll
          for (int b = 0; b < SIGMA; ++b) {
            const long long u = sset[k] * SIGMA + b;
            id[k][b] = ((nw[k] >> b) & 1u) ? (orig_id ? orig_id[u] : static_cast<int32_t>(u)) : 0;
          }
#pragma unroll
        for (int k = 0; k < SPT; ++k)
#pragma unroll
          for (int b = 0; b < SIGMA; ++b)
            if ((nw[k] >> b) & 1u) levels[id[k][b]] = new_level;
      }
#pragma unroll
      for (int k = 0; k < SPT; ++k) {
        if (!nw[k] || !need_rp) continue;
#pragma unroll
        for (int b = 0; b < SIGMA; ++b) {
          if (!((nw[k] >> b) & 1u)) continue;
          const int d = r[k][b + 1] - r[k][b];
          if constexpr (UPDATE) {
            st[0] += 1;
            st[2] += d;
            st[3] += d >= 32;
            st[4] += d >= 1024;
          }
          if (d > kLightMax)
            nh[k] += (d + kHeavyChunk - 1) / kHeavyChunk;
          else
            nl[k] += 1;
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < SPT; ++k) {
        const M x = nw[k];
        if (!x || !need_rp) continue;
        const long long s = sset[k];
        int r[SIGMA + 1];
        load_set_rp<SIGMA>(rp, s, r);
#pragma unroll
        for (int b = 0; b < SIGMA; ++b) {
          if (!((x >> b) & 1u)) continue;
          const long long u = s * SIGMA + b;
          const int d = r[b + 1] - r[b];
          if constexpr (UPDATE) {
            st[0] += 1;
            st[2] += d;
            st[3] += d >= 32;
            st[4] += d >= 1024;
            levels[orig_id ? orig_id[u] : u] = new_level;
          }
          if (d > kLightMax)
            nh[k] += (d + kHeavyChunk - 1) / kHeavyChunk;
          else
            nl[k] += 1;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
      if (nw[k] && need_sp) {
        const uint32_t ns = p1[k] - p0[k];
        nq[k] = static_cast<int>((ns + tau - 1) / tau);
        if constexpr (UPDATE) st[1] += ns;
      }
      if (MODE == FIN_EMIT && !want_push) nl[k] = nh[k] = 0;
    }
    if constexpr (UPDATE) {
#pragma unroll
      for (int k = 0; k < SPT; ++k) {
        st[5] += nl[k];
        st[6] += nh[k];
        st[7] += nq[k];
      }
    }
    if constexpr (MODE == FIN_COUNT) continue;
    int cnt[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
      cnt[0] += nl[k];
      cnt[1] += nh[k];
      cnt[2] += nq[k];
    }
    if (!__syncthreads_or(cnt[0] | cnt[1] | cnt[2])) continue;
    int ex[3], tot[3];
    block_exclusive_scan<BLOCK, 3>(cnt, ex, tot, lds32);
    if (threadIdx.x == 0) {
      if (MODE != FIN_ATOMIC) {
        for (int f = 0; f < 3; ++f) {
          bases[f] = local[f];
          local[f] += tot[f];
        }
      } else {
        bases[0] = tot[0] ? fetch_add_u64(acc + F_LIGHT * kPad, tot[0]) : 0ULL;
        bases[1] = tot[1] ? fetch_add_u64(acc + F_HEAVY * kPad, tot[1]) : 0ULL;
        bases[2] = tot[2] ? fetch_add_u64(acc + F_QUEUE * kPad, tot[2]) : 0ULL;
      }
    }
    __syncthreads();
    // light vertices: the owning lane writes its (at most SIGMA) entries
    long long ol = static_cast<long long>(bases[0]) + ex[0];
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
      if (!nl[k]) continue;
      int r[SIGMA + 1];
      load_set_rp<SIGMA>(rp, sset[k], r);
#pragma unroll
      for (int b = 0; b < SIGMA; ++b)
        if (((nw[k] >> b) & 1u) && r[b + 1] - r[b] <= kLightMax) light[ol++] = static_cast<int32_t>(sset[k] * SIGMA + b);
    }
    // queue descriptors and heavy chunks: wave-cooperative expansion
    long long oq = static_cast<long long>(bases[2]) + ex[2];
    long long oh = static_cast<long long>(bases[1]) + ex[1];
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
      const uint32_t s0 = nq[k] ? sp[sset[k]] : 0u;
      const uint32_t ns = nq[k] ? sp[sset[k] + 1] - s0 : 0u;
      {  // VSS descriptors of this lane's set k
        const int incl = wave_inclusive_scan(nq[k]);
        const int total = __shfl(incl, 63, 64);
        for (int b0 = 0; b0 < total; b0 += 64) {
          const int i = b0 + lane;
          int lo = 0;
#pragma unroll
          for (int stp = 32; stp >= 1; stp >>= 1)
            if (__shfl(incl, lo + stp - 1, 64) <= i) lo += stp;
          const int owner = lo & 63;
          const int start = __shfl(incl, owner, 64) - __shfl(nq[k], owner, 64);
          const long long o = __shfl(oq, owner, 64);
          const uint32_t os0 = __shfl(s0, owner, 64), ons = __shfl(ns, owner, 64);
          const uint32_t obits = __shfl(static_cast<uint32_t>(nw[k]), owner, 64);
          const long long os = __shfl(sset[k], owner, 64);
          if (i < total) {
            const uint32_t j = static_cast<uint32_t>(i - start), off = j * tau;
            queue[o + j] = make_uint4(os0 + off, min(tau, ons - off), obits, static_cast<uint32_t>(os));
          }
        }
        oq += nq[k];
      }
      {  // heavy edge chunks of this lane's set k
        const int incl = wave_inclusive_scan(nh[k]);
        const int total = __shfl(incl, 63, 64);
        for (int b0 = 0; b0 < total; b0 += 64) {
          const int i = b0 + lane;
          int lo = 0;
#pragma unroll
          for (int stp = 32; stp >= 1; stp >>= 1)
            if (__shfl(incl, lo + stp - 1, 64) <= i) lo += stp;
          const int owner = lo & 63;
          const int start = __shfl(incl, owner, 64) - __shfl(nh[k], owner, 64);
          const long long o = __shfl(oh, owner, 64);
          const uint32_t obits = __shfl(static_cast<uint32_t>(nw[k]), owner, 64);
          const long long os = __shfl(sset[k], owner, 64);
          if (i < total) {
            int j = i - start;
            int r[SIGMA + 1];
            load_set_rp<SIGMA>(rp, os, r);
#pragma unroll
            for (int b = 0; b < SIGMA; ++b) {
              const int d = r[b + 1] - r[b];
              if (!((obits >> b) & 1u) || d <= kLightMax || j < 0) continue;
              const int nch = (d + kHeavyChunk - 1) / kHeavyChunk;
              if (j < nch)
                heavy[o + (i - start)] = (static_cast<unsigned long long>(os * SIGMA + b) << 32) |
                                         static_cast<unsigned long long>(j * kHeavyChunk);
              j -= nch;
            }
          }
        }
        oh += nh[k];
      }
    }
    __syncthreads();
  }
}

// Adds a block's Stage 2 statistics to the level slot (block 0 also carries
// the cumulative counts of the previous level).
template <int BLOCK>
__device__ void finalize_stats(gptr<unsigned long long> acc, const long long (&st8)[8], long long cumv_in,
                               long long cume_in) {
  __shared__ long long lds64[5 * (BLOCK / 64)];
  long long st[5] = {st8[0], st8[1], st8[2], st8[3], st8[4]};
  block_sum64<BLOCK, 5>(st, lds64);
  if (threadIdx.x == 0) {
    if (st[0]) {
      add_u64(acc + F_FRONTIER * kPad, st[0]);
      add_u64(acc + F_CUMV * kPad, st[0]);
    }
    if (st[1]) add_u64(acc + F_QSLICES * kPad, st[1]);
    if (st[2]) {
      add_u64(acc + F_FEDGES * kPad, st[2]);
      add_u64(acc + F_CUME * kPad, st[2]);
    }
    if (st[3]) add_u64(acc + F_DEG32 * kPad, st[3]);
    if (st[4]) add_u64(acc + F_DEG1024 * kPad, st[4]);
    if (blockIdx.x == 0) {
      add_u64(acc + F_CUMV * kPad, cumv_in);
      add_u64(acc + F_CUME * kPad, cume_in);
    }
  }
}

// Stage 2 of the whole grid: every slice set, windows spread over the blocks.
template <int SIGMA, int BLOCK>
__device__ void finalize(const BfsArgs& a, int new_level, int slot_out, int sel_out, long long cumv_in,
                         long long cume_in, unsigned nblocks) {
  constexpr long long WIN = static_cast<long long>(BLOCK) * kFinSpt;
  const gptr<unsigned long long> acc = to_global(&a.ctl->acc[slot_out][0][0]);
  long long st[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // frontier, queued slices, frontier edges, deg>=32, deg>=1024
  const long long nsets = a.nsets;
  const long long tid = threadIdx.x;
  finalize_windows<SIGMA, BLOCK, FIN_ATOMIC>(a, new_level, acc, sel_out, blockIdx.x, (nsets + WIN - 1) / WIN, nblocks,
                                        [=](long long win, int k) -> long long {
                                          const long long s = win * WIN + k * BLOCK + tid;
                                          return s < nsets ? s : -1;
                                        },
                                        st, nullptr);
  finalize_stats<BLOCK>(acc, st, cumv_in, cume_in);
}

// ------------------------------------------------- two-phase grid Stage 2
//
// In the persistent kernel a grid level's Stage 2 runs in two phases with no
// device atomics. Count: every workgroup sweeps its windows (marks ->
// visited/frontier/levels) and stores its partial counters with plain stores.
// After the barrier every workgroup sums the partials in the same order, so
// all of them hold the same level statistics and pick the same engine for
// the next level, and each knows the sum of the list sizes of the workgroups
// before it. Emit: only when that engine reads a list (the VSS queue for BVSS
// over the queue, the vertex lists for push; all lists in probe mode) do the
// workgroups sweep again and write it at those offsets, behind one more
// barrier. Bottom-up and panel levels skip the emit phase.

// MODE = FIN_COUNT (counts only) or FIN_ATOMIC (lists too, output space
// reserved with one device atomic per window and list on the cursors of
// slot `slot_out`); either way the level statistics go to the partials.
template <int SIGMA, int BLOCK, int MODE>
__device__ void finalize_count(const BfsArgs& a, int new_level, int slot_out, int sel_out) {
  constexpr long long WIN = static_cast<long long>(BLOCK) * kFinSpt;
  __shared__ long long lds64[kParts * (BLOCK / 64)];
  long long st[kParts] = {0, 0, 0, 0, 0, 0, 0, 0};
  const long long nsets = a.nsets;
  const long long tid = threadIdx.x;
  finalize_windows<SIGMA, BLOCK, MODE>(a, new_level, to_global(&a.ctl->acc[slot_out][0][0]), sel_out, blockIdx.x,
                                            (nsets + WIN - 1) / WIN, gridDim.x,
                                            [=](long long win, int k) -> long long {
                                              const long long s = win * WIN + k * BLOCK + tid;
                                              return s < nsets ? s : -1;
                                            },
                                            st, nullptr);
  block_sum64<BLOCK, kParts>(st, lds64);
  const gptr<long long> part = to_global(a.part);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int f = 0; f < kParts; ++f) part[static_cast<long long>(blockIdx.x) * kParts + f] = st[f];
  }
}

// Sums the partial counters of all workgroups (after the barrier that follows
// finalize_count). before[] = light, heavy and queue entries of the
// workgroups with a smaller index (this workgroup's list offsets).
template <int BLOCK>
__device__ void reduce_parts(const BfsArgs& a, long long (&tot)[kParts], long long (&before)[3]) {
  __shared__ long long s_tot[kParts], s_bef[3];
  const gptr<const long long> part = to_global(static_cast<const long long*>(a.part));
  const int nb = static_cast<int>(gridDim.x);
  const int me = static_cast<int>(blockIdx.x);
  const int lane = lane_id(), w = wave_in_block();
  for (int f = w; f < kParts; f += BLOCK / 64) {
    long long t = 0, bs = 0;
    for (int b = lane; b < nb; b += 64) {
      const long long x = part[static_cast<long long>(b) * kParts + f];
      t += x;
      bs += b < me ? x : 0;
    }
    t = wave_sum(t);
    bs = wave_sum(bs);
    if (lane == 0) {
      s_tot[f] = t;
      if (f >= 5) s_bef[f - 5] = bs;
    }
  }
  __syncthreads();
#pragma unroll
  for (int f = 0; f < kParts; ++f) tot[f] = s_tot[f];
#pragma unroll
  for (int f = 0; f < 3; ++f) before[f] = s_bef[f];
  __syncthreads();
}

// panel_part: the counts came from the fused panel step, so each workgroup
// emits the lists of the slice sets of its own panels (the partition its
// partial counters, and hence its offsets, were computed over); otherwise
// the window partition of finalize_count.
template <int SIGMA, int BLOCK>
__device__ void finalize_emit(const BfsArgs& a, int sel_out, const long long (&before)[3], bool want_push,
                              bool want_queue, bool panel_part) {
  constexpr long long WIN = static_cast<long long>(BLOCK) * kFinSpt;
  __shared__ unsigned long long cursor[3];
  if (threadIdx.x < 3) cursor[threadIdx.x] = static_cast<unsigned long long>(before[threadIdx.x]);
  __syncthreads();
  long long st[kParts] = {0, 0, 0, 0, 0, 0, 0, 0};
  const long long nsets = a.nsets;
  const long long tid = threadIdx.x;
  const gptr<unsigned long long> acc0 = to_global(&a.ctl->acc[0][0][0]);
  if (panel_part) {
    // panel p holds sets [p * sp, (p + 1) * sp); this workgroup owns panels
    // blockIdx.x, blockIdx.x + G, ...; window w is window w % wpp of its
    // (w / wpp)-th panel
    const long long sp = 1LL << (a.panel_rb - 3);
    const long long wpp = (sp + WIN - 1) / WIN;
    const long long mine = a.npanels > static_cast<int>(blockIdx.x)
                               ? (a.npanels - 1 - static_cast<long long>(blockIdx.x)) / gridDim.x + 1
                               : 0;
    const long long b = blockIdx.x, G = gridDim.x;
    finalize_windows<SIGMA, BLOCK, FIN_EMIT>(a, 0, acc0, sel_out, 0, mine * wpp, 1,
                                             [=](long long win, int k) -> long long {
                                               const long long p = b + (win / wpp) * G;
                                               const long long end = min((p + 1) * sp, nsets);
                                               const long long s = p * sp + (win % wpp) * WIN + k * BLOCK + tid;
                                               return s < end ? s : -1;
                                             },
                                             st, cursor, want_push, want_queue);
    return;
  }
  finalize_windows<SIGMA, BLOCK, FIN_EMIT>(a, 0, acc0, sel_out, blockIdx.x, (nsets + WIN - 1) / WIN, gridDim.x,
                                           [=](long long win, int k) -> long long {
                                             const long long s = win * WIN + k * BLOCK + tid;
                                             return s < nsets ? s : -1;
                                           },
                                           st, cursor, want_push, want_queue);
}

// ------------------------------------------------- single-workgroup levels
//
// A level whose Stage 1 can mark at most kSingleMaxMarks rows (BVSS: queued
// slices; push: frontier edges) is run by workgroup 0 alone: the engine
// records every slice set it marks in an LDS hash set, and Stage 2 finalises
// only those sets, with workgroup barriers instead of device-wide ones. The
// other workgroups wait on a flag until workgroup 0 reaches a level that is
// not small (or the end), then all continue together.

__device__ __forceinline__ bool single_eligible(const BfsArgs& a, int engine, const LevelView& v) {
  if (!a.single_block || a.probe) return false;
  if (engine == BLEST_ENGINE_BVSS) return v.qslices <= kSingleMaxMarks && !(a.npanels > 0 && a.panel_mode == 2);
  if (engine == BLEST_ENGINE_PUSH) return v.fedges <= kSingleMaxMarks;
  return false;
}

// Stage 2 of one workgroup over the sets recorded during Stage 1 (the LDS
// list after the hash set); empties both. Output cursors are block-local and
// the level's counters are stored at the end (the slot was zeroed before).
template <int SIGMA, int BLOCK>
__device__ void finalize_list(const BfsArgs& a, int new_level, int slot_out, int sel_out, long long cumv_in,
                              long long cume_in, lptr<int> hs) {
  constexpr int WIN = BLOCK * kFinSpt;
  __shared__ unsigned long long local[3];
  __shared__ long long lds64[5 * (BLOCK / 64)];
  const gptr<unsigned long long> acc = to_global(&a.ctl->acc[slot_out][0][0]);
  if (threadIdx.x < 3) local[threadIdx.x] = 0ULL;
  __syncthreads();
  const int count = hs[kSingleHash];
  const lptr<const int> list = hs + kSingleHash + 1;
  long long st8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int tid = threadIdx.x;
  finalize_windows<SIGMA, BLOCK, FIN_LOCAL>(a, new_level, acc, sel_out, 0, (count + WIN - 1) / WIN, 1,
                                       [=](long long win, int k) -> long long {
                                         const long long i = win * WIN + k * BLOCK + tid;
                                         return i < count ? static_cast<long long>(list[i]) : -1;
                                       },
                                       st8, local);
  __syncthreads();
  for (int i = tid; i < kSingleHash + 1; i += BLOCK) hs[i] = (i == kSingleHash) ? 0 : -1;
  long long st[5] = {st8[0], st8[1], st8[2], st8[3], st8[4]};
  block_sum64<BLOCK, 5>(st, lds64);
  if (threadIdx.x == 0) {
    auto put = [&](int f, unsigned long long v) {
      __hip_atomic_store(acc + f * kPad, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    put(F_LIGHT, local[0]);
    put(F_HEAVY, local[1]);
    put(F_QUEUE, local[2]);
    put(F_FRONTIER, static_cast<unsigned long long>(st[0]));
    put(F_QSLICES, static_cast<unsigned long long>(st[1]));
    put(F_FEDGES, static_cast<unsigned long long>(st[2]));
    put(F_DEG32, static_cast<unsigned long long>(st[3]));
    put(F_DEG1024, static_cast<unsigned long long>(st[4]));
    put(F_CUMV, static_cast<unsigned long long>(cumv_in + st[0]));
    put(F_CUME, static_cast<unsigned long long>(cume_in + st[2]));
  }
}

// ------------------------------------------------------- init and seeding

template <int SIGMA>
// seeded: the threads that clear the source's visited/frontier word and
// level write the source's values instead (level 0), so no barrier is needed
// between the clear and those writes.
__device__ __forceinline__ void clear_state(const BfsArgs& a, long long gtid, long long nthreads, bool seeded = false) {
  using M = typename MaskOf<SIGMA>::T;
  M* vis = static_cast<M*>(a.vis);
  M* front0 = static_cast<M*>(front_buf(a, 0));
  M* front1 = static_cast<M*>(front_buf(a, 1));
  const long long src_set = seeded ? a.src / SIGMA : -1;
  const M src_bit = static_cast<M>(M(1) << (a.src % SIGMA));
  const long long src_in = seeded ? (a.orig_id ? a.orig_id[a.src] : a.src) : -1;
  for (long long i = gtid; i < a.n; i += nthreads) a.levels[i] = i == src_in ? 0 : -1;
  for (long long s = gtid; s < a.nsets; s += nthreads) {
    vis[s] = s == src_set ? src_bit : M(0);
    front0[s] = s == src_set ? src_bit : M(0);
    front1[s] = 0;
  }
  if (blockIdx.x == 0)
    for (int t = threadIdx.x; t < kStatSlots * kStatFields; t += blockDim.x)
      a.ctl->acc[t / kStatFields][t % kStatFields][0] = 0ULL;
}

// Level 0: frontier = {src}, queue = the VSSs of src's slice set. One block.
template <int SIGMA>
// lists_only: clear_state(seeded) already wrote the visited/frontier bit and level.
__device__ __forceinline__ void seed_source(const BfsArgs& a, bool lists_only = false) {
  using M = typename MaskOf<SIGMA>::T;
  const long long src = a.src;
  const long long s = src / SIGMA;
  const M bit = static_cast<M>(M(1) << (src % SIGMA));
  const uint32_t s0 = a.slice_ptr[s], ns = a.slice_ptr[s + 1] - s0;
  const uint32_t tau = static_cast<uint32_t>(a.tau);
  const uint32_t nq = (ns + tau - 1) / tau;
  const int d = a.rp[src + 1] - a.rp[src];
  for (uint32_t k = threadIdx.x; k < nq; k += blockDim.x)
    a.queue[0][k] = make_uint4(s0 + k * tau, min(tau, ns - k * tau), static_cast<uint32_t>(bit), static_cast<uint32_t>(s));
  const int nh = d > kLightMax ? (d + kHeavyChunk - 1) / kHeavyChunk : 0;
  for (int c = threadIdx.x; c < nh; c += blockDim.x)
    a.fheavy[0][c] = (static_cast<unsigned long long>(src) << 32) | static_cast<unsigned long long>(c * kHeavyChunk);
  if (threadIdx.x == 0) {
    if (!lists_only) {
      static_cast<M*>(a.vis)[s] = bit;
      static_cast<M*>(front_buf(a, 0))[s] = bit;
      a.levels[a.orig_id ? a.orig_id[src] : src] = 0;
    }
    if (nh == 0) a.flight[0][0] = static_cast<int32_t>(src);
    unsigned long long* acc = &a.ctl->acc[0][0][0];
    acc[F_FRONTIER * kPad] = 1;
    acc[F_QUEUE * kPad] = nq;
    acc[F_QSLICES * kPad] = ns;
    acc[F_FEDGES * kPad] = static_cast<unsigned long long>(d);
    acc[F_DEG32 * kPad] = d >= 32;
    acc[F_DEG1024 * kPad] = d >= 1024;
    acc[F_LIGHT * kPad] = nh == 0 ? 1 : 0;
    acc[F_HEAVY * kPad] = static_cast<unsigned long long>(nh);
    acc[F_CUMV * kPad] = 1;
    acc[F_CUME * kPad] = static_cast<unsigned long long>(d);
  }
}

__device__ __forceinline__ void log_level(const BfsArgs& a, int level, const LevelView& v, int engine, int fallback,
                                          const float (&feat)[kMaxSwitchFeatures]) {
  if (level >= a.log_cap) return;
  LevelRec& r = a.log[level];
  r.frontier = v.frontier;
  r.queue = v.queue;
  r.qslices = v.qslices;
  r.fedges = v.fedges;
  r.unvisited = a.n - v.cumv;
  r.unvisited_edges = a.m - v.cume;
  r.deg32 = v.deg32;
  r.deg1024 = v.deg1024;
  r.engine = engine;
  r.fallback = fallback;
  r.panel = engine == BLEST_ENGINE_BVSS && use_panel(a, v);
  r.t_begin = dev_ticks();
  r.t_mid = 0;
  r.t_end = 0;
  r.t_count = 0;
  r.t_engine[0] = r.t_engine[1] = r.t_engine[2] = 0;
  r.work = 0;
#pragma unroll
  for (int k = 0; k < kMaxSwitchFeatures; ++k) r.feat[k] = feat[k];
}

// ------------------------------------------------------ persistent kernel

// Waits until every wave of the block has its memory operations performed,
// then synchronises the block.
__device__ __forceinline__ void block_sync_mem() {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

// Workgroup 0 runs consecutive small levels alone, starting at `level` with
// its view, chosen engine and features. Returns the first level it did not
// run (its slot holds that level's statistics).
template <int SIGMA, class SliceT, int BLOCK>
__device__ int single_episode(const BfsArgs& a, int level, int engine, int fallback, float (&feat)[kMaxSwitchFeatures],
                              LevelView v, const float* s_mlp, lptr<int> hs) {
  const long long gtid = threadIdx.x, nthreads = BLOCK;
  const long long gwave = wave_in_block(), nwaves = BLOCK / 64;
  for (;;) {
    const int slot = level % kStatSlots, nslot = (level + 1) % kStatSlots;
    if (threadIdx.x == 0) log_level(a, level, v, engine, fallback, feat);
    if (threadIdx.x < kStatFields)
      __hip_atomic_store(&a.ctl->acc[nslot][threadIdx.x][0], 0ULL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    block_sync_mem();
    run_engine<SIGMA, SliceT, BLOCK>(a, engine, level & 1, slot, v, gtid, nthreads, gwave, nwaves, hs, nullptr);
    block_sync_mem();
    if (threadIdx.x == 0 && level < a.log_cap) a.log[level].t_mid = dev_ticks();
    finalize_list<SIGMA, BLOCK>(a, level + 1, nslot, (level & 1) ^ 1, v.cumv, v.cume, hs);
    block_sync_mem();
    if (threadIdx.x == 0 && level < a.log_cap) {
      a.log[level].t_end = dev_ticks();
      a.log[level].work = static_cast<long long>(ld_relaxed_u64(&a.ctl->acc[slot][F_WORK][0]));
    }
    const long long prev = v.frontier;
    ++level;
    // progress for the waiting workgroups: their time bound restarts with every level
    if (threadIdx.x == 0)
      __hip_atomic_store(&a.ctl->single_progress[0], level, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v = read_level_atomic(a.ctl, level % kStatSlots);
    if (v.frontier == 0) return level;
    if (__hip_atomic_load(&a.ctl->error[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return level;
    level_features(feat, v, a, level, prev);
    engine = choose_engine(a, v, feat, level, s_mlp, &fallback);
    if (!single_eligible(a, engine, v)) return level;
  }
}

template <int SIGMA, class SliceT, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_bfs_persistent(BfsArgs a) {
  extern __shared__ float s_mlp[];
  __shared__ __attribute__((aligned(16))) int hs[kSingleLds];
  __shared__ int s_level;
  const unsigned nblocks = gridDim.x;
  const long long nthreads = static_cast<long long>(nblocks) * BLOCK;
  const long long gtid = static_cast<long long>(blockIdx.x) * BLOCK + threadIdx.x;
  const long long gwave = static_cast<long long>(blockIdx.x) * (BLOCK / 64) + wave_in_block();
  const long long nwaves = static_cast<long long>(nblocks) * (BLOCK / 64);
  const bool learned = a.policy == BLEST_POLICY_LEARNED && a.mlp != nullptr && a.mlp->valid;
  if (learned) mlp_to_lds(a.mlp, s_mlp);
  for (int i = threadIdx.x; i < kSingleHash + 1; i += BLOCK) hs[i] = (i == kSingleHash) ? 0 : -1;
  // state clear and level-0 seed before the registration barrier, which also
  // publishes them (one device-wide barrier at kernel start)
  clear_state<SIGMA>(a, gtid, nthreads, true);
  if (blockIdx.x == 0) {
    __syncthreads();  // block 0's counter clear before its seed counters
    seed_source<SIGMA>(a, true);
    if (threadIdx.x == 0) a.ctl->single_gen[0] = 0u;
  }
  BarrierCtx bc;
  if (!barrier_register(a.ctl, &bc, a.timeout_ticks)) return;
  unsigned episodes = 0;
  int level = 0;
  constexpr bool kPanelFmt = SIGMA == 8 && sizeof(SliceT) == 4;
  LevelView v = read_level(a.ctl, 0);
  long long prev_frontier = 0;
  bool decided = false;  // engine/feat/fallback already computed for `level`
  int engine = 0, fallback = 0;
  float feat[kMaxSwitchFeatures];
  for (;;) {
    const int slot = level % kStatSlots;
    if (v.frontier == 0) break;
    if (!decided) {
      level_features(feat, v, a, level, prev_frontier);
      fallback = 0;
      engine = choose_engine(a, v, feat, level, learned ? s_mlp : nullptr, &fallback);
    }
    decided = false;
    if (single_eligible(a, engine, v)) {
      ++episodes;
      if (blockIdx.x == 0) {
        const int next = single_episode<SIGMA, SliceT, BLOCK>(a, level, engine, fallback, feat, v,
                                                              learned ? s_mlp : nullptr, to_lds(hs));
        block_sync_mem();
        if (threadIdx.x == 0) {
          __hip_atomic_store(&a.ctl->single_level[0], next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&a.ctl->single_gen[0], episodes, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          // counters were updated by device atomics during the episode; drop
          // any cached copies before the plain loads of grid mode
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          s_level = next;
        }
      } else if (threadIdx.x == 0) {
        // wait for workgroup 0 to finish the episode, bounded like a barrier;
        // the bound restarts whenever the episode finishes a level, so it
        // measures a stall, not the length of a long run of small levels
        unsigned long long t0 = dev_ticks();
        int seen = -1;
        bool ok = true;
        while (__hip_atomic_load(&a.ctl->single_gen[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < episodes) {
          if (__hip_atomic_load(&a.ctl->error[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            ok = false;
            break;
          }
          const int prog = __hip_atomic_load(&a.ctl->single_progress[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (prog != seen) {
            seen = prog;
            t0 = dev_ticks();
          }
          if (dev_ticks() - t0 > a.timeout_ticks) {
            __hip_atomic_store(&a.ctl->error[0], static_cast<int>(BLEST_ERR_TIMEOUT), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            ok = false;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_level = ok ? __hip_atomic_load(&a.ctl->single_level[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : -1;
      }
      __syncthreads();
      if (s_level < 0 || __hip_atomic_load(&a.ctl->error[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
        return;
      level = s_level;
      v = read_level(a.ctl, level % kStatSlots);
      prev_frontier = level > 0 ? read_level(a.ctl, (level + kStatSlots - 1) % kStatSlots).frontier : 0;
      continue;
    }
    if (blockIdx.x == 0) {
      if (threadIdx.x == 0) log_level(a, level, v, a.probe ? -1 : engine, fallback, feat);
      const int nslot = (level + 1) % kStatSlots;
      for (int t = threadIdx.x; t < kStatFields; t += BLOCK) a.ctl->acc[nslot][t][0] = 0ULL;
    }
    const int sel = level & 1;
    // A BVSS step over the panel copy does Stage 2 itself (two-phase modes):
    // its partial counters are ready after the Stage 1 barrier.
    const bool fused = !a.probe && a.count_first != 0 && engine == BLEST_ENGINE_BVSS && kPanelFmt && use_panel(a, v);
    if (a.probe) {
      for (int e = 0; e < 3; ++e) {
        const unsigned long long t0 = dev_ticks();
        run_engine<SIGMA, SliceT, BLOCK>(a, e, sel, slot, v, gtid, nthreads, gwave, nwaves, nullptr,
                                         to_lds(reinterpret_cast<uint32_t*>(hs)));
        if (!grid_barrier(a.ctl, bc)) return;
        if (blockIdx.x == 0 && threadIdx.x == 0 && level < a.log_cap) a.log[level].t_engine[e] = dev_ticks() - t0;
      }
    } else {
      run_engine<SIGMA, SliceT, BLOCK>(a, engine, sel, slot, v, gtid, nthreads, gwave, nwaves, nullptr,
                                       to_lds(reinterpret_cast<uint32_t*>(hs)), fused ? level + 1 : -1);
      if (!grid_barrier(a.ctl, bc)) return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && level < a.log_cap) a.log[level].t_mid = dev_ticks();
    // Stage 2. When the next level is likely dense (this step was BVSS over
    // the panel copy, or bottom-up on a frontier that did not shrink, or the
    // frontier's mean degree is at least 8, so the next frontier will be much
    // larger) it will likely read no list: the two-phase form counts first
    // and writes lists only if the chosen engine needs them. Otherwise (a
    // shrinking bottom-up tail is usually followed by a small queue step)
    // the lists are built in the same pass (one device atomic per window and
    // list), which saves a barrier.
    // The level statistics come from the per-workgroup partials either way.
    const bool dense_next = (engine == BLEST_ENGINE_BOTTOM_UP && v.frontier >= prev_frontier) ||
                            (engine == BLEST_ENGINE_BVSS && kPanelFmt && use_panel(a, v)) ||
                            v.fedges >= 8 * v.frontier;
    const bool two_phase = fused || (!a.probe && (a.count_first == 2 || (a.count_first == 1 && dense_next)));
    LevelView nv;
    bool emitted = false;
    long long before[3] = {0, 0, 0};
    {
      if (!fused) {
        if (two_phase)
          finalize_count<SIGMA, BLOCK, FIN_COUNT>(a, level + 1, (level + 1) % kStatSlots, sel ^ 1);
        else
          finalize_count<SIGMA, BLOCK, FIN_ATOMIC>(a, level + 1, (level + 1) % kStatSlots, sel ^ 1);
        if (!grid_barrier(a.ctl, bc)) return;
      }
      long long tot[kParts];
      reduce_parts<BLOCK>(a, tot, before);
      nv.frontier = tot[0];
      nv.qslices = tot[1];
      nv.fedges = tot[2];
      nv.deg32 = tot[3];
      nv.deg1024 = tot[4];
      nv.light = tot[5];
      nv.heavy = tot[6];
      nv.queue = tot[7];
      nv.cumv = v.cumv + tot[0];
      nv.cume = v.cume + tot[2];
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (level < a.log_cap) a.log[level].t_count = dev_ticks();
        // the level's counters, for a single-workgroup episode that may follow
        unsigned long long* acc = &a.ctl->acc[(level + 1) % kStatSlots][0][0];
        const long long vals[10] = {nv.frontier, nv.queue, nv.qslices, nv.fedges, nv.deg32,
                                    nv.deg1024,  nv.light, nv.heavy,   nv.cumv,   nv.cume};
        for (int f = 0; f < 10; ++f)
          __hip_atomic_store(acc + f * kPad, static_cast<unsigned long long>(vals[f]), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (nv.frontier > 0) {
      level_features(feat, nv, a, level + 1, v.frontier);
      fallback = 0;
      engine = choose_engine(a, nv, feat, level + 1, learned ? s_mlp : nullptr, &fallback);
      decided = true;
      if (two_phase) {
        const bool want_queue = engine == BLEST_ENGINE_BVSS && !(kPanelFmt && use_panel(a, nv));
        const bool want_push = engine == BLEST_ENGINE_PUSH;
        if (want_queue || want_push) {
          finalize_emit<SIGMA, BLOCK>(a, sel ^ 1, before, want_push, want_queue, fused);
          emitted = true;
        }
      }
    }
    if (emitted && !grid_barrier(a.ctl, bc)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0 && level < a.log_cap) {
      a.log[level].t_end = dev_ticks();
      a.log[level].work = static_cast<long long>(a.ctl->acc[slot][F_WORK][0]);
    }
    prev_frontier = v.frontier;
    v = nv;
    ++level;
  }
  if (blockIdx.x == 0) {
    // Nothing reads the XCD registration after barrier_register; clear it
    // for the next launch.
    if (threadIdx.x < 8) a.ctl->xcd_blocks[threadIdx.x][0] = 0u;
    if (threadIdx.x == 8) a.ctl->xcd_active[0] = 0u;
    if (threadIdx.x == 0) a.ctl->nlevels[0] = level;
  }
}

// ------------------------------------------- eager vertex updates (Alg. 2)
//
// Alg. 2 (Section "Compute Mechanics") updates a vertex as soon as a slice
// hits it: the level is written, the vertex's bit is ORed into the next
// frontier word by an atomic whose returned value identifies the first
// writer of each slice set, and that writer enqueues the set's VSSs. There is
// no Stage 2 sweep and one device-wide barrier per level, which suits graphs
// whose rows inside a VSS are clustered (update divergence at most 25,000,
// Section "Ablation Studies"): there the scattered updates that the lazy
// scheme defers are cheap, and its per-level Stage 2 pass is what dominates
// thousands of small levels.
//
// Buffers rotate over three levels. Level l reads the frontier words F_l and
// the queue Q_l (buffers l mod 3), builds F_{l+1} and Q_{l+1} (buffers
// (l + 1) mod 3, all-zero words when the level starts), ORs F_l into the
// visited words walking Q_l, and zeroes the words of F_{l-1} walking Q_{l-1},
// which makes that buffer clean for level l + 1. Visited words therefore hold
// every vertex of levels < l and possibly some of level l, so a vertex was
// reached before level l + 1 iff its bit is set in visited | F_l, whichever
// of the two copies a wave reads. The statistics of level l + 1 (the inputs
// of Eq. 3 and of the switch network) are summed by device atomics into the
// rotating counter slot (l + 1) mod 3, which level l - 1 zeroed.

__device__ __forceinline__ void* eager_front(const BfsArgs& a, int b) {
  return static_cast<char*>(a.front) + static_cast<long long>(b) * a.fstride;
}

// Atomic OR of a sigma-bit word (8- and 16-bit words through the aligned
// 32-bit word that holds them); returns the word's previous value.
template <int SIGMA>
__device__ __forceinline__ typename MaskOf<SIGMA>::T atomic_or_word(typename MaskOf<SIGMA>::T* p,
                                                                    typename MaskOf<SIGMA>::T bits) {
  using M = typename MaskOf<SIGMA>::T;
  if constexpr (SIGMA == 32) {
    return __hip_atomic_fetch_or(p, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    const uintptr_t addr = reinterpret_cast<uintptr_t>(p);
    uint32_t* w = reinterpret_cast<uint32_t*>(addr & ~uintptr_t(3));
    const uint32_t sh = static_cast<uint32_t>(addr & 3u) * 8u;
    const uint32_t old =
        __hip_atomic_fetch_or(w, static_cast<uint32_t>(bits) << sh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return static_cast<M>(old >> sh);
  }
}

// Per-lane counts of a level's new vertices, summed per wave at the end.
struct EagerStats {
  long long frontier = 0, qslices = 0, fedges = 0, deg32 = 0, deg1024 = 0, work = 0;
};

__device__ __forceinline__ void eager_new_vertex(const BfsArgs& a, uint32_t u, int32_t deg, int new_level,
                                                 EagerStats& st) {
  a.levels[a.orig_id ? a.orig_id[u] : static_cast<int32_t>(u)] = new_level;
  st.frontier += 1;
  st.fedges += deg;
  st.deg32 += deg >= 32;
  st.deg1024 += deg >= 1024;
}

// Appends every VSS of slice set s to q; qcur is the F_QUEUE counter of the
// next level's slot, which doubles as q's append cursor.
__device__ __forceinline__ void eager_enqueue(const BfsArgs& a, uint32_t s, uint4* q, unsigned long long* qcur,
                                              EagerStats& st) {
  const uint32_t s0 = a.slice_ptr[s], ns = a.slice_ptr[s + 1] - s0;
  const uint32_t tau = static_cast<uint32_t>(a.tau);
  const uint32_t nv = (ns + tau - 1) / tau;
  if (nv == 0) return;
  const unsigned long long off = fetch_add_u64(qcur, nv);
  for (uint32_t k = 0; k < nv; ++k) q[off + k] = make_uint4(s0 + k * tau, min(tau, ns - k * tau), 0u, s);
  st.qslices += ns;
}

// Top-down step of Alg. 2: a wave takes G queued VSSs at a time, reads their
// sets' frontier words from F_l and all their slices, then handles the hits.
template <int SIGMA, class SliceT, int K>
__device__ void eager_td_k(const BfsArgs& a, int level, long long qlen, long long gwave, long long nwaves,
                           EagerStats& st) {
  using M = typename MaskOf<SIGMA>::T;
  constexpr int G = 4;
  const int cb = level % 3, nb = (level + 1) % 3;
  const gptr<const uint4> qg = to_global(static_cast<const uint4*>(a.queue[cb]));
  uint4* qn = a.queue[nb];
  unsigned long long* qcur = &a.ctl->acc[(level + 1) % kStatSlots][F_QUEUE][0];
  gptr<const SliceT> __restrict__ sl = to_global(static_cast<const SliceT*>(a.slices));
  gptr<const M> vis = to_global(static_cast<const M*>(a.vis));
  gptr<const M> fc = to_global(static_cast<const M*>(eager_front(a, cb)));
  M* fn = static_cast<M*>(eager_front(a, nb));
  gptr<const int32_t> rp = to_global(a.rp);
  const uint32_t lane = static_cast<uint32_t>(lane_id());
  for (long long base = gwave * G; base < qlen; base += nwaves * G) {
    uint4 dl = make_uint4(0u, 0u, 0u, 0u);
    uint32_t al_l = 0;
    if (lane < G && base + lane < qlen) {
      dl = qg[base + lane];
      al_l = static_cast<uint32_t>(fc[dl.w]);
    }
    uint32_t s0[G], cn[G];
    SliceT al[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      s0[g] = __builtin_amdgcn_readlane(dl.x, g);
      cn[g] = __builtin_amdgcn_readlane(dl.y, g);
      al[g] = static_cast<SliceT>(static_cast<uint32_t>(__builtin_amdgcn_readlane(al_l, g)));
    }
    SliceT w[G][K];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint32_t j = lane + 64u * k;
        st.work += j < cn[g];
        w[g][k] = (j < cn[g]) ? sl[s0[g] + j] : SliceT(0);
      }
    // visited | F_l of every hit row, all loads issued before any test
    M seen[G][K];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint32_t row = static_cast<uint32_t>(w[g][k] >> SliceFmt<SliceT>::kRowShift);
        seen[g][k] = (w[g][k] & al[g]) ? static_cast<M>(vis[row / SIGMA] | fc[row / SIGMA]) : M(~M(0));
      }
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint32_t row = static_cast<uint32_t>(w[g][k] >> SliceFmt<SliceT>::kRowShift);
        const M bit = static_cast<M>(M(1) << (row % SIGMA));
        if (!(seen[g][k] & bit)) {
          const M old = atomic_or_word<SIGMA>(fn + row / SIGMA, bit);
          if (!(old & bit)) {
            eager_new_vertex(a, row, rp[row + 1] - rp[row], level + 1, st);
            if (old == 0) eager_enqueue(a, row / SIGMA, qn, qcur, st);
          }
        }
      }
  }
}

template <int SIGMA, class SliceT>
__device__ __forceinline__ void eager_td(const BfsArgs& a, int level, long long qlen, long long gwave,
                                                   long long nwaves, EagerStats& st) {
  switch (a.tau) {
    case 64:
      return eager_td_k<SIGMA, SliceT, 1>(a, level, qlen, gwave, nwaves, st);
    case 128:
      return eager_td_k<SIGMA, SliceT, 2>(a, level, qlen, gwave, nwaves, st);
    case 192:
      return eager_td_k<SIGMA, SliceT, 3>(a, level, qlen, gwave, nwaves, st);
    default:
      return eager_td_k<SIGMA, SliceT, 4>(a, level, qlen, gwave, nwaves, st);
  }
}

// Bottom-up step (Alg. 4) with eager updates: a lane owns a vertex, an
// unvisited vertex scans its row (the whole wave scans rows longer than
// kPullLight) for a neighbour in F_l. The wave owns all sigma vertices of each
// of its sets, so it writes their F_{l+1} words with plain stores and
// enqueues the sets that gained vertices.
template <int SIGMA>
__device__ __forceinline__ void eager_bu(const BfsArgs& a, int level, long long gwave, long long nwaves,
                                                   EagerStats& st) {
  using M = typename MaskOf<SIGMA>::T;
  const int cb = level % 3, nb = (level + 1) % 3;
  gptr<const M> vis = to_global(static_cast<const M*>(a.vis));
  gptr<const M> fc = to_global(static_cast<const M*>(eager_front(a, cb)));
  gptr<const M> degm = to_global(static_cast<const M*>(a.degmask_in));
  M* fn = static_cast<M*>(eager_front(a, nb));
  uint4* qn = a.queue[nb];
  unsigned long long* qcur = &a.ctl->acc[(level + 1) % kStatSlots][F_QUEUE][0];
  gptr<const int32_t> rp = to_global(a.rp_in);
  gptr<const int32_t> col = to_global(a.col_in);
  gptr<const int32_t> rp_out = to_global(a.rp);
  const long long nv = a.nsets * SIGMA;
  const int lane = lane_id();
  const long long nchunks = (nv + 63) / 64;
  // 64-vertex chunks, round k rotated by k (as in the lazy bottom-up engine)
  for (long long k = 0; k * nwaves < nchunks; ++k) {
    const long long chunk = k * nwaves + (gwave + k) % nwaves;
    if (chunk >= nchunks) continue;
    const long long u = chunk * 64 + lane;
    bool cand = false;
    int p = 0, e = 0;
    if (u < nv) {
      const long long s = u / SIGMA;
      const M unv = static_cast<M>(~(vis[s] | fc[s]) & degm[s]);
      cand = (unv >> (u % SIGMA)) & 1u;
    }
    if (!__ballot(cand)) continue;
    if (cand) {
      p = rp[u];
      e = rp[u + 1];
    }
    const bool heavy = cand && e - p > kPullLight;
    bool found = false;
    if (cand && !heavy) {
      for (int q = p; q < e && !found; ++q) {
        const int v = col[q];
        found = (fc[v / SIGMA] >> (v % SIGMA)) & 1u;
        ++st.work;
      }
    }
    unsigned long long hb = __ballot(heavy);
    while (hb) {
      const int l = __builtin_ctzll(hb);
      hb &= hb - 1;
      const int hp = __builtin_amdgcn_readlane(p, l), he = __builtin_amdgcn_readlane(e, l);
      for (int q = hp; q < he; q += 64) {
        const int i = q + lane;
        bool f = false;
        if (i < he) {
          const int v = col[i];
          f = (fc[v / SIGMA] >> (v % SIGMA)) & 1u;
          ++st.work;
        }
        if (__ballot(f)) {
          if (lane == l) found = true;
          break;
        }
      }
    }
    const unsigned long long got = __ballot(found);
    if (!got) continue;
    // the statistics count out-arcs (the frontier's edges for the next step)
    if (found) eager_new_vertex(a, static_cast<uint32_t>(u), rp_out[u + 1] - rp_out[u], level + 1, st);
    if (lane % SIGMA == 0) {
      const M bits = static_cast<M>(got >> lane);
      if (bits) {
        fn[u / SIGMA] = bits;
        eager_enqueue(a, static_cast<uint32_t>(u / SIGMA), qn, qcur, st);
      }
    }
  }
}

// Adds the wave's counts to the next level's slot (one atomic per wave and field).
__device__ __forceinline__ void eager_flush(const BfsArgs& a, const EagerStats& st, int nslot, int slot) {
  long long v[6] = {st.frontier, st.qslices, st.fedges, st.deg32, st.deg1024, st.work};
#pragma unroll
  for (int k = 0; k < 6; ++k) v[k] = wave_sum(v[k]);
  if (lane_id() == 0) {
    constexpr int f[5] = {F_FRONTIER, F_QSLICES, F_FEDGES, F_DEG32, F_DEG1024};
#pragma unroll
    for (int k = 0; k < 5; ++k)
      if (v[k]) add_u64(&a.ctl->acc[nslot][f[k]][0], static_cast<unsigned long long>(v[k]));
    if (v[5] && (a.count_work || a.probe)) add_u64(&a.ctl->acc[slot][F_WORK][0], static_cast<unsigned long long>(v[5]));
  }
}

// Levels whose queue holds at most this many slices run on workgroup 0 alone
// (workgroup barriers instead of device-wide ones), consecutively, while the
// other workgroups wait; a bottom-up level never does.
constexpr long long kEagerSingleSlices = 256;

// One level of the eager scheme by the calling workgroups (the whole grid,
// or workgroup 0 alone): bookkeeping, the engine and its counters. The caller
// synchronises afterwards (device-wide or workgroup barrier).
template <int SIGMA, class SliceT, int BLOCK>
__device__ __forceinline__ void eager_level(const BfsArgs& a, int level, const LevelView& v, long long prev_queue,
                                            int engine, int fallback, const float (&feat)[kMaxSwitchFeatures],
                                            long long gtid, long long nthreads, long long gwave, long long nwaves) {
  using M = typename MaskOf<SIGMA>::T;
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) {
      log_level(a, level, v, engine, fallback, feat);
      if (level < a.log_cap) a.log[level].panel = 0;
    }
    // the slot level + 2 accumulates into during the next level
    const int zslot = (level + 2) % kStatSlots;
    for (int t = threadIdx.x; t < kStatFields; t += BLOCK)
      __hip_atomic_store(&a.ctl->acc[zslot][t][0], 0ULL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  EagerStats st;
  if (engine == BLEST_ENGINE_BOTTOM_UP)
    eager_bu<SIGMA>(a, level, gwave, nwaves, st);
  else
    eager_td<SIGMA, SliceT>(a, level, v.queue, gwave, nwaves, st);
  {
    // F_l into the visited words (walking Q_l); F_{l-1} cleared (walking Q_{l-1})
    const gptr<const uint4> qc = to_global(static_cast<const uint4*>(a.queue[level % 3]));
    const gptr<const uint4> qp = to_global(static_cast<const uint4*>(a.queue[(level + 2) % 3]));
    gptr<M> vis = to_global(static_cast<M*>(a.vis));
    const gptr<const M> fc = to_global(static_cast<const M*>(eager_front(a, level % 3)));
    gptr<M> fp = to_global(static_cast<M*>(eager_front(a, (level + 2) % 3)));
    for (long long i = gtid; i < v.queue; i += nthreads) {
      const uint32_t s = qc[i].w;
      vis[s] = static_cast<M>(vis[s] | fc[s]);
    }
    for (long long i = gtid; i < prev_queue; i += nthreads) fp[qp[i].w] = 0;
  }
  eager_flush(a, st, (level + 1) % kStatSlots, level % kStatSlots);
}

template <int SIGMA, class SliceT, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_bfs_eager(BfsArgs a) {
  extern __shared__ float s_mlp[];
  __shared__ int s_level;
  using M = typename MaskOf<SIGMA>::T;
  const unsigned nblocks = gridDim.x;
  const long long nthreads = static_cast<long long>(nblocks) * BLOCK;
  const long long gtid = static_cast<long long>(blockIdx.x) * BLOCK + threadIdx.x;
  const long long gwave = static_cast<long long>(blockIdx.x) * (BLOCK / 64) + wave_in_block();
  const long long nwaves = static_cast<long long>(nblocks) * (BLOCK / 64);
  const bool learned = a.policy == BLEST_POLICY_LEARNED && a.mlp != nullptr && a.mlp->valid;
  if (learned) mlp_to_lds(a.mlp, s_mlp);
  // levels, visited words and F_0, F_1 as in the lazy scheme, plus F_2; the
  // registration barrier publishes them with the level-0 counters and queue
  clear_state<SIGMA>(a, gtid, nthreads, true);
  {
    M* f2 = static_cast<M*>(eager_front(a, 2));
    for (long long s = gtid; s < a.nsets; s += nthreads) f2[s] = 0;
  }
  if (blockIdx.x == 0) {
    __syncthreads();  // block 0's counter clear before its seed counters
    seed_source<SIGMA>(a, true);
    if (threadIdx.x == 0) a.ctl->single_gen[0] = 0u;
  }
  BarrierCtx bc;
  if (!barrier_register(a.ctl, &bc, a.timeout_ticks)) return;
  int level = 0;
  unsigned episodes = 0;
  bool in_episode = false;  // workgroup 0: running consecutive levels alone
  LevelView v = read_level(a.ctl, 0);
  long long prev_frontier = 0, prev_queue = 0;
  float feat[kMaxSwitchFeatures];
  for (;;) {
    const bool done = v.frontier == 0;
    int engine = 0, fallback = 0;
    bool single = false;
    if (!done) {
      level_features(feat, v, a, level, prev_frontier);
      engine = choose_engine_inl(a, v, feat, level, learned ? s_mlp : nullptr, &fallback);
      if (engine == BLEST_ENGINE_PUSH) engine = BLEST_ENGINE_BVSS;
      single = a.single_block && engine != BLEST_ENGINE_BOTTOM_UP && v.qslices <= kEagerSingleSlices;
    }
    if (blockIdx.x == 0 && in_episode && (done || !single)) {
      // end of an episode: hand the state to the waiting workgroups, with the
      // cumulative counts they did not follow
      block_sync_mem();
      if (threadIdx.x == 0) {
        unsigned long long* acc = &a.ctl->acc[level % kStatSlots][0][0];
        __hip_atomic_store(acc + F_CUMV * kPad, static_cast<unsigned long long>(v.cumv), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(acc + F_CUME * kPad, static_cast<unsigned long long>(v.cume), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&a.ctl->single_level[0], level, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&a.ctl->single_gen[0], episodes, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
      in_episode = false;
    }
    if (done) break;
    if (single && blockIdx.x == 0) {
      // a small level on workgroup 0 alone, workgroup barrier only
      if (!in_episode) {
        in_episode = true;
        ++episodes;
      }
      eager_level<SIGMA, SliceT, BLOCK>(a, level, v, prev_queue, engine, fallback, feat, threadIdx.x, BLOCK,
                                        wave_in_block(), BLOCK / 64);
      block_sync_mem();
      if (threadIdx.x == 0 && level < a.log_cap) {
        const unsigned long long t = dev_ticks();
        a.log[level].t_mid = t;
        a.log[level].t_end = t;
      }
      LevelView nv = read_level_atomic(a.ctl, (level + 1) % kStatSlots);
      nv.light = 0;
      nv.heavy = 0;
      nv.cumv = v.cumv + nv.frontier;
      nv.cume = v.cume + nv.fedges;
      prev_frontier = v.frontier;
      prev_queue = v.queue;
      v = nv;
      ++level;
      // progress for the waiting workgroups: their time bound restarts with every level
      if (threadIdx.x == 0)
        __hip_atomic_store(&a.ctl->single_progress[0], level, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (__hip_atomic_load(&a.ctl->error[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
      continue;
    }
    if (single) {
      // wait for workgroup 0's episode, bounded like a barrier; the bound
      // restarts at every level the episode finishes
      ++episodes;
      if (threadIdx.x == 0) {
        unsigned long long t0 = dev_ticks();
        int seen = -1;
        bool ok = true;
        while (__hip_atomic_load(&a.ctl->single_gen[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < episodes) {
          if (__hip_atomic_load(&a.ctl->error[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            ok = false;
            break;
          }
          const int prog = __hip_atomic_load(&a.ctl->single_progress[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (prog != seen) {
            seen = prog;
            t0 = dev_ticks();
          }
          if (dev_ticks() - t0 > a.timeout_ticks) {
            __hip_atomic_store(&a.ctl->error[0], static_cast<int>(BLEST_ERR_TIMEOUT), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            ok = false;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_level = ok ? __hip_atomic_load(&a.ctl->single_level[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : -1;
      }
      __syncthreads();
      if (s_level < 0 || __hip_atomic_load(&a.ctl->error[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
        return;
      level = s_level;
      v = read_level(a.ctl, level % kStatSlots);
      v.light = 0;
      v.heavy = 0;
      const LevelView pv = read_level(a.ctl, (level + kStatSlots - 1) % kStatSlots);
      prev_frontier = pv.frontier;
      prev_queue = pv.queue;
      continue;
    }
    eager_level<SIGMA, SliceT, BLOCK>(a, level, v, prev_queue, engine, fallback, feat, gtid, nthreads, gwave, nwaves);
    if (!grid_barrier(a.ctl, bc)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0 && level < a.log_cap) {
      const unsigned long long t = dev_ticks();
      a.log[level].t_mid = t;
      a.log[level].t_end = t;
      a.log[level].work = static_cast<long long>(a.ctl->acc[level % kStatSlots][F_WORK][0]);
    }
    LevelView nv = read_level(a.ctl, (level + 1) % kStatSlots);
    nv.light = 0;
    nv.heavy = 0;
    nv.cumv = v.cumv + nv.frontier;
    nv.cume = v.cume + nv.fedges;
    prev_frontier = v.frontier;
    prev_queue = v.queue;
    v = nv;
    ++level;
  }
  if (blockIdx.x == 0) {
    if (threadIdx.x < 8) a.ctl->xcd_blocks[threadIdx.x][0] = 0u;
    if (threadIdx.x == 8) a.ctl->xcd_active[0] = 0u;
    if (threadIdx.x == 0) a.ctl->nlevels[0] = level;
  }
}

// ------------------------------------------------------ per-stage kernels

template <int SIGMA, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_bfs_clear(BfsArgs a) {
  const long long nthreads = static_cast<long long>(gridDim.x) * BLOCK;
  clear_state<SIGMA>(a, static_cast<long long>(blockIdx.x) * BLOCK + threadIdx.x, nthreads);
  if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->done[0] = 0;
}

template <int SIGMA, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_bfs_seed(BfsArgs a) {
  seed_source<SIGMA>(a);
}

template <int SIGMA, class SliceT, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_bfs_stage1(BfsArgs a, int level, long long prev_slot_frontier_unused) {
  extern __shared__ float s_mlp[];
  if (a.ctl->done[0]) return;
  const unsigned nblocks = gridDim.x;
  const long long nthreads = static_cast<long long>(nblocks) * BLOCK;
  const long long gtid = static_cast<long long>(blockIdx.x) * BLOCK + threadIdx.x;
  const long long gwave = static_cast<long long>(blockIdx.x) * (BLOCK / 64) + wave_in_block();
  const long long nwaves = static_cast<long long>(nblocks) * (BLOCK / 64);
  const LevelView v = read_level(a.ctl, level % kStatSlots);
  if (v.frontier == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.ctl->done[0] = 1;
      a.ctl->nlevels[0] = level;
    }
    return;
  }
  const long long prev = level > 0 ? read_level(a.ctl, (level + kStatSlots - 1) % kStatSlots).frontier : 0;
  const bool learned = a.policy == BLEST_POLICY_LEARNED && a.mlp != nullptr && a.mlp->valid;
  if (learned) {
    mlp_to_lds(a.mlp, s_mlp);
    __syncthreads();
  }
  float feat[kMaxSwitchFeatures];
  level_features(feat, v, a, level, prev);
  int fallback = 0;
  const int engine = choose_engine(a, v, feat, level, learned ? s_mlp : nullptr, &fallback);
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) log_level(a, level, v, engine, fallback, feat);
    const int nslot = (level + 1) % kStatSlots;
    for (int t = threadIdx.x; t < kStatFields; t += BLOCK) a.ctl->acc[nslot][t][0] = 0ULL;
  }
  __shared__ __attribute__((aligned(16))) uint32_t pm[kPanelMaxBytes / 4];
  run_engine<SIGMA, SliceT, BLOCK>(a, engine, level & 1, level % kStatSlots, v, gtid, nthreads, gwave, nwaves, nullptr,
                                   to_lds(pm));
}

template <int SIGMA, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_bfs_stage2(BfsArgs a, int level) {
  if (a.ctl->done[0]) return;
  const LevelView v = read_level(a.ctl, level % kStatSlots);
  if (v.frontier == 0) return;
  if (blockIdx.x == 0 && threadIdx.x == 0 && level < a.log_cap) a.log[level].t_mid = dev_ticks();
  finalize<SIGMA, BLOCK>(a, level + 1, (level + 1) % kStatSlots, (level & 1) ^ 1, v.cumv, v.cume, gridDim.x);
  if (blockIdx.x == 0 && threadIdx.x == 0 && level < a.log_cap) {
    a.log[level].t_end = dev_ticks();
    a.log[level].work = static_cast<long long>(a.ctl->acc[level % kStatSlots][F_WORK][0]);
  }
}

// ------------------------------------------------------------ host side

namespace {

template <int SIGMA, class SliceT, int BLOCK>
const void* persistent_fn() {
  return reinterpret_cast<const void*>(&k_bfs_persistent<SIGMA, SliceT, BLOCK>);
}

template <int SIGMA, class SliceT, int BLOCK>
const void* eager_fn() {
  return reinterpret_cast<const void*>(&k_bfs_eager<SIGMA, SliceT, BLOCK>);
}

template <int SIGMA, class SliceT, int BLOCK>
hipError_t run_t(const DevGraph& g, BfsArgs& a, hipStream_t st) {
  const size_t shmem = (a.policy == BLEST_POLICY_LEARNED) ? kLdsMlpFloats * sizeof(float) : 0;
  if (g.eager && !a.probe) {
    void* args[] = {static_cast<void*>(&a)};
    return hipLaunchCooperativeKernel(eager_fn<SIGMA, SliceT, BLOCK>(), dim3(g.grid_eager), dim3(BLOCK), args,
                                      static_cast<unsigned>(shmem), st);
  }
  if (g.persistent || a.probe) {
    void* args[] = {static_cast<void*>(&a)};
    return hipLaunchCooperativeKernel(persistent_fn<SIGMA, SliceT, BLOCK>(), dim3(g.grid), dim3(BLOCK), args,
                                      static_cast<unsigned>(shmem), st);
  }
  hipLaunchKernelGGL((k_bfs_clear<SIGMA, BLOCK>), dim3(g.grid), dim3(BLOCK), 0, st, a);
  hipLaunchKernelGGL((k_bfs_seed<SIGMA, BLOCK>), dim3(1), dim3(BLOCK), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int level = 0;
  int batch = 4;
  for (;;) {
    for (int i = 0; i < batch; ++i, ++level) {
      hipLaunchKernelGGL((k_bfs_stage1<SIGMA, SliceT, BLOCK>), dim3(g.grid), dim3(BLOCK), shmem, st, a, level, 0LL);
      hipLaunchKernelGGL((k_bfs_stage2<SIGMA, BLOCK>), dim3(g.grid), dim3(BLOCK), 0, st, a, level);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(g.host_flags, &g.ctl->done[0], sizeof(int), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    if (g.host_flags[0]) break;
    if (level > g.n + 2) return hipErrorUnknown;
    batch = batch < 64 ? batch * 2 : 64;
  }
  return hipSuccess;
}

template <int SIGMA, class SliceT>
hipError_t run_block(const DevGraph& g, BfsArgs& a, hipStream_t st) {
  switch (g.block) {
    case 256:
      return run_t<SIGMA, SliceT, 256>(g, a, st);
    case 1024:
      return run_t<SIGMA, SliceT, 1024>(g, a, st);
    default:
      return run_t<SIGMA, SliceT, 512>(g, a, st);
  }
}

template <int SIGMA, class SliceT>
hipError_t occupancy_block(const DevGraph& g, size_t shmem, int* nb) {
  switch (g.block) {
    case 256:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, persistent_fn<SIGMA, SliceT, 256>(), 256, shmem);
    case 1024:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, persistent_fn<SIGMA, SliceT, 1024>(), 1024, shmem);
    default:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, persistent_fn<SIGMA, SliceT, 512>(), 512, shmem);
  }
}

template <int SIGMA, class SliceT>
hipError_t occupancy_eager(const DevGraph& g, size_t shmem, int* nb) {
  switch (g.block) {
    case 256:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, eager_fn<SIGMA, SliceT, 256>(), 256, shmem);
    case 1024:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, eager_fn<SIGMA, SliceT, 1024>(), 1024, shmem);
    default:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, eager_fn<SIGMA, SliceT, 512>(), 512, shmem);
  }
}

}  // namespace

hipError_t bfs_grid_size_eager(const DevGraph& g, int blocks_per_cu, int* grid) {
  // sized with the switch network's LDS, which the learned policy adds
  const size_t shmem = kLdsMlpFloats * sizeof(float);
  int nb = 0;
  hipError_t e;
  if (g.sigma == 8 && !g.wide)
    e = occupancy_eager<8, uint32_t>(g, shmem, &nb);
  else if (g.sigma == 8)
    e = occupancy_eager<8, uint64_t>(g, shmem, &nb);
  else if (g.sigma == 16)
    e = occupancy_eager<16, uint64_t>(g, shmem, &nb);
  else
    e = occupancy_eager<32, uint64_t>(g, shmem, &nb);
  if (e != hipSuccess) return e;
  if (nb < 1) return hipErrorInvalidConfiguration;
  // its levels are small and latency-bound: one workgroup per compute unit
  // (fewer arrivals per device-wide barrier) unless asked otherwise
  nb = blocks_per_cu > 0 ? std::min(nb, blocks_per_cu) : 1;
  *grid = nb * g.num_cu;
  return hipSuccess;
}

BfsArgs bfs_args(const DevGraph& g) {
  BfsArgs a{};
  a.rp = g.rp;
  a.col = g.col;
  a.slice_ptr = g.slice_ptr;
  a.slices = g.slices;
  a.degmask = g.degmask;
  a.rp_in = g.rp_in;
  a.col_in = g.col_in;
  a.degmask_in = g.degmask_in;
  a.orig_id = g.orig_id;
  a.n = g.n;
  a.m = g.m;
  a.nsets = g.nsets;
  a.tau = g.tau;
  a.vis = g.vis;
  a.front = g.front;
  a.fstride = static_cast<long long>(g.fstride);
  a.mark = g.mark;
  a.queue[2] = g.queue[2];
  for (int i = 0; i < 2; ++i) {
    a.queue[i] = g.queue[i];
    a.flight[i] = g.flight[i];
    a.fheavy[i] = g.fheavy[i];
  }
  a.ctl = g.ctl;
  a.part = g.part;
  a.log = g.log;
  a.log_cap = g.log_cap;
  a.mlp = g.mlp;
  a.prefilter = g.prefilter;
  a.count_work = g.count_work;
  a.single_block = g.single_block;
  a.pwords = g.pwords;
  a.pbase = g.pbase;
  a.pptr = g.pptr;
  a.npanels = static_cast<int32_t>(g.npanels);
  a.panel_rb = g.panel_rb;
  a.panel_mode = g.panel_mode;
  a.panel_slots = g.nchunks * kPanelChunk;
  a.nvss = g.nvss;
  a.nslices = g.nslices;
  a.count_first = g.count_first;
  a.timeout_ticks = 1000000000ULL;  // 10 s at the 100 MHz device clock
  return a;
}

hipError_t bfs_run(const DevGraph& g, BfsArgs a, hipStream_t st) {
  if (g.sigma == 8 && !g.wide) return run_block<8, uint32_t>(g, a, st);
  if (g.sigma == 8) return run_block<8, uint64_t>(g, a, st);
  if (g.sigma == 16) return run_block<16, uint64_t>(g, a, st);
  return run_block<32, uint64_t>(g, a, st);
}

hipError_t bfs_grid_size(const DevGraph& g, int policy_learned, int blocks_per_cu, int* grid) {
  const size_t shmem = policy_learned ? kLdsMlpFloats * sizeof(float) : 0;
  int nb = 0;
  hipError_t e;
  if (g.sigma == 8 && !g.wide)
    e = occupancy_block<8, uint32_t>(g, shmem, &nb);
  else if (g.sigma == 8)
    e = occupancy_block<8, uint64_t>(g, shmem, &nb);
  else if (g.sigma == 16)
    e = occupancy_block<16, uint64_t>(g, shmem, &nb);
  else
    e = occupancy_block<32, uint64_t>(g, shmem, &nb);
  if (e != hipSuccess) return e;
  if (nb < 1) return hipErrorInvalidConfiguration;
  if (blocks_per_cu > 0 && blocks_per_cu < nb) nb = blocks_per_cu;
  *grid = nb * g.num_cu;
  return hipSuccess;
}

}  // namespace blest
