// C ABI of the BVSS BFS library: argument checking, graph construction and
// ownership, error reporting, and dispatch to the device code.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "blest.h"
#include "blest_internal.h"
#include "host_build.h"
#include "msbfs.h"

struct blest_graph {
  blest::DevGraph d;
  blest_opts opts{};
  std::vector<int32_t> perm;  // input id -> internal id; empty when not reordered
  std::vector<int64_t> real_ptrs;
  std::vector<uint32_t> slice_ptr;
  int reordered = 0;
  int64_t bvss_bytes = 0, csr_bytes = 0, work_bytes = 0;
  int nlevels = 0;
  blest::MsDev ms;  // multi-source buffers, allocated on first use
  std::vector<void*> allocations;
};

namespace {

thread_local std::string g_err;

blest_status fail(blest_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

blest_status hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) return fail(BLEST_ERR_OOM, std::string(what) + ": out of device memory");
  return fail(BLEST_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define CK(expr)                                  \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)

std::mutex g_model_mu;
bool g_model_set = false;
float g_min_conf = 0.5f;
blest::MlpDev g_model{};
bool g_ms_model_set = false;
blest::MlpDev g_ms_model{};

hipError_t dalloc(blest_graph* g, void** p, size_t bytes) {
  *p = nullptr;
  hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 256));
  if (e == hipSuccess) g->allocations.push_back(*p);
  return e;
}

template <class T>
hipError_t dalloc_t(blest_graph* g, T** p, size_t count) {
  void* q = nullptr;
  hipError_t e = dalloc(g, &q, count * sizeof(T));
  *p = static_cast<T*>(q);
  return e;
}

void release(blest_graph* g) {
  if (!g) return;
  for (void* p : g->allocations) (void)hipFree(p);
  g->allocations.clear();
  if (g->d.host_flags) (void)hipHostFree(g->d.host_flags);
  g->d.host_flags = nullptr;
  blest::ms_free_all(&g->ms);
}

blest_status check_device(int want, int* dev, int* num_cu, double* tick_us) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return fail(BLEST_ERR_NO_DEVICE, "no HIP device");
  if (want >= 0) {
    if (want >= count) return fail(BLEST_ERR_NO_DEVICE, "device ordinal out of range");
    CK(hipSetDevice(want));
  }
  CK(hipGetDevice(dev));
  hipDeviceProp_t prop;
  CK(hipGetDeviceProperties(&prop, *dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(BLEST_ERR_NO_DEVICE, std::string("library is built for gfx950, device is ") + prop.gcnArchName);
  int coop = 0;
  CK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, *dev));
  if (!coop) return fail(BLEST_ERR_NO_DEVICE, "device lacks cooperative launch");
  *num_cu = prop.multiProcessorCount;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, *dev) != hipSuccess || khz <= 0) khz = 100000;
  *tick_us = 1000.0 / khz;
  return BLEST_OK;
}

blest_status wait_and_check(blest_graph* g, hipStream_t st) {
  CK(hipStreamSynchronize(st));
  int flags[2] = {0, 0};
  CK(hipMemcpy(&flags[0], &g->d.ctl->error[0], sizeof(int), hipMemcpyDeviceToHost));
  CK(hipMemcpy(&flags[1], &g->d.ctl->nlevels[0], sizeof(int), hipMemcpyDeviceToHost));
  g->nlevels = flags[1];
  if (flags[0] != 0) {
    // Leave the working state clean for the next call.
    CK(hipMemset(g->d.ctl, 0, sizeof(blest::Ctl)));
    CK(hipMemset(g->d.mark, 0, g->d.mark_bytes));
    blest::ms_reset(&g->ms);
    if (flags[0] == BLEST_ERR_TIMEOUT) return fail(BLEST_ERR_TIMEOUT, "device-wide barrier timed out");
    if (flags[0] == BLEST_ERR_OVERFLOW) return fail(BLEST_ERR_OVERFLOW, "a distance exceeds the int16 range");
    return fail(flags[0], "device-side error");
  }
  return BLEST_OK;
}

blest_status bfs_common(blest_graph* g, int32_t src, int32_t* levels_dev, void* stream, int probe) {
  if (!g || !levels_dev) return fail(BLEST_ERR_INVALID_ARG, "NULL graph or output");
  if (src < 0 || src >= g->d.n) return fail(BLEST_ERR_OUT_OF_RANGE, "source vertex out of range");
  hipStream_t st = static_cast<hipStream_t>(stream);
  CK(hipSetDevice(g->d.device));
  blest::BfsArgs a = blest::bfs_args(g->d);
  a.levels = levels_dev;
  a.src = g->perm.empty() ? src : g->perm[src];
  a.policy = g->opts.policy;
  a.eta = g->opts.eta;
  a.seed = g->opts.random_seed;
  a.probe = probe;
  hipError_t e = blest::bfs_run(g->d, a, st);
  if (e != hipSuccess) return hip_fail(e, "bfs launch");
  if (g->opts.async && !probe) return BLEST_OK;
  return wait_and_check(g, st);
}

}  // namespace

extern "C" {

const char* blest_status_str(blest_status s) {
  switch (s) {
    case BLEST_OK: return "OK";
    case BLEST_ERR_INVALID_ARG: return "INVALID_ARG";
    case BLEST_ERR_INVALID_GRAPH: return "INVALID_GRAPH";
    case BLEST_ERR_OUT_OF_RANGE: return "OUT_OF_RANGE";
    case BLEST_ERR_OOM: return "OOM";
    case BLEST_ERR_HIP: return "HIP";
    case BLEST_ERR_OVERFLOW: return "OVERFLOW";
    case BLEST_ERR_UNSUPPORTED: return "UNSUPPORTED";
    case BLEST_ERR_TIMEOUT: return "TIMEOUT";
    case BLEST_ERR_NO_DEVICE: return "NO_DEVICE";
    case BLEST_ERR_IO: return "IO";
    default: return "UNKNOWN";
  }
}

const char* blest_last_error(void) { return g_err.c_str(); }

void blest_default_opts(blest_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->sigma = 8;
  o->tau = 128;
  o->reorder = BLEST_REORDER_AUTO;
  o->policy = BLEST_POLICY_HEURISTIC;
  o->eta = 10.0f;
  o->block_size = 512;
  o->blocks_per_cu = 0;
  o->persistent = 1;
  o->wide_slices = 0;
  o->prefilter = 1;
  o->async = 0;
  o->msbfs_width = 512;
  o->random_seed = 1;
  o->device = -1;
  o->single_block = 1;
  o->panel = 1;
  o->stage2_count_first = 1;
  o->update_scheme = BLEST_UPDATE_AUTO;
}

blest_status blest_build(const blest_csr* csr, const blest_opts* opts_in, blest_graph** out) {
  if (!csr || !out) return fail(BLEST_ERR_INVALID_ARG, "NULL csr or out");
  *out = nullptr;
  blest_opts o;
  blest_default_opts(&o);
  if (opts_in) o = *opts_in;
  if (o.sigma != 8 && o.sigma != 16 && o.sigma != 32) return fail(BLEST_ERR_UNSUPPORTED, "sigma must be 8, 16 or 32");
  if (o.tau != 64 && o.tau != 128 && o.tau != 192 && o.tau != 256)
    return fail(BLEST_ERR_UNSUPPORTED, "tau must be 64, 128, 192 or 256");
  if (o.block_size != 256 && o.block_size != 512 && o.block_size != 1024)
    return fail(BLEST_ERR_UNSUPPORTED, "block_size must be 256, 512 or 1024");
  if (o.policy < BLEST_POLICY_HEURISTIC || o.policy > BLEST_POLICY_RANDOM)
    return fail(BLEST_ERR_INVALID_ARG, "unknown policy");
  if (o.reorder < BLEST_REORDER_NONE || o.reorder > BLEST_REORDER_JACCARD)
    return fail(BLEST_ERR_INVALID_ARG, "unknown reorder mode");
  if (o.jaccard_window < 0 || (o.jaccard_window != 0 && (o.jaccard_window <= o.sigma || o.jaccard_window % o.sigma)))
    return fail(BLEST_ERR_INVALID_ARG, "jaccard_window must be 0 or a multiple of sigma greater than sigma");
  if (!(o.eta >= 0.0f)) return fail(BLEST_ERR_INVALID_ARG, "eta must be >= 0");
  if (o.msbfs_width != 64 && o.msbfs_width != 128 && o.msbfs_width != 256 && o.msbfs_width != 512)
    return fail(BLEST_ERR_UNSUPPORTED, "msbfs_width must be 64, 128, 256 or 512");
  if (o.panel < 0 || o.panel > 2) return fail(BLEST_ERR_INVALID_ARG, "panel must be 0, 1 or 2");
  if (o.msbfs_graph < 0 || o.msbfs_graph > 1) return fail(BLEST_ERR_INVALID_ARG, "msbfs_graph must be 0 or 1");
  if (o.stage2_count_first < 0 || o.stage2_count_first > 2)
    return fail(BLEST_ERR_INVALID_ARG, "stage2_count_first must be 0, 1 or 2");
  if (o.directed < 0 || o.directed > 1) return fail(BLEST_ERR_INVALID_ARG, "directed must be 0 or 1");
  if (o.ms_mfma < 0 || o.ms_mfma > 1) return fail(BLEST_ERR_INVALID_ARG, "ms_mfma must be 0 or 1");
  if ((o.ms_mfma || o.ms_ablation) && o.sigma != 8)
    return fail(BLEST_ERR_UNSUPPORTED, "ms_mfma and ms_ablation need sigma = 8");
  if (o.ms_ablation < 0 || o.ms_ablation > (BLEST_MS_NO_GETVI | BLEST_MS_NO_DIRTY))
    return fail(BLEST_ERR_INVALID_ARG, "ms_ablation must combine BLEST_MS_NO_GETVI and BLEST_MS_NO_DIRTY");
  if (o.update_scheme < BLEST_UPDATE_LAZY || o.update_scheme > BLEST_UPDATE_AUTO)
    return fail(BLEST_ERR_INVALID_ARG, "update_scheme must be 0 (lazy), 1 (eager) or 2 (auto)");
  if (o.panel_log2_rows != 0 && (o.panel_log2_rows < 5 || o.panel_log2_rows > 15))
    return fail(BLEST_ERR_UNSUPPORTED, "panel_log2_rows must be 0 (auto) or in [5, 15]");
  const int64_t n = csr->n, m = csr->m;
  std::string why;
  if (!blest::validate_csr(n, m, csr->row_ptr, csr->col_idx, &why, o.directed == 0))
    return fail(BLEST_ERR_INVALID_GRAPH, why);
  int dev = 0, num_cu = 0;
  double tick_us = 0.01;
  blest_status s = check_device(o.device, &dev, &num_cu, &tick_us);
  if (s != BLEST_OK) return s;

  blest_graph* g = new (std::nothrow) blest_graph;
  if (!g) return fail(BLEST_ERR_OOM, "host allocation");
  g->opts = o;
  const int32_t* rp = csr->row_ptr;
  const int32_t* col = csr->col_idx;
  std::vector<int32_t> rp2, col2, orig, rps, cols;
  // The orderings work on the undirected graph underlying a directed one.
  const bool want_order = o.reorder != BLEST_REORDER_NONE && n > 1;
  if (o.directed && want_order) {
    try {
      blest::symmetrize_csr(n, rp, col, rps, cols);
    } catch (...) {
      delete g;
      return fail(BLEST_ERR_OOM, "host allocation during reordering");
    }
  }
  const int32_t* ord_rp = o.directed && want_order ? rps.data() : rp;
  const int32_t* ord_col = o.directed && want_order ? cols.data() : col;
  // AUTO follows the section "Reordering the Graph": JaccardWithWindows for
  // scale-free-like degree distributions, RCM for the others.
  const bool scale_free = o.reorder == BLEST_REORDER_AUTO && blest::is_scale_free_like(n, ord_rp);
  const bool rcm = o.reorder == BLEST_REORDER_RCM || (o.reorder == BLEST_REORDER_AUTO && !scale_free);
  const bool jac = o.reorder == BLEST_REORDER_JACCARD || scale_free;
  if ((rcm || jac) && n > 1) {
    try {
      if (rcm) {
        orig = blest::rcm_order(n, ord_rp, ord_col);
      } else {
        const std::vector<int32_t> nof =
            blest::jaccard_order(n, ord_rp, ord_col, o.sigma, o.jaccard_window ? o.jaccard_window : 1024);
        orig.assign(static_cast<size_t>(n), 0);
        for (int64_t i = 0; i < n; ++i) orig[nof[i]] = static_cast<int32_t>(i);
      }
      blest::permute_csr(n, rp, col, orig, g->perm, rp2, col2);
    } catch (...) {
      delete g;
      return fail(BLEST_ERR_OOM, "host allocation during reordering");
    }
    rp = rp2.data();
    col = col2.data();
    g->reordered = rcm ? 1 : 3;
  }
  rps.clear();
  rps.shrink_to_fit();
  cols.clear();
  cols.shrink_to_fit();
  // in-arcs of a directed graph, for the bottom-up engines (Alg. 4 reads the CSR of the transpose)
  std::vector<int32_t> rpt, colt;
  if (o.directed) {
    try {
      blest::transpose_csr(n, rp, col, rpt, colt);
    } catch (...) {
      delete g;
      return fail(BLEST_ERR_OOM, "host allocation during the transpose");
    }
  }
  const bool wide = o.sigma != 8 || o.wide_slices || n > (int64_t(1) << 24);
  blest::Bvss b;
  blest::Panels pn;
  try {
    blest::build_bvss(n, rp, col, o.sigma, o.tau, wide, &b);
  } catch (...) {
    delete g;
    return fail(BLEST_ERR_OOM, "host allocation during BVSS build");
  }
  blest::DevGraph& d = g->d;
  d.device = dev;
  d.sigma = o.sigma;
  d.tau = o.tau;
  d.wide = wide ? 1 : 0;
  d.n = n;
  d.m = m;
  d.nsets = b.nsets;
  d.nvss = b.nvss;
  d.nslices = b.nslices;
  d.block = o.block_size;
  d.num_cu = num_cu;
  d.persistent = o.persistent;
  d.prefilter = o.prefilter;
  d.single_block = o.single_block;
  d.count_first = o.stage2_count_first;
  d.tick_us = tick_us;
  // the paper's dispatch between Alg. 2 and Alg. 3 (Section "Ablation Studies")
  d.u_div = blest::update_divergence(b, o.tau);
  d.eager = o.update_scheme == BLEST_UPDATE_EAGER ||
            (o.update_scheme == BLEST_UPDATE_AUTO && d.u_div <= blest::kEagerMaxUdiv);
  {
    hipError_t ge = blest::bfs_grid_size(d, 1, o.blocks_per_cu, &d.grid);
    if (ge == hipSuccess) ge = blest::bfs_grid_size_eager(d, o.blocks_per_cu, &d.grid_eager);
    if (ge != hipSuccess) {
      delete g;
      return hip_fail(ge, "bfs_grid_size");
    }
  }
  if (o.panel) {
    try {
      const int rb = o.panel_log2_rows ? o.panel_log2_rows : blest::panel_log2_rows(n, d.grid);
      blest::build_panels(n, b, rb, &pn);
    } catch (...) {
      delete g;
      return fail(BLEST_ERR_OOM, "host allocation during panel build");
    }
  }
  d.npanels = pn.npanels;
  d.nchunks = pn.nchunks;
  d.panel_rb = pn.rb;
  d.panel_mode = pn.npanels > 0 ? o.panel : 0;
  d.log_cap = 1 << 16;
  int64_t nheavy = 0;
  for (int64_t u = 0; u < n; ++u) {
    int32_t dg = rp[u + 1] - rp[u];
    if (dg > blest::kLightMax) nheavy += (dg + blest::kHeavyChunk - 1) / blest::kHeavyChunk;
  }
  d.nheavy_cap = std::max<int64_t>(nheavy, 1);
  const size_t mb = static_cast<size_t>(o.sigma / 8);  // bytes per sigma-bit word
  const size_t ns = static_cast<size_t>(b.nsets);
  hipError_t e = hipSuccess;
#define TRY(expr)                 \
  do {                            \
    e = (expr);                   \
    if (e != hipSuccess) {        \
      release(g);                 \
      delete g;                   \
      return hip_fail(e, #expr);  \
    }                             \
  } while (0)
  // rp is padded to N_s*sigma + 1 entries (tail = m) so a slice set's row
  // pointers can be read with aligned 16-byte loads.
  // The fused panel step also reads whole 32-row groups (33 entries) and the
  // 5 slice pointers of their 4 sets, hence the extra padding of both.
  const size_t rp_len = static_cast<size_t>(b.nsets) * o.sigma + 1;
  TRY(dalloc_t(g, &d.rp, rp_len + 32));
  // col is padded by 4 entries: the bottom-up engine reads 4 neighbours at a time
  TRY(dalloc_t(g, &d.col, static_cast<size_t>(m) + 4));
  d.directed = o.directed;
  d.ms_ablation = o.ms_ablation;
  d.ms_mfma = o.ms_mfma;
  if (o.directed) {
    int32_t* rpi = nullptr;
    int32_t* coli = nullptr;
    void* dmi = nullptr;
    TRY(dalloc_t(g, &rpi, rp_len + 32));
    TRY(dalloc_t(g, &coli, static_cast<size_t>(m) + 4));
    TRY(dalloc(g, &dmi, ns * mb));
    std::vector<int32_t> rpp(rp_len + 4, static_cast<int32_t>(m));
    std::copy(rpt.begin(), rpt.end(), rpp.begin());
    TRY(hipMemcpy(rpi, rpp.data(), sizeof(int32_t) * rpp.size(), hipMemcpyHostToDevice));
    if (m > 0) TRY(hipMemcpy(coli, colt.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice));
    std::vector<uint8_t> dm(ns * mb, 0);
    for (int64_t u = 0; u < n; ++u)
      if (rpt[u + 1] > rpt[u]) dm[(u / o.sigma) * mb + (u % o.sigma) / 8] |= static_cast<uint8_t>(1u << (u % 8));
    TRY(hipMemcpy(dmi, dm.data(), dm.size(), hipMemcpyHostToDevice));
    d.rp_in = rpi;
    d.col_in = coli;
    d.degmask_in = dmi;
  }
  TRY(dalloc_t(g, &d.slice_ptr, ns + 8));
  TRY(dalloc(g, &d.slices, static_cast<size_t>(std::max<int64_t>(b.nslices, 1)) * (wide ? 8 : 4)));
  TRY(dalloc(g, &d.degmask, ns * mb));
  // The panel engine reads visited words and writes mark bytes in whole
  // 32-row groups up to the end of the last panel.
  const size_t prow = static_cast<size_t>(pn.npanels) << pn.rb;
  // 512 bytes of slack: a wave reads a chunk's frontier window as 64 8-byte
  // words starting at its first set (rounded down to 8).
  const size_t state_bytes = std::max(ns * mb, prow / 8) + 512;
  const size_t mark_bytes = std::max(ns * static_cast<size_t>(o.sigma), prow);
  // the frontier is double-buffered by level parity in the lazy scheme: level
  // l reads buffer l & 1 while Stage 2 (or the fused panel step) writes the
  // other; the eager scheme rotates three buffers (level mod 3)
  const size_t fstride = (state_bytes + 255) / 256 * 256;
  TRY(dalloc(g, &d.vis, state_bytes));
  TRY(dalloc(g, &d.front, 3 * fstride));
  TRY(hipMemset(d.vis, 0, state_bytes));
  TRY(hipMemset(d.front, 0, 3 * fstride));
  d.fstride = fstride;
  TRY(dalloc_t(g, &d.mark, mark_bytes));
  d.mark_bytes = mark_bytes;
  if (pn.npanels > 0) {
    TRY(dalloc_t(g, &d.pwords, pn.words.size()));
    TRY(dalloc_t(g, &d.pbase, pn.base.size() + blest::kPanelBasePad));
    TRY(dalloc_t(g, &d.pptr, pn.ptr.size()));
    TRY(hipMemcpy(d.pwords, pn.words.data(), 4 * pn.words.size(), hipMemcpyHostToDevice));
    TRY(hipMemcpy(d.pbase, pn.base.data(), 4 * pn.base.size(), hipMemcpyHostToDevice));
    TRY(hipMemset(d.pbase + pn.base.size(), 0, 4 * blest::kPanelBasePad));
    TRY(hipMemcpy(d.pptr, pn.ptr.data(), 4 * pn.ptr.size(), hipMemcpyHostToDevice));
  }
  TRY(dalloc_t(g, &d.queue[2], static_cast<size_t>(std::max<int64_t>(b.nvss, 1))));
  for (int i = 0; i < 2; ++i) {
    TRY(dalloc_t(g, &d.queue[i], static_cast<size_t>(std::max<int64_t>(b.nvss, 1))));
    TRY(dalloc_t(g, &d.flight[i], static_cast<size_t>(n)));
    TRY(dalloc_t(g, &d.fheavy[i], static_cast<size_t>(d.nheavy_cap)));
  }
  TRY(dalloc_t(g, &d.ctl, 1));
  TRY(dalloc_t(g, &d.part, static_cast<size_t>(d.grid) * 8));
  TRY(dalloc_t(g, &d.log, static_cast<size_t>(d.log_cap)));
  TRY(dalloc_t(g, &d.mlp, 1));
  TRY(dalloc_t(g, &d.ms_mlp, 1));
  if (g->reordered) {
    TRY(dalloc_t(g, &d.orig_id, static_cast<size_t>(n)));
    TRY(hipMemcpy(d.orig_id, orig.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
  }
  TRY(hipHostMalloc(reinterpret_cast<void**>(&d.host_flags), 64, hipHostMallocDefault));
  {
    std::vector<int32_t> rpp(rp_len + 4, static_cast<int32_t>(m));
    std::copy(rp, rp + n + 1, rpp.begin());
    TRY(hipMemcpy(d.rp, rpp.data(), sizeof(int32_t) * rpp.size(), hipMemcpyHostToDevice));
  }
  if (m > 0) TRY(hipMemcpy(d.col, col, sizeof(int32_t) * m, hipMemcpyHostToDevice));
  TRY(hipMemcpy(d.slice_ptr, b.slice_ptr.data(), sizeof(uint32_t) * (ns + 1), hipMemcpyHostToDevice));
  if (b.nslices > 0) {
    if (wide)
      TRY(hipMemcpy(d.slices, b.slices64.data(), 8 * b.nslices, hipMemcpyHostToDevice));
    else
      TRY(hipMemcpy(d.slices, b.slices32.data(), 4 * b.nslices, hipMemcpyHostToDevice));
  }
  {
    std::vector<uint8_t> dm(ns * mb);
    for (size_t s2 = 0; s2 < ns; ++s2) std::memcpy(&dm[s2 * mb], &b.degmask[s2], mb);  // little endian
    TRY(hipMemcpy(d.degmask, dm.data(), dm.size(), hipMemcpyHostToDevice));
  }
  TRY(hipMemset(d.mark, 0, mark_bytes));
  TRY(hipMemset(d.ctl, 0, sizeof(blest::Ctl)));
  TRY(hipMemset(d.mlp, 0, sizeof(blest::MlpDev)));
  TRY(hipMemset(d.ms_mlp, 0, sizeof(blest::MlpDev)));
  {
    std::lock_guard<std::mutex> lk(g_model_mu);
    if (g_model_set) TRY(hipMemcpy(d.mlp, &g_model, sizeof(g_model), hipMemcpyHostToDevice));
    if (g_ms_model_set) TRY(hipMemcpy(d.ms_mlp, &g_ms_model, sizeof(g_ms_model), hipMemcpyHostToDevice));
  }
  if (!o.directed) {
    d.rp_in = d.rp;
    d.col_in = d.col;
    d.degmask_in = d.degmask;
  }
  TRY(hipDeviceSynchronize());
#undef TRY
  g->real_ptrs = std::move(b.real_ptrs);
  g->slice_ptr = std::move(b.slice_ptr);
  g->csr_bytes = 4 * (n + 1) + 4 * m;
  g->bvss_bytes = 4 * static_cast<int64_t>(ns + 1) + (wide ? 8 : 4) * b.nslices +
                  4 * static_cast<int64_t>(pn.words.size() + pn.base.size() + pn.ptr.size());
  g->work_bytes = static_cast<int64_t>(ns * mb * 4 + ns * o.sigma) + 3 * 16 * std::max<int64_t>(b.nvss, 1) +
                  2 * 4 * n + 2 * 8 * d.nheavy_cap;
  g->ms.device = dev;
  *out = g;
  return BLEST_OK;
}

void blest_free(blest_graph* g) {
  if (!g) return;
  (void)hipSetDevice(g->d.device);
  (void)hipDeviceSynchronize();
  release(g);
  delete g;
}

blest_status blest_bfs(blest_graph* g, int32_t src, int32_t* levels_dev, void* stream) {
  return bfs_common(g, src, levels_dev, stream, 0);
}

blest_status blest_bfs_probe(blest_graph* g, int32_t src, int32_t* levels_dev, void* stream) {
  return bfs_common(g, src, levels_dev, stream, 1);
}

blest_status blest_sync(blest_graph* g, void* stream) {
  if (!g) return fail(BLEST_ERR_INVALID_ARG, "NULL graph");
  CK(hipSetDevice(g->d.device));
  return wait_and_check(g, static_cast<hipStream_t>(stream));
}

blest_status blest_set_policy(blest_graph* g, int32_t policy, float eta, uint64_t seed) {
  if (!g) return fail(BLEST_ERR_INVALID_ARG, "NULL graph");
  if (policy < BLEST_POLICY_HEURISTIC || policy > BLEST_POLICY_RANDOM) return fail(BLEST_ERR_INVALID_ARG, "unknown policy");
  if (!(eta >= 0.0f)) return fail(BLEST_ERR_INVALID_ARG, "eta must be >= 0");
  g->opts.policy = policy;
  g->opts.eta = eta;
  g->opts.random_seed = seed;
  return BLEST_OK;
}

blest_status blest_graph_info(const blest_graph* g, blest_graph_stats* out) {
  if (!g || !out) return fail(BLEST_ERR_INVALID_ARG, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  out->n = g->d.n;
  out->m = g->d.m;
  out->sigma = g->d.sigma;
  out->tau = g->d.tau;
  out->slice_bytes = g->d.wide ? 8 : 4;
  out->reordered = g->reordered;
  out->n_slice_sets = g->d.nsets;
  out->n_vss = g->d.nvss;
  out->n_slices = g->d.nslices;
  out->bvss_bytes = g->bvss_bytes;
  out->csr_bytes = g->csr_bytes;
  out->work_bytes = g->work_bytes;
  out->grid_blocks = g->d.grid;
  out->block_size = g->d.block;
  out->device = g->d.device;
  out->panel_log2_rows = g->d.npanels > 0 ? g->d.panel_rb : 0;
  out->update_scheme = g->d.eager ? BLEST_UPDATE_EAGER : BLEST_UPDATE_LAZY;
  out->directed = g->d.directed;
  out->ms_graph_captures = static_cast<int32_t>(g->ms.gcaptures);
  out->u_div = g->d.u_div;
  return BLEST_OK;
}

blest_status blest_update_divergence(const blest_csr* csr, int32_t sigma, int32_t tau, double* u_div) {
  if (!csr || !u_div) return fail(BLEST_ERR_INVALID_ARG, "NULL argument");
  if (sigma != 8 && sigma != 16 && sigma != 32) return fail(BLEST_ERR_UNSUPPORTED, "sigma must be 8, 16 or 32");
  if (tau != 64 && tau != 128 && tau != 192 && tau != 256)
    return fail(BLEST_ERR_UNSUPPORTED, "tau must be 64, 128, 192 or 256");
  std::string why;
  if (!blest::validate_csr(csr->n, csr->m, csr->row_ptr, csr->col_idx, &why))
    return fail(BLEST_ERR_INVALID_GRAPH, why);
  try {
    blest::Bvss b;
    blest::build_bvss(csr->n, csr->row_ptr, csr->col_idx, sigma, tau, true, &b);
    *u_div = blest::update_divergence(b, tau);
  } catch (...) {
    return fail(BLEST_ERR_OOM, "host allocation during the BVSS build");
  }
  return BLEST_OK;
}

blest_status blest_reorder_jaccard(const blest_csr* csr, int32_t sigma, int32_t window, int32_t* new_of_old) {
  if (!csr || !new_of_old) return fail(BLEST_ERR_INVALID_ARG, "NULL argument");
  if (sigma < 1 || window <= sigma || window % sigma != 0)
    return fail(BLEST_ERR_INVALID_ARG, "window must be a multiple of sigma greater than sigma");
  std::string why;
  if (!blest::validate_csr(csr->n, csr->m, csr->row_ptr, csr->col_idx, &why))
    return fail(BLEST_ERR_INVALID_GRAPH, why);
  try {
    const std::vector<int32_t> nof = blest::jaccard_order(csr->n, csr->row_ptr, csr->col_idx, sigma, window);
    std::memcpy(new_of_old, nof.data(), sizeof(int32_t) * nof.size());
  } catch (...) {
    return fail(BLEST_ERR_OOM, "host allocation during reordering");
  }
  return BLEST_OK;
}

blest_status blest_last_level_stats(const blest_graph* g, blest_level_stat* buf, int32_t cap, int32_t* nlevels) {
  if (!g || !nlevels || (cap > 0 && !buf)) return fail(BLEST_ERR_INVALID_ARG, "NULL argument");
  *nlevels = g->nlevels;
  const int k = std::min({cap, g->nlevels, g->d.log_cap});
  if (k <= 0) return BLEST_OK;
  std::vector<blest::LevelRec> rec(static_cast<size_t>(k));
  CK(hipSetDevice(g->d.device));
  CK(hipMemcpy(rec.data(), g->d.log, sizeof(blest::LevelRec) * k, hipMemcpyDeviceToHost));
  for (int i = 0; i < k; ++i) {
    const blest::LevelRec& r = rec[i];
    blest_level_stat& o = buf[i];
    std::memset(&o, 0, sizeof(o));
    o.level = i;
    o.engine = (i == g->nlevels - 1) ? -1 : r.engine;
    o.frontier = r.frontier;
    o.queue = r.queue;
    o.queue_slices = r.qslices;
    o.frontier_edges = r.fedges;
    o.unvisited = r.unvisited;
    o.unvisited_edges = r.unvisited_edges;
    o.deg_ge_32 = r.deg32;
    o.deg_ge_1024 = r.deg1024;
    o.t_step_us = r.t_end > r.t_begin ? (r.t_end - r.t_begin) * g->d.tick_us : 0.0;
    o.t_stage1_us = r.t_mid > r.t_begin ? (r.t_mid - r.t_begin) * g->d.tick_us : 0.0;
    o.t_count_us = r.t_count > r.t_begin ? (r.t_count - r.t_begin) * g->d.tick_us : 0.0;
    for (int e = 0; e < 3; ++e) o.t_engine_us[e] = r.t_engine[e] ? r.t_engine[e] * g->d.tick_us : -1.0;
    o.mlp_fallback = r.fallback;
    o.bvss_panel = r.panel;
    o.work = r.work;
  }
  return BLEST_OK;
}

blest_status blest_last_level_features(const blest_graph* g, float* feat, int32_t cap, int32_t* nlevels) {
  if (!g || !nlevels || (cap > 0 && !feat)) return fail(BLEST_ERR_INVALID_ARG, "NULL argument");
  *nlevels = g->nlevels;
  const int k = std::min({cap, g->nlevels, g->d.log_cap});
  if (k <= 0) return BLEST_OK;
  std::vector<blest::LevelRec> rec(static_cast<size_t>(k));
  CK(hipSetDevice(g->d.device));
  CK(hipMemcpy(rec.data(), g->d.log, sizeof(blest::LevelRec) * k, hipMemcpyDeviceToHost));
  for (int i = 0; i < k; ++i) std::memcpy(feat + i * BLEST_MLP_IN, rec[i].feat, sizeof(float) * BLEST_MLP_IN);
  return BLEST_OK;
}

blest_status blest_export_bvss(const blest_graph* g, int64_t* real_ptrs, int64_t* v2r, int64_t* slice_ptr,
                               int32_t* slice_row, uint64_t* slice_mask, int32_t* perm) {
  if (!g) return fail(BLEST_ERR_INVALID_ARG, "NULL graph");
  const int64_t ns = g->d.nsets;
  if (real_ptrs) std::copy(g->real_ptrs.begin(), g->real_ptrs.end(), real_ptrs);
  if (v2r)
    for (int64_t s = 0; s < ns; ++s)
      for (int64_t v = g->real_ptrs[s]; v < g->real_ptrs[s + 1]; ++v) v2r[v] = s;
  if (slice_ptr)
    for (int64_t s = 0; s <= ns; ++s) slice_ptr[s] = g->slice_ptr[s];
  if ((slice_row || slice_mask) && g->d.nslices > 0) {
    CK(hipSetDevice(g->d.device));
    const int64_t k = g->d.nslices;
    if (g->d.wide) {
      std::vector<uint64_t> w(static_cast<size_t>(k));
      CK(hipMemcpy(w.data(), g->d.slices, 8 * k, hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < k; ++i) {
        if (slice_row) slice_row[i] = static_cast<int32_t>(w[i] >> 32);
        if (slice_mask) slice_mask[i] = w[i] & 0xffffffffULL;
      }
    } else {
      std::vector<uint32_t> w(static_cast<size_t>(k));
      CK(hipMemcpy(w.data(), g->d.slices, 4 * k, hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < k; ++i) {
        if (slice_row) slice_row[i] = static_cast<int32_t>(w[i] >> 8);
        if (slice_mask) slice_mask[i] = w[i] & 0xffu;
      }
    }
  }
  if (perm) {
    if (g->perm.empty())
      for (int64_t i = 0; i < g->d.n; ++i) perm[i] = static_cast<int32_t>(i);
    else
      std::copy(g->perm.begin(), g->perm.end(), perm);
  }
  return BLEST_OK;
}

namespace {

// Validates and packs switch-network weights (the same format for both networks).
blest_status make_model(const float* params, int32_t nparams, const float* mean, const float* std_,
                        blest::MlpDev* out) {
  if (!params || !mean || !std_) return fail(BLEST_ERR_INVALID_ARG, "NULL argument");
  if (nparams != BLEST_MLP_NPARAMS) return fail(BLEST_ERR_INVALID_ARG, "wrong parameter count");
  blest::MlpDev m{};
  std::memcpy(m.params, params, sizeof(m.params));
  for (int i = 0; i < BLEST_MLP_IN; ++i) {
    if (!(std_[i] > 0.0f) || !std::isfinite(std_[i]) || !std::isfinite(mean[i]))
      return fail(BLEST_ERR_INVALID_ARG, "feature std must be positive and finite");
    m.mean[i] = mean[i];
    m.inv_std[i] = 1.0f / std_[i];
  }
  for (int i = 0; i < BLEST_MLP_NPARAMS; ++i)
    if (!std::isfinite(params[i])) return fail(BLEST_ERR_INVALID_ARG, "non-finite parameter");
  {
    std::lock_guard<std::mutex> lk(g_model_mu);
    m.max_ratio = 1.0f / g_min_conf;
  }
  m.valid = 1;
  *out = m;
  return BLEST_OK;
}

}  // namespace

blest_status blest_set_ms_switch_model(blest_graph* g, const float* params, int32_t nparams, const float* mean,
                                       const float* std_) {
  blest::MlpDev m{};
  const blest_status s = make_model(params, nparams, mean, std_, &m);
  if (s != BLEST_OK) return s;
  if (!g) {
    std::lock_guard<std::mutex> lk(g_model_mu);
    g_ms_model = m;
    g_ms_model_set = true;
    return BLEST_OK;
  }
  CK(hipSetDevice(g->d.device));
  CK(hipMemcpy(g->d.ms_mlp, &m, sizeof(m), hipMemcpyHostToDevice));
  return BLEST_OK;
}

blest_status blest_set_switch_model(blest_graph* g, const float* params, int32_t nparams, const float* mean,
                                    const float* std_) {
  blest::MlpDev m{};
  const blest_status s = make_model(params, nparams, mean, std_, &m);
  if (s != BLEST_OK) return s;
  if (!g) {
    std::lock_guard<std::mutex> lk(g_model_mu);
    g_model = m;
    g_model_set = true;
    return BLEST_OK;
  }
  CK(hipSetDevice(g->d.device));
  CK(hipMemcpy(g->d.mlp, &m, sizeof(m), hipMemcpyHostToDevice));
  return BLEST_OK;
}

blest_status blest_set_switch_confidence(blest_graph* g, float min_prob) {
  if (!(min_prob > 0.0f && min_prob <= 1.0f)) return fail(BLEST_ERR_INVALID_ARG, "min_prob must be in (0, 1]");
  const float r = 1.0f / min_prob;
  if (!g) {
    std::lock_guard<std::mutex> lk(g_model_mu);
    g_min_conf = min_prob;
    g_model.max_ratio = r;
    g_ms_model.max_ratio = r;
    return BLEST_OK;
  }
  CK(hipSetDevice(g->d.device));
  CK(hipMemcpy(reinterpret_cast<char*>(g->d.mlp) + offsetof(blest::MlpDev, max_ratio), &r, sizeof(float),
               hipMemcpyHostToDevice));
  CK(hipMemcpy(reinterpret_cast<char*>(g->d.ms_mlp) + offsetof(blest::MlpDev, max_ratio), &r, sizeof(float),
               hipMemcpyHostToDevice));
  return BLEST_OK;
}

blest_status blest_set_log_work(blest_graph* g, int32_t on) {
  if (!g) return fail(BLEST_ERR_INVALID_ARG, "NULL graph");
  g->d.count_work = on ? 1 : 0;
  return BLEST_OK;
}

blest_status blest_msbfs(blest_graph* g, const int32_t* srcs, int32_t k, int16_t* levels_dev, void* stream) {
  if (!g) return fail(BLEST_ERR_INVALID_ARG, "NULL graph");
  if (k < 0) return fail(BLEST_ERR_INVALID_ARG, "negative source count");
  if (k == 0) return BLEST_OK;
  if (!srcs || !levels_dev) return fail(BLEST_ERR_INVALID_ARG, "NULL sources or output");
  for (int32_t c = 0; c < k; ++c)
    if (srcs[c] < 0 || srcs[c] >= g->d.n) return fail(BLEST_ERR_OUT_OF_RANGE, "source vertex out of range");
  CK(hipSetDevice(g->d.device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<int32_t> internal(srcs, srcs + k);
  if (!g->perm.empty())
    for (auto& s : internal) s = g->perm[s];
  const int32_t w = g->opts.msbfs_width;
  hipError_t e = blest::ms_run(g->d, &g->ms, internal.data(), k, &w, 1, g->opts.policy, g->opts.eta,
                               g->opts.random_seed, levels_dev, nullptr, nullptr, nullptr, st, g->opts.msbfs_graph);
  if (e != hipSuccess) return hip_fail(e, "msbfs");
  if (g->opts.async) return BLEST_OK;
  return wait_and_check(g, st);
}

blest_status blest_msbfs_noalloc(blest_graph* g, const int32_t* srcs, int32_t k, int16_t* levels_dev, void* stream) {
  if (!g) return fail(BLEST_ERR_INVALID_ARG, "NULL graph");
  if (k < 0) return fail(BLEST_ERR_INVALID_ARG, "negative source count");
  if (k > BLEST_MSBFS_NOALLOC_MAX_SOURCES)
    return fail(BLEST_ERR_INVALID_ARG, "blest_msbfs_noalloc takes at most BLEST_MSBFS_NOALLOC_MAX_SOURCES (" +
                                           std::to_string(BLEST_MSBFS_NOALLOC_MAX_SOURCES) + ") sources per call");
  if (k == 0) return BLEST_OK;
  if (!srcs || !levels_dev) return fail(BLEST_ERR_INVALID_ARG, "NULL sources or output");
  for (int32_t c = 0; c < k; ++c)
    if (srcs[c] < 0 || srcs[c] >= g->d.n) return fail(BLEST_ERR_OUT_OF_RANGE, "source vertex out of range");
  CK(hipSetDevice(g->d.device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = blest::ms_run_noalloc(g->d, &g->ms, srcs, g->perm.empty() ? nullptr : g->perm.data(), k,
                                       g->opts.msbfs_width, g->opts.policy, g->opts.eta, g->opts.random_seed,
                                       levels_dev, st);
  if (e == hipErrorNotReady)
    return fail(BLEST_ERR_UNSUPPORTED,
                "the graph's multi-source buffers are not allocated yet: make one blest_msbfs call of this batch "
                "width on the graph first");
  if (e != hipSuccess) return hip_fail(e, "msbfs_noalloc");
  if (g->opts.async) return BLEST_OK;
  return wait_and_check(g, st);
}

blest_status blest_msbfs_batched(blest_graph* g, const int32_t* srcs, int32_t k, const int32_t* widths,
                                 int32_t nwidths, int16_t* levels_dev, void* stream) {
  if (!g) return fail(BLEST_ERR_INVALID_ARG, "NULL graph");
  if (k < 0 || nwidths < 1 || !widths) return fail(BLEST_ERR_INVALID_ARG, "bad source count or widths");
  for (int32_t i = 0; i < nwidths; ++i)
    if (widths[i] != 64 && widths[i] != 128 && widths[i] != 256 && widths[i] != 512)
      return fail(BLEST_ERR_UNSUPPORTED, "batch widths must be 64, 128, 256 or 512");
  if (k == 0) return BLEST_OK;
  if (!srcs || !levels_dev) return fail(BLEST_ERR_INVALID_ARG, "NULL sources or output");
  for (int32_t c = 0; c < k; ++c)
    if (srcs[c] < 0 || srcs[c] >= g->d.n) return fail(BLEST_ERR_OUT_OF_RANGE, "source vertex out of range");
  CK(hipSetDevice(g->d.device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<int32_t> internal(srcs, srcs + k);
  if (!g->perm.empty())
    for (auto& s : internal) s = g->perm[s];
  hipError_t e = blest::ms_run(g->d, &g->ms, internal.data(), k, widths, nwidths, g->opts.policy, g->opts.eta,
                               g->opts.random_seed, levels_dev, nullptr, nullptr, nullptr, st, g->opts.msbfs_graph);
  if (e != hipSuccess) return hip_fail(e, "msbfs");
  if (g->opts.async) return BLEST_OK;
  return wait_and_check(g, st);
}

blest_status blest_msbfs_probe(blest_graph* g, const int32_t* srcs, int32_t k, const int32_t* widths, int32_t nwidths,
                               int16_t* levels_dev, void* stream) {
  if (!g) return fail(BLEST_ERR_INVALID_ARG, "NULL graph");
  if (k < 0 || nwidths < 1 || !widths) return fail(BLEST_ERR_INVALID_ARG, "bad source count or widths");
  for (int32_t i = 0; i < nwidths; ++i)
    if (widths[i] != 64 && widths[i] != 128 && widths[i] != 256 && widths[i] != 512)
      return fail(BLEST_ERR_UNSUPPORTED, "batch widths must be 64, 128, 256 or 512");
  if (k == 0) return BLEST_OK;
  if (!srcs || !levels_dev) return fail(BLEST_ERR_INVALID_ARG, "NULL sources or output");
  for (int32_t c = 0; c < k; ++c)
    if (srcs[c] < 0 || srcs[c] >= g->d.n) return fail(BLEST_ERR_OUT_OF_RANGE, "source vertex out of range");
  CK(hipSetDevice(g->d.device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<int32_t> internal(srcs, srcs + k);
  if (!g->perm.empty())
    for (auto& s : internal) s = g->perm[s];
  hipError_t e = blest::ms_run(g->d, &g->ms, internal.data(), k, widths, nwidths, g->opts.policy, g->opts.eta,
                               g->opts.random_seed, levels_dev, nullptr, nullptr, nullptr, st, 0, nullptr, 1);
  if (e != hipSuccess) return hip_fail(e, "msbfs probe");
  return wait_and_check(g, st);
}

blest_status blest_msbfs_last_levels(const blest_graph* g, blest_ms_level_stat* buf, int32_t cap, int32_t* nrec) {
  if (!g || !nrec || (cap > 0 && !buf)) return fail(BLEST_ERR_INVALID_ARG, "NULL argument");
  CK(hipSetDevice(g->d.device));
  int n = 0;
  CK(hipMemcpy(&n, &g->d.ctl->ms_nrec[0], sizeof(int), hipMemcpyDeviceToHost));
  n = std::min(n, g->ms.log_cap);
  *nrec = n;
  const int k = std::min(cap, n);
  if (k <= 0 || !g->ms.log) return BLEST_OK;
  std::vector<blest::MsLevelRec> rec(static_cast<size_t>(k));
  CK(hipMemcpy(rec.data(), g->ms.log, sizeof(blest::MsLevelRec) * k, hipMemcpyDeviceToHost));
  for (int i = 0; i < k; ++i) {
    const blest::MsLevelRec& r = rec[i];
    blest_ms_level_stat& o = buf[i];
    std::memset(&o, 0, sizeof(o));
    o.batch = r.batch;
    o.level = r.level;
    o.engine = r.engine;
    o.mlp_fallback = r.fallback;
    o.width = r.width;
    o.live = r.live;
    o.new_pairs = r.fresh;
    o.queue = r.queue;
    o.queue_slices = r.qslices;
    o.unvisited_pairs = r.unvisited;
    for (int e = 0; e < 2; ++e) o.t_engine_us[e] = r.t_engine[e] ? r.t_engine[e] * g->d.tick_us : -1.0;
    std::memcpy(o.feat, r.feat, sizeof(o.feat));
  }
  return BLEST_OK;
}

blest_status blest_closeness(blest_graph* g, const int32_t* srcs, int64_t k, int64_t* sums_dev, int64_t* reach_dev,
                             double* cc_dev, void* stream) {
  if (!g) return fail(BLEST_ERR_INVALID_ARG, "NULL graph");
  if (k < 0 || k > INT32_MAX) return fail(BLEST_ERR_INVALID_ARG, "bad source count");
  if (k == 0) return BLEST_OK;
  if (!srcs) return fail(BLEST_ERR_INVALID_ARG, "NULL sources");
  for (int64_t c = 0; c < k; ++c)
    if (srcs[c] < 0 || srcs[c] >= g->d.n) return fail(BLEST_ERR_OUT_OF_RANGE, "source vertex out of range");
  CK(hipSetDevice(g->d.device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<int32_t> internal(srcs, srcs + k);
  if (!g->perm.empty())
    for (auto& s : internal) s = g->perm[s];
  const int32_t w = g->opts.msbfs_width;
  hipError_t e = blest::ms_run(g->d, &g->ms, internal.data(), static_cast<int32_t>(k), &w, 1, g->opts.policy,
                               g->opts.eta, g->opts.random_seed, nullptr, sums_dev, reach_dev, cc_dev, st,
                               g->opts.msbfs_graph);
  if (e != hipSuccess) return hip_fail(e, "closeness");
  if (g->opts.async) return BLEST_OK;
  return wait_and_check(g, st);
}

namespace {

// Checkpoint of a resumable closeness run: header, then sums[done], reach[done].
struct CcHeader {
  char magic[8];
  int64_t n, m, k;
  uint64_t src_hash;  // FNV-1a over the source list
  int64_t done;
};

uint64_t fnv1a(const int32_t* p, int64_t k) {
  uint64_t h = 1469598103934665603ULL;
  const unsigned char* b = reinterpret_cast<const unsigned char*>(p);
  for (int64_t i = 0; i < k * 4; ++i) h = (h ^ b[i]) * 1099511628211ULL;
  return h;
}

bool write_checkpoint(const std::string& path, const CcHeader& h, const std::vector<int64_t>& sums,
                      const std::vector<int64_t>& reach) {
  const std::string tmp = path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return false;
  bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1;
  if (h.done > 0) {
    ok = ok && std::fwrite(sums.data(), sizeof(int64_t), h.done, f) == static_cast<size_t>(h.done);
    ok = ok && std::fwrite(reach.data(), sizeof(int64_t), h.done, f) == static_cast<size_t>(h.done);
  }
  ok = (std::fclose(f) == 0) && ok;
  return ok && std::rename(tmp.c_str(), path.c_str()) == 0;
}

}  // namespace

blest_status blest_closeness_resumable(blest_graph* g, const int32_t* srcs, int64_t k, int64_t* sums_dev,
                                       int64_t* reach_dev, double* cc_dev, const char* path, int64_t max_sources,
                                       int64_t* done, void* stream) {
  if (!g || !path || !done) return fail(BLEST_ERR_INVALID_ARG, "NULL graph, path or done");
  if (k < 0 || k > INT32_MAX || max_sources < 0) return fail(BLEST_ERR_INVALID_ARG, "bad source count");
  *done = 0;
  if (k > 0 && !srcs) return fail(BLEST_ERR_INVALID_ARG, "NULL sources");
  for (int64_t c = 0; c < k; ++c)
    if (srcs[c] < 0 || srcs[c] >= g->d.n) return fail(BLEST_ERR_OUT_OF_RANGE, "source vertex out of range");
  CcHeader h{};
  std::memcpy(h.magic, "BLESTCC1", 8);
  h.n = g->d.n;
  h.m = g->d.m;
  h.k = k;
  h.src_hash = fnv1a(srcs, k);
  std::vector<int64_t> sums, reach;
  if (FILE* f = std::fopen(path, "rb")) {
    CcHeader r{};
    bool ok = std::fread(&r, sizeof(r), 1, f) == 1;
    if (ok && (std::memcmp(r.magic, h.magic, 8) != 0 || r.n != h.n || r.m != h.m || r.k != h.k ||
               r.src_hash != h.src_hash || r.done < 0 || r.done > k)) {
      std::fclose(f);
      return fail(BLEST_ERR_INVALID_ARG, "checkpoint file belongs to another graph or source list");
    }
    if (ok && r.done > 0) {
      sums.resize(r.done);
      reach.resize(r.done);
      ok = std::fread(sums.data(), sizeof(int64_t), r.done, f) == static_cast<size_t>(r.done) &&
           std::fread(reach.data(), sizeof(int64_t), r.done, f) == static_cast<size_t>(r.done);
    }
    std::fclose(f);
    if (!ok) return fail(BLEST_ERR_IO, "checkpoint file is truncated");
    h.done = r.done;
  }
  CK(hipSetDevice(g->d.device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (h.done > 0) {
    // results of the finished sources, cc as the kernels compute it
    std::vector<double> cc(h.done);
    for (int64_t c = 0; c < h.done; ++c)
      cc[c] = sums[c] ? static_cast<double>(reach[c] - 1) / static_cast<double>(sums[c]) : 0.0;
    if (sums_dev) CK(hipMemcpyAsync(sums_dev, sums.data(), sizeof(int64_t) * h.done, hipMemcpyHostToDevice, st));
    if (reach_dev) CK(hipMemcpyAsync(reach_dev, reach.data(), sizeof(int64_t) * h.done, hipMemcpyHostToDevice, st));
    if (cc_dev) CK(hipMemcpyAsync(cc_dev, cc.data(), sizeof(double) * h.done, hipMemcpyHostToDevice, st));
    CK(hipStreamSynchronize(st));
  }
  const int64_t chunk = static_cast<int64_t>(g->opts.msbfs_width) * 64;
  int64_t budget = max_sources > 0 ? max_sources : k;
  // device scratch for one chunk's sums and reach, so they can be saved
  int64_t* dsum = nullptr;
  int64_t* dreach = nullptr;
  const int64_t cap = std::min(chunk, std::max<int64_t>(k - h.done, 1));
  CK(hipMalloc(&dsum, sizeof(int64_t) * cap));
  if (hipMalloc(&dreach, sizeof(int64_t) * cap) != hipSuccess) {
    (void)hipFree(dsum);
    return fail(BLEST_ERR_OOM, "device scratch");
  }
  blest_status s = BLEST_OK;
  const int32_t saved_async = g->opts.async;
  g->opts.async = 0;
  while (h.done < k && budget > 0) {
    const int64_t c = std::min({chunk, k - h.done, budget});
    s = blest_closeness(g, srcs + h.done, c, dsum, dreach, cc_dev ? cc_dev + h.done : nullptr, stream);
    if (s != BLEST_OK) break;
    sums.resize(h.done + c);
    reach.resize(h.done + c);
    if (hipMemcpy(sums.data() + h.done, dsum, sizeof(int64_t) * c, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(reach.data() + h.done, dreach, sizeof(int64_t) * c, hipMemcpyDeviceToHost) != hipSuccess) {
      s = fail(BLEST_ERR_HIP, "copy of closeness results");
      break;
    }
    if ((sums_dev && hipMemcpy(sums_dev + h.done, dsum, sizeof(int64_t) * c, hipMemcpyDeviceToDevice) != hipSuccess) ||
        (reach_dev &&
         hipMemcpy(reach_dev + h.done, dreach, sizeof(int64_t) * c, hipMemcpyDeviceToDevice) != hipSuccess)) {
      s = fail(BLEST_ERR_HIP, "copy of closeness results");
      break;
    }
    h.done += c;
    budget -= c;
    if (!write_checkpoint(path, h, sums, reach)) {
      s = fail(BLEST_ERR_IO, std::string("cannot write checkpoint ") + path);
      break;
    }
  }
  g->opts.async = saved_async;
  (void)hipFree(dsum);
  (void)hipFree(dreach);
  *done = h.done;
  return s;
}

blest_status blest_far(blest_graph* g, const int32_t* srcs, int64_t k, int64_t* far_dev, void* stream) {
  if (!g) return fail(BLEST_ERR_INVALID_ARG, "NULL graph");
  if (k < 0 || k > INT32_MAX) return fail(BLEST_ERR_INVALID_ARG, "bad source count");
  if (!far_dev) return fail(BLEST_ERR_INVALID_ARG, "NULL output");
  if (k > 0 && !srcs) return fail(BLEST_ERR_INVALID_ARG, "NULL sources");
  for (int64_t c = 0; c < k; ++c)
    if (srcs[c] < 0 || srcs[c] >= g->d.n) return fail(BLEST_ERR_OUT_OF_RANGE, "source vertex out of range");
  CK(hipSetDevice(g->d.device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  CK(hipMemsetAsync(far_dev, 0, sizeof(int64_t) * static_cast<size_t>(g->d.n), st));
  if (k == 0) return g->opts.async ? BLEST_OK : wait_and_check(g, st);
  std::vector<int32_t> internal(srcs, srcs + k);
  if (!g->perm.empty())
    for (auto& s : internal) s = g->perm[s];
  const int32_t w = g->opts.msbfs_width;
  hipError_t e = blest::ms_run(g->d, &g->ms, internal.data(), static_cast<int32_t>(k), &w, 1, g->opts.policy,
                               g->opts.eta, g->opts.random_seed, nullptr, nullptr, nullptr, nullptr, st,
                               g->opts.msbfs_graph, far_dev);
  if (e != hipSuccess) return hip_fail(e, "far");
  if (g->opts.async) return BLEST_OK;
  return wait_and_check(g, st);
}

blest_status blest_mlp_forward(const float* params, const float* x, int32_t batch, float* logits, void* stream) {
  if (batch < 0) return fail(BLEST_ERR_INVALID_ARG, "negative batch");
  if (batch == 0) return BLEST_OK;
  if (!params || !x || !logits) return fail(BLEST_ERR_INVALID_ARG, "NULL argument");
  CK(blest::mlp_forward_launch(params, x, batch, logits, static_cast<hipStream_t>(stream)));
  return BLEST_OK;
}

blest_status blest_mlp_loss_grad(const float* params, const float* x, const int32_t* y, const float* w, int32_t batch,
                                 float* loss, float* grad, void* stream) {
  if (!params || !x || !y || !grad) return fail(BLEST_ERR_INVALID_ARG, "NULL argument");
  if (batch <= 0) return fail(BLEST_ERR_INVALID_ARG, "batch must be positive");
  CK(blest::mlp_loss_grad_launch(params, x, y, w, batch, loss, grad, static_cast<hipStream_t>(stream)));
  return BLEST_OK;
}

blest_status blest_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t n, int32_t t, float lr,
                            float beta1, float beta2, float eps, void* stream) {
  if (!params || !grad || !m || !v) return fail(BLEST_ERR_INVALID_ARG, "NULL argument");
  if (n <= 0 || t < 1) return fail(BLEST_ERR_INVALID_ARG, "n must be positive and t >= 1");
  CK(blest::mlp_adam_launch(params, grad, m, v, n, t, lr, beta1, beta2, eps, static_cast<hipStream_t>(stream)));
  return BLEST_OK;
}

blest_status blest_mlp_train(float* params, float* m, float* v, const float* x, const int32_t* y, const float* w,
                             int32_t nsamples, int32_t batch, int32_t steps, float lr, uint64_t seed, float* loss_log,
                             void* stream) {
  if (!params || !m || !v || !x || !y) return fail(BLEST_ERR_INVALID_ARG, "NULL argument");
  if (nsamples <= 0 || batch <= 0 || steps < 0) return fail(BLEST_ERR_INVALID_ARG, "bad sizes");
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* grad = nullptr;
  CK(hipMallocAsync(reinterpret_cast<void**>(&grad), sizeof(float) * BLEST_MLP_NPARAMS, st));
  hipError_t e = blest::mlp_train_launch(params, m, v, x, y, w, nsamples, batch, steps, lr, seed, loss_log, grad, st);
  hipError_t e2 = hipFreeAsync(grad, st);
  if (e != hipSuccess) return hip_fail(e, "mlp training");
  if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
  return BLEST_OK;
}

}  // extern "C"
