// Host-side preprocessing: CSR validation, reordering and BVSS construction.
//
// BVSS (Section "Binarized Virtual Slice Sets"): the columns of the
// transposed adjacency A (A[i][j] = 1 iff edge (j, i)) are cut into slice
// sets of sigma consecutive columns. Row i owns a slice in set s iff it has a
// nonzero in those columns; the slice's mask has bit b set iff A[i][s*sigma+b]
// is 1. Slices of a set are stored in ascending row order, and the set is
// split into virtual slice sets of at most tau slices. For an undirected
// graph the rows of set s are the union of the neighbour lists of its sigma
// vertices, so each set is a sigma-way merge of sorted CSR rows.
//
// Reordering (Section "Reordering the Graph"): Reverse Cuthill-McKee for
// graphs that are not scale-free-like, by the degree-share / log-log test in
// that section's footnote.
#include "host_build.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <iterator>
#include <numeric>
#include <thread>

namespace blest {

namespace {

int host_threads() {
  unsigned h = std::thread::hardware_concurrency();
  if (h == 0) h = 4;
  return static_cast<int>(std::min<unsigned>(h, 16));
}

template <class F>
void parallel_for(int64_t n, F&& f) {
  const int t = host_threads();
  if (n < 8192 || t <= 1) {
    f(int64_t(0), n);
    return;
  }
  std::vector<std::thread> pool;
  const int64_t chunk = (n + t - 1) / t;
  for (int i = 0; i < t; ++i) {
    const int64_t b = i * chunk, e = std::min<int64_t>(n, b + chunk);
    if (b >= e) break;
    pool.emplace_back([=, &f] { f(b, e); });
  }
  for (auto& th : pool) th.join();
}

}  // namespace

bool validate_csr(int64_t n, int64_t m, const int32_t* rp, const int32_t* col, std::string* why, bool symmetric) {
  if (n <= 0 || n > INT32_MAX - 1) return *why = "n must be in [1, 2^31-1)", false;
  if (m < 0 || m >= (int64_t(1) << 31)) return *why = "m must be in [0, 2^31)", false;
  if (!rp || (m > 0 && !col)) return *why = "NULL CSR array", false;
  if (rp[0] != 0 || rp[n] != m) return *why = "row_ptr[0] must be 0 and row_ptr[n] must be m", false;
  std::atomic<int> bad{0};
  std::atomic<int64_t> where{-1};
  parallel_for(n, [&](int64_t b, int64_t e) {
    for (int64_t u = b; u < e && !bad.load(std::memory_order_relaxed); ++u) {
      const int64_t lo = rp[u], hi = rp[u + 1];
      if (hi < lo) { bad = 1; where = u; return; }
      for (int64_t p = lo; p < hi; ++p) {
        const int32_t v = col[p];
        if (v < 0 || v >= n) { bad = 2; where = u; return; }
        if (v == u) { bad = 3; where = u; return; }
        if (p > lo && col[p - 1] >= v) { bad = 4; where = u; return; }
        if (!symmetric) continue;
        // symmetric: u must appear in row v
        const int32_t* first = col + rp[v];
        const int32_t* last = col + rp[v + 1];
        if (!std::binary_search(first, last, static_cast<int32_t>(u))) { bad = 5; where = u; return; }
      }
    }
  });
  static const char* msg[] = {"", "row_ptr decreases", "column index out of range", "self loop",
                              "row not strictly ascending (unsorted or duplicate)", "graph is not symmetric"};
  if (bad) {
    *why = std::string(msg[bad.load()]) + " at vertex " + std::to_string(where.load());
    return false;
  }
  return true;
}

void transpose_csr(int64_t n, const int32_t* rp, const int32_t* col, std::vector<int32_t>& rpt,
                   std::vector<int32_t>& colt) {
  rpt.assign(static_cast<size_t>(n) + 1, 0);
  for (int64_t p = 0; p < rp[n]; ++p) ++rpt[col[p] + 1];
  for (int64_t v = 0; v < n; ++v) rpt[v + 1] += rpt[v];
  colt.resize(static_cast<size_t>(rp[n]));
  std::vector<int32_t> next(rpt.begin(), rpt.end() - 1);
  // sources in ascending order, so every transposed row comes out sorted
  for (int64_t u = 0; u < n; ++u)
    for (int32_t p = rp[u]; p < rp[u + 1]; ++p) colt[next[col[p]]++] = static_cast<int32_t>(u);
}

void symmetrize_csr(int64_t n, const int32_t* rp, const int32_t* col, std::vector<int32_t>& rps,
                    std::vector<int32_t>& cols) {
  std::vector<int32_t> rpt, colt;
  transpose_csr(n, rp, col, rpt, colt);
  rps.assign(static_cast<size_t>(n) + 1, 0);
  std::vector<int32_t> merged;
  cols.clear();
  cols.reserve(static_cast<size_t>(2 * rp[n]));
  for (int64_t u = 0; u < n; ++u) {
    merged.clear();
    std::merge(col + rp[u], col + rp[u + 1], colt.begin() + rpt[u], colt.begin() + rpt[u + 1],
               std::back_inserter(merged));
    merged.erase(std::unique(merged.begin(), merged.end()), merged.end());
    cols.insert(cols.end(), merged.begin(), merged.end());
    rps[u + 1] = static_cast<int32_t>(cols.size());
  }
}

bool is_scale_free_like(int64_t n, const int32_t* rp) {
  // Degree share: top 1% of vertices hold >= 5% and top 10% hold >= 40% of all degree.
  std::vector<int32_t> deg(n);
  for (int64_t u = 0; u < n; ++u) deg[u] = rp[u + 1] - rp[u];
  const double total = static_cast<double>(rp[n]);
  if (total <= 0) return false;
  std::vector<int32_t> sorted = deg;
  std::sort(sorted.begin(), sorted.end(), std::greater<int32_t>());
  auto share = [&](double frac) {
    const int64_t k = std::max<int64_t>(1, static_cast<int64_t>(std::ceil(frac * n)));
    double s = 0;
    for (int64_t i = 0; i < k && i < n; ++i) s += sorted[i];
    return s / total;
  };
  if (share(0.01) >= 0.05 && share(0.10) >= 0.40) return true;
  // Log-log fit of the degree histogram for k >= 5: slope -gamma, R^2 >= 0.70, gamma in [1, 5].
  std::vector<int64_t> hist(static_cast<size_t>(sorted.empty() ? 1 : sorted[0] + 1), 0);
  for (int32_t d : deg) hist[d]++;
  double sx = 0, sy = 0, sxx = 0, sxy = 0, syy = 0;
  int64_t cnt = 0;
  for (size_t k = 5; k < hist.size(); ++k) {
    if (!hist[k]) continue;
    const double x = std::log(static_cast<double>(k)), y = std::log(static_cast<double>(hist[k]));
    sx += x; sy += y; sxx += x * x; sxy += x * y; syy += y * y; ++cnt;
  }
  if (cnt < 3) return false;
  const double mx = sx / cnt, my = sy / cnt;
  const double vx = sxx / cnt - mx * mx, vy = syy / cnt - my * my, cxy = sxy / cnt - mx * my;
  if (vx <= 0 || vy <= 0) return false;
  const double slope = cxy / vx, r2 = (cxy * cxy) / (vx * vy);
  const double gamma = -slope;
  return r2 >= 0.70 && gamma >= 1.0 && gamma <= 5.0;
}

// Reverse Cuthill-McKee. Components are taken in order of their smallest
// vertex id; each starts at a pseudo-peripheral vertex found by the
// George-Liu iteration from the component's minimum-degree vertex; children
// are visited by ascending degree, ties by id; the final order is reversed.
std::vector<int32_t> rcm_order(int64_t n, const int32_t* rp, const int32_t* col) {
  auto deg = [&](int32_t u) { return rp[u + 1] - rp[u]; };
  std::vector<int32_t> order;
  order.reserve(n);
  std::vector<char> placed(n, 0);
  std::vector<int32_t> dist(n, -1), comp, frontier;
  std::vector<int32_t> touched;
  auto bfs_levels = [&](int32_t s, int32_t& ecc, std::vector<int32_t>& last_level) {
    // plain BFS restricted to the component; returns eccentricity and last level
    for (int32_t v : touched) dist[v] = -1;
    touched.clear();
    std::vector<int32_t> q{s};
    dist[s] = 0;
    touched.push_back(s);
    size_t h = 0;
    ecc = 0;
    while (h < q.size()) {
      int32_t u = q[h++];
      for (int32_t p = rp[u]; p < rp[u + 1]; ++p) {
        int32_t v = col[p];
        if (dist[v] < 0) {
          dist[v] = dist[u] + 1;
          ecc = std::max(ecc, dist[v]);
          q.push_back(v);
          touched.push_back(v);
        }
      }
    }
    last_level.clear();
    for (int32_t v : q)
      if (dist[v] == ecc) last_level.push_back(v);
    return q;
  };
  std::vector<int32_t> last;
  for (int64_t r = 0; r < n; ++r) {
    if (placed[r]) continue;
    int32_t ecc = 0;
    std::vector<int32_t> members = bfs_levels(static_cast<int32_t>(r), ecc, last);
    int32_t start = members[0];
    for (int32_t v : members)
      if (deg(v) < deg(start) || (deg(v) == deg(start) && v < start)) start = v;
    // George-Liu pseudo-peripheral search
    bfs_levels(start, ecc, last);
    for (int it = 0; it < 16; ++it) {
      int32_t cand = last[0];
      for (int32_t v : last)
        if (deg(v) < deg(cand) || (deg(v) == deg(cand) && v < cand)) cand = v;
      int32_t ecc2 = 0;
      std::vector<int32_t> last2;
      bfs_levels(cand, ecc2, last2);
      if (ecc2 > ecc) {
        start = cand;
        ecc = ecc2;
        last = last2;
      } else {
        break;
      }
    }
    // Cuthill-McKee from start
    size_t h = order.size();
    order.push_back(start);
    placed[start] = 1;
    std::vector<int32_t> kids;
    while (h < order.size()) {
      int32_t u = order[h++];
      kids.clear();
      for (int32_t p = rp[u]; p < rp[u + 1]; ++p)
        if (!placed[col[p]]) {
          placed[col[p]] = 1;
          kids.push_back(col[p]);
        }
      std::sort(kids.begin(), kids.end(), [&](int32_t a, int32_t b) {
        return deg(a) != deg(b) ? deg(a) < deg(b) : a < b;
      });
      order.insert(order.end(), kids.begin(), kids.end());
    }
  }
  std::reverse(order.begin(), order.end());
  return order;  // order[new id] = old id
}

std::vector<int32_t> jaccard_order(int64_t n, const int32_t* rp, const int32_t* col, int sigma, int64_t window) {
  std::vector<int32_t> new_of_old(static_cast<size_t>(n), 0);
  if (n <= 0) return new_of_old;
  const int64_t nwin = (n + window - 1) / window;
  const int t = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(host_threads(), nwin)));
  std::vector<std::thread> pool;
  for (int ti = 0; ti < t; ++ti) {
    pool.emplace_back([&, ti] {
      // per-thread scratch: membership stamps of R over all rows, and the
      // window-local candidate state
      std::vector<uint32_t> in_r(static_cast<size_t>(n), 0u);
      uint32_t stamp = 0;
      std::vector<int32_t> inter(static_cast<size_t>(window), 0);
      std::vector<char> assigned(static_cast<size_t>(window), 0), in_q(static_cast<size_t>(window), 0);
      std::vector<int32_t> q, touched, by_deg;
      auto deg = [&](int64_t j) { return static_cast<int64_t>(rp[j + 1] - rp[j]); };
      for (int64_t w = ti; w < nwin; w += t) {
        const int64_t ws = w * window, we = std::min(ws + window, n), wn = we - ws;
        std::fill(assigned.begin(), assigned.begin() + wn, 0);
        by_deg.resize(static_cast<size_t>(wn));
        for (int64_t j = 0; j < wn; ++j) by_deg[j] = static_cast<int32_t>(j);
        std::stable_sort(by_deg.begin(), by_deg.end(),
                         [&](int32_t x, int32_t y) { return deg(ws + x) > deg(ws + y); });
        size_t next_deg = 0;
        auto highest = [&]() {
          while (assigned[by_deg[next_deg]]) ++next_deg;
          return by_deg[next_deg];
        };
        int64_t rsize = 0;
        // adds row i to R and updates inter/Q of the window's unassigned columns
        auto add_row = [&](int32_t i) {
          in_r[i] = stamp;
          ++rsize;
          const int32_t* b = col + rp[i];
          const int32_t* e = col + rp[i + 1];
          for (const int32_t* p = std::lower_bound(b, e, static_cast<int32_t>(ws)); p < e && *p < we; ++p) {
            const int32_t j = static_cast<int32_t>(*p - ws);
            if (assigned[j]) continue;
            if (inter[j] == 0) {
              touched.push_back(j);
              if (!in_q[j]) {
                in_q[j] = 1;
                q.push_back(j);
              }
            }
            ++inter[j];
          }
        };
        auto take = [&](int32_t j, int64_t pos) {
          assigned[j] = 1;
          new_of_old[ws + j] = static_cast<int32_t>(pos);
          for (int32_t p = rp[ws + j]; p < rp[ws + j + 1]; ++p)
            if (in_r[col[p]] != stamp) add_row(col[p]);
        };
        for (int64_t ss = ws; ss < we; ss += sigma) {
          const int64_t se = std::min<int64_t>(ss + sigma, we);
          ++stamp;
          rsize = 0;
          take(highest(), ss);
          for (int64_t pos = ss + 1; pos < se; ++pos) {
            // best candidate of Q: largest inter / (|R| + deg - inter), ties to the smaller id
            int32_t best = -1;
            int64_t bn = 0, bd = 1;
            size_t keep = 0;
            for (size_t k = 0; k < q.size(); ++k) {
              const int32_t j = q[k];
              if (assigned[j]) {
                in_q[j] = 0;
                continue;
              }
              q[keep++] = j;
              const int64_t num = inter[j], den = rsize + deg(ws + j) - inter[j];
              if (best < 0 || num * bd > bn * den || (num * bd == bn * den && j < best)) {
                best = j;
                bn = num;
                bd = den;
              }
            }
            q.resize(keep);
            take(best >= 0 ? best : highest(), pos);
          }
          // reset the candidate state of this slice set
          for (int32_t j : touched) inter[j] = 0;
          for (int32_t j : q) in_q[j] = 0;
          touched.clear();
          q.clear();
        }
      }
    });
  }
  for (auto& th : pool) th.join();
  return new_of_old;
}

void permute_csr(int64_t n, const int32_t* rp, const int32_t* col, const std::vector<int32_t>& old_of_new,
                 std::vector<int32_t>& new_of_old, std::vector<int32_t>& rp2, std::vector<int32_t>& col2) {
  new_of_old.assign(n, 0);
  for (int64_t i = 0; i < n; ++i) new_of_old[old_of_new[i]] = static_cast<int32_t>(i);
  rp2.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t o = old_of_new[i];
    rp2[i + 1] = rp2[i] + (rp[o + 1] - rp[o]);
  }
  col2.resize(static_cast<size_t>(rp[n]));
  parallel_for(n, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      const int32_t o = old_of_new[i];
      int32_t* out = col2.data() + rp2[i];
      int64_t k = 0;
      for (int32_t p = rp[o]; p < rp[o + 1]; ++p) out[k++] = new_of_old[col[p]];
      std::sort(out, out + k);
    }
  });
}

bool build_bvss(int64_t n, const int32_t* rp, const int32_t* col, int sigma, int tau, bool wide, Bvss* out) {
  const int64_t ns = (n + sigma - 1) / sigma;
  out->nsets = ns;
  std::vector<int64_t> count(ns, 0);
  // Pass 1: slice count per set (size of the union of sigma sorted rows).
  auto merge_set = [&](int64_t s, auto&& emit) {
    const int64_t j0 = s * sigma, j1 = std::min<int64_t>(n, j0 + sigma);
    int32_t head[64], tail[64];
    int k = 0;
    for (int64_t j = j0; j < j1; ++j, ++k) {
      head[k] = rp[j];
      tail[k] = rp[j + 1];
    }
    for (;;) {
      int32_t best = INT32_MAX;
      for (int i = 0; i < k; ++i)
        if (head[i] < tail[i] && col[head[i]] < best) best = col[head[i]];
      if (best == INT32_MAX) break;
      uint64_t mask = 0;
      for (int i = 0; i < k; ++i)
        if (head[i] < tail[i] && col[head[i]] == best) {
          mask |= uint64_t(1) << i;
          ++head[i];
        }
      emit(best, mask);
    }
  };
  parallel_for(ns, [&](int64_t b, int64_t e) {
    for (int64_t s = b; s < e; ++s) {
      int64_t c = 0;
      merge_set(s, [&](int32_t, uint64_t) { ++c; });
      count[s] = c;
    }
  });
  out->slice_ptr.assign(ns + 1, 0);
  out->real_ptrs.assign(ns + 1, 0);
  for (int64_t s = 0; s < ns; ++s) {
    out->slice_ptr[s + 1] = out->slice_ptr[s] + static_cast<uint32_t>(count[s]);
    out->real_ptrs[s + 1] = out->real_ptrs[s] + (count[s] + tau - 1) / tau;
  }
  const int64_t nsl = static_cast<int64_t>(out->slice_ptr[ns]);
  out->nslices = nsl;
  out->nvss = out->real_ptrs[ns];
  out->wide = wide;
  if (wide)
    out->slices64.resize(static_cast<size_t>(nsl));
  else
    out->slices32.resize(static_cast<size_t>(nsl));
  // Pass 2: fill packed slice words.
  parallel_for(ns, [&](int64_t b, int64_t e) {
    for (int64_t s = b; s < e; ++s) {
      int64_t o = out->slice_ptr[s];
      if (wide)
        merge_set(s, [&](int32_t row, uint64_t mask) {
          out->slices64[o++] = (static_cast<uint64_t>(static_cast<uint32_t>(row)) << 32) | mask;
        });
      else
        merge_set(s, [&](int32_t row, uint64_t mask) {
          out->slices32[o++] = (static_cast<uint32_t>(row) << 8) | static_cast<uint32_t>(mask);
        });
    }
  });
  // Degree masks per set.
  out->degmask.assign(static_cast<size_t>(ns), 0);
  for (int64_t u = 0; u < n; ++u)
    if (rp[u + 1] > rp[u]) out->degmask[u / sigma] |= uint64_t(1) << (u % sigma);
  return true;
}

double update_divergence(const Bvss& b, int tau) {
  if (b.nvss == 0) return 0.0;
  const int theta = std::max(1, tau / 32);
  std::vector<double> part(static_cast<size_t>(b.nsets), 0.0);
  parallel_for(b.nsets, [&](int64_t lo, int64_t hi) {
    for (int64_t s = lo; s < hi; ++s) {
      const int64_t s0 = b.slice_ptr[s], s1 = b.slice_ptr[s + 1];
      auto row = [&](int64_t k) -> double {
        return b.wide ? static_cast<double>(b.slices64[k] >> 32) : static_cast<double>(b.slices32[k] >> 8);
      };
      double acc = 0.0;
      for (int64_t v0 = s0; v0 < s1; v0 += tau) {
        const int64_t v1 = std::min<int64_t>(s1, v0 + tau);
        double sum = 0.0;
        int cols = 0;
        for (int c = 0; c < theta; ++c) {
          int64_t cnt = 0;
          double mean = 0.0;
          for (int64_t k = v0 + c; k < v1; k += theta, ++cnt) mean += row(k);
          if (cnt == 0) continue;
          mean /= static_cast<double>(cnt);
          double m2 = 0.0;
          for (int64_t k = v0 + c; k < v1; k += theta) m2 += (row(k) - mean) * (row(k) - mean);
          sum += std::sqrt(m2 / static_cast<double>(cnt));
          ++cols;
        }
        acc += sum / cols;
      }
      part[s] = acc;
    }
  });
  double tot = 0.0;
  for (double x : part) tot += x;
  return tot / static_cast<double>(b.nvss);
}

int panel_log2_rows(int64_t n, int64_t workgroups) {
  const int64_t rows = (n + std::max<int64_t>(workgroups, 1) - 1) / std::max<int64_t>(workgroups, 1);
  int lg = 0;
  while ((int64_t(1) << lg) < rows) ++lg;
  return std::max(5, std::min(15, lg));
}

bool build_panels(int64_t n, const Bvss& b, int rb, Panels* out) {
  if (b.wide || b.nslices == 0 || n > (int64_t(1) << 24) || rb < 5 || rb > 15) return false;
  const int rshift = 32 - rb;
  const uint32_t dlim = std::min<uint32_t>(1u << (24 - rb), 505u);
  const int64_t np = (n + (int64_t(1) << rb) - 1) >> rb;
  const int64_t ns = b.nsets;
  // Counting sort of (set, slice) pairs by panel, stable in set order: each
  // thread owns a contiguous range of sets and writes behind the counts of
  // the threads before it in every panel.
  const int t = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(host_threads(), ns / 1024 + 1)));
  const int64_t span = (ns + t - 1) / t;
  std::vector<int64_t> hist(static_cast<size_t>(t) * np, 0);
  auto run = [&](auto&& body) {
    std::vector<std::thread> pool;
    for (int i = 0; i < t; ++i) pool.emplace_back([&, i] { body(i); });
    for (auto& th : pool) th.join();
  };
  run([&](int i) {
    int64_t* h = &hist[static_cast<size_t>(i) * np];
    const int64_t s0 = std::min(ns, i * span), s1 = std::min(ns, s0 + span);
    for (uint32_t k = b.slice_ptr[s0]; k < b.slice_ptr[s1]; ++k) ++h[(b.slices32[k] >> 8) >> rb];
  });
  std::vector<int64_t> start(np + 1, 0);
  {
    int64_t acc = 0;
    for (int64_t p = 0; p < np; ++p) {
      start[p] = acc;
      for (int i = 0; i < t; ++i) {
        const int64_t c = hist[static_cast<size_t>(i) * np + p];
        hist[static_cast<size_t>(i) * np + p] = acc;
        acc += c;
      }
    }
    start[np] = acc;
  }
  std::vector<uint32_t> tset(static_cast<size_t>(b.nslices)), tword(static_cast<size_t>(b.nslices));
  run([&](int i) {
    int64_t* h = &hist[static_cast<size_t>(i) * np];
    const int64_t s0 = std::min(ns, i * span), s1 = std::min(ns, s0 + span);
    for (int64_t s = s0; s < s1; ++s)
      for (uint32_t k = b.slice_ptr[s]; k < b.slice_ptr[s + 1]; ++k) {
        const uint32_t w = b.slices32[k];
        const uint32_t row = w >> 8;
        const int64_t o = h[row >> rb]++;
        tset[o] = static_cast<uint32_t>(s);
        tword[o] = ((row & ((1u << rb) - 1u)) << rshift) | (w & 0xffu);
      }
  });
  // Chunking per panel: kPanelChunk slices, or fewer where the next slice's
  // set is dlim or more past the chunk's first set.
  auto chunk_panel = [&](int64_t p, auto&& emit) {
    int64_t i = start[p];
    const int64_t e = start[p + 1];
    int64_t c = 0;
    while (i < e) {
      const uint32_t base = tset[i];
      const uint32_t lim = std::min<uint32_t>(dlim, 512u - (base & 7u));
      int k = 0;
      while (i < e && k < kPanelChunk && tset[i] - base < lim) {
        emit(c, k, base, tword[i] | ((tset[i] - base) << 8));
        ++i;
        ++k;
      }
      ++c;
    }
    return c;
  };
  std::vector<int64_t> cnt(np, 0);
  parallel_for(np, [&](int64_t p0, int64_t p1) {
    for (int64_t p = p0; p < p1; ++p) cnt[p] = chunk_panel(p, [](int64_t, int, uint32_t, uint32_t) {});
  });
  out->rb = rb;
  out->npanels = np;
  out->ptr.assign(np + 1, 0);
  for (int64_t p = 0; p < np; ++p) out->ptr[p + 1] = out->ptr[p] + static_cast<uint32_t>(cnt[p]);
  out->nchunks = out->ptr[np];
  out->words.assign(static_cast<size_t>(out->nchunks) * kPanelChunk, 0u);
  out->base.assign(static_cast<size_t>(out->nchunks), 0u);
  parallel_for(np, [&](int64_t p0, int64_t p1) {
    for (int64_t p = p0; p < p1; ++p) {
      const int64_t c0 = out->ptr[p];
      chunk_panel(p, [&](int64_t c, int k, uint32_t base, uint32_t word) {
        out->base[c0 + c] = base;
        out->words[(c0 + c) * kPanelChunk + k] = word;
      });
    }
  });
  return true;
}

}  // namespace blest

