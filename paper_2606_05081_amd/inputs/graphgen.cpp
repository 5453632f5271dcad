// Seeded synthetic graph inputs: R-MAT, 2-D grids with random edge deletion,
// Erdos-Renyi pair graphs, random vertex relabelling and source sampling.
//
// This module only manufactures inputs. It holds none of the BFS arithmetic
// and is shared by the CPU oracle (tests) and the GPU library's callers.
//
// Every random number is counter based: draw i of stream `seed` is the i-th
// output of the splitmix64 generator (Steele, Lea, Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014) started at `seed`, i.e.
// mix64(seed + (i + 1) * 0x9E3779B97F4A7C15). Results therefore do not depend
// on the number of threads.
//
// Output graphs are undirected simple graphs in CSR form: int32 row_ptr[n+1],
// int32 col[m], every row sorted ascending, no self loops, no duplicates, and
// (u,v) present iff (v,u) present.

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ULL;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
inline uint64_t draw_u64(uint64_t seed, uint64_t i) { return mix64(seed + (i + 1) * kGolden); }
// 53-bit uniform double in [0,1).
inline double draw_unit(uint64_t seed, uint64_t i) {
  return static_cast<double>(draw_u64(seed, i) >> 11) * (1.0 / 9007199254740992.0);
}
// Uniform integer in [0, bound) by Lemire's multiply-shift (bias < bound / 2^64).
inline uint64_t draw_below(uint64_t seed, uint64_t i, uint64_t bound) {
  return static_cast<uint64_t>((static_cast<unsigned __int128>(draw_u64(seed, i)) * bound) >> 64);
}
// Independent sub-streams of one user seed.
inline uint64_t substream(uint64_t seed, uint64_t tag) { return mix64(mix64(seed) ^ mix64(tag * kGolden + 0x5851F42D4C957F2DULL)); }

int pick_threads(int t) {
  if (t > 0) return t;
  unsigned h = std::thread::hardware_concurrency();
  if (h == 0) h = 4;
  return static_cast<int>(std::min<unsigned>(h, 16));
}

template <class F>
void parallel_for(int64_t n, int threads, F&& f) {
  threads = pick_threads(threads);
  if (n < 4096 || threads <= 1) {
    f(int64_t(0), n);
    return;
  }
  std::vector<std::thread> pool;
  int64_t chunk = (n + threads - 1) / threads;
  for (int t = 0; t < threads; ++t) {
    int64_t b = t * chunk, e = std::min<int64_t>(n, b + chunk);
    if (b >= e) break;
    pool.emplace_back([=, &f] { f(b, e); });
  }
  for (auto& th : pool) th.join();
}

struct Csr {
  int64_t n = 0;
  std::vector<int64_t> rp;  // n+1
  std::vector<int32_t> col;
};

// Builds the symmetric, deduplicated, loop-free CSR of the undirected pairs
// (u_i, v_i), i < npairs (directed: only the arc u_i -> v_i is kept). `pairs`
// packs u in the high and v in the low 32 bits.
Csr csr_from_pairs(int64_t n, const std::vector<uint64_t>& pairs, int threads, bool directed = false) {
  const int64_t np = static_cast<int64_t>(pairs.size());
  std::vector<std::atomic<int64_t>> cnt(n + 1);
  parallel_for(n + 1, threads, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) cnt[i].store(0, std::memory_order_relaxed);
  });
  parallel_for(np, threads, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      uint32_t u = static_cast<uint32_t>(pairs[i] >> 32), v = static_cast<uint32_t>(pairs[i]);
      if (u == v) continue;
      cnt[u].fetch_add(1, std::memory_order_relaxed);
      if (!directed) cnt[v].fetch_add(1, std::memory_order_relaxed);
    }
  });
  std::vector<int64_t> off(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + cnt[i].load(std::memory_order_relaxed);
  std::vector<int32_t> adj(static_cast<size_t>(off[n]));
  parallel_for(n, threads, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) cnt[i].store(off[i], std::memory_order_relaxed);
  });
  parallel_for(np, threads, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      uint32_t u = static_cast<uint32_t>(pairs[i] >> 32), v = static_cast<uint32_t>(pairs[i]);
      if (u == v) continue;
      adj[cnt[u].fetch_add(1, std::memory_order_relaxed)] = static_cast<int32_t>(v);
      if (!directed) adj[cnt[v].fetch_add(1, std::memory_order_relaxed)] = static_cast<int32_t>(u);
    }
  });
  // Sort and deduplicate each row in place; record the unique length.
  std::vector<int64_t> ulen(n, 0);
  parallel_for(n, threads, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      int32_t* first = adj.data() + off[i];
      int32_t* last = adj.data() + off[i + 1];
      std::sort(first, last);
      ulen[i] = std::unique(first, last) - first;
    }
  });
  Csr g;
  g.n = n;
  g.rp.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) g.rp[i + 1] = g.rp[i] + ulen[i];
  g.col.resize(static_cast<size_t>(g.rp[n]));
  parallel_for(n, threads, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i)
      std::memcpy(g.col.data() + g.rp[i], adj.data() + off[i], sizeof(int32_t) * ulen[i]);
  });
  return g;
}

// Uniform random permutation of [0,n) by Fisher-Yates over stream `seed`.
std::vector<int32_t> random_permutation(int64_t n, uint64_t seed) {
  std::vector<int32_t> p(n);
  for (int64_t i = 0; i < n; ++i) p[i] = static_cast<int32_t>(i);
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = static_cast<int64_t>(draw_below(seed, static_cast<uint64_t>(i), static_cast<uint64_t>(i + 1)));
    std::swap(p[i], p[j]);
  }
  return p;
}

// Relabels vertex u as p[u].
Csr relabel(const Csr& g, const std::vector<int32_t>& p, int threads) {
  const int64_t n = g.n;
  Csr h;
  h.n = n;
  std::vector<int64_t> deg(n);
  for (int64_t u = 0; u < n; ++u) deg[p[u]] = g.rp[u + 1] - g.rp[u];
  h.rp.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) h.rp[i + 1] = h.rp[i] + deg[i];
  h.col.resize(g.col.size());
  parallel_for(n, threads, [&](int64_t b, int64_t e) {
    for (int64_t u = b; u < e; ++u) {
      int32_t* out = h.col.data() + h.rp[p[u]];
      int64_t k = 0;
      for (int64_t q = g.rp[u]; q < g.rp[u + 1]; ++q) out[k++] = p[g.col[q]];
      std::sort(out, out + k);
    }
  });
  return h;
}

struct Result {
  int64_t n = 0, m = 0;
  int32_t* rp = nullptr;
  int32_t* col = nullptr;
};

Result* publish(const Csr& g) {
  if (g.rp[g.n] > INT32_MAX) return nullptr;
  Result* r = new (std::nothrow) Result;
  if (!r) return nullptr;
  r->n = g.n;
  r->m = g.rp[g.n];
  r->rp = static_cast<int32_t*>(std::malloc(sizeof(int32_t) * (g.n + 1)));
  r->col = static_cast<int32_t*>(std::malloc(sizeof(int32_t) * std::max<int64_t>(1, r->m)));
  if (!r->rp || !r->col) {
    std::free(r->rp);
    std::free(r->col);
    delete r;
    return nullptr;
  }
  for (int64_t i = 0; i <= g.n; ++i) r->rp[i] = static_cast<int32_t>(g.rp[i]);
  if (r->m) std::memcpy(r->col, g.col.data(), sizeof(int32_t) * r->m);
  return r;
}

}  // namespace

extern "C" {

void* gg_rmat_directed(int32_t scale, int32_t edgefactor, double a, double b, double c, uint64_t seed,
                       int32_t permute, int32_t threads, int32_t directed);
void* gg_directed_from_pairs(int64_t n, int64_t npairs, const int32_t* us, const int32_t* vs, int32_t directed);

// Releases a graph returned by one of the generators below.
void gg_free(void* h) {
  Result* r = static_cast<Result*>(h);
  if (!r) return;
  std::free(r->rp);
  std::free(r->col);
  delete r;
}
int64_t gg_n(const void* h) { return static_cast<const Result*>(h)->n; }
int64_t gg_m(const void* h) { return static_cast<const Result*>(h)->m; }
const int32_t* gg_row_ptr(const void* h) { return static_cast<const Result*>(h)->rp; }
const int32_t* gg_col(const void* h) { return static_cast<const Result*>(h)->col; }

// R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): edgefactor * 2^scale samples;
// at every one of `scale` bit levels the quadrant is (0,0),(0,1),(1,0),(1,1)
// with probabilities a, b, c, 1-a-b-c. Then symmetrised, self loops and
// duplicates dropped and, if `permute`, vertices relabelled by a uniform
// random permutation. Returns NULL on bad arguments or out of memory.
void* gg_rmat(int32_t scale, int32_t edgefactor, double a, double b, double c, uint64_t seed,
              int32_t permute, int32_t threads) {
  return gg_rmat_directed(scale, edgefactor, a, b, c, seed, permute, threads, 0);
}

// The same samples kept as arcs u -> v when `directed` (self loops and
// duplicate arcs dropped), else symmetrised as above.
void* gg_rmat_directed(int32_t scale, int32_t edgefactor, double a, double b, double c, uint64_t seed,
                       int32_t permute, int32_t threads, int32_t directed) {
  if (scale < 1 || scale > 30 || edgefactor < 1 || a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return nullptr;
  const int64_t n = int64_t(1) << scale;
  const int64_t ne = n * edgefactor;
  const uint64_t s_edge = substream(seed, 1), s_perm = substream(seed, 2);
  const double ab = a + b, abc = a + b + c;
  try {
    std::vector<uint64_t> pairs(ne);
    parallel_for(ne, threads, [&](int64_t lo, int64_t hi) {
      for (int64_t e = lo; e < hi; ++e) {
        uint64_t u = 0, v = 0;
        for (int l = 0; l < scale; ++l) {
          double r = draw_unit(s_edge, static_cast<uint64_t>(e) * scale + l);
          uint64_t ub = 0, vb = 0;
          if (r < a) {
          } else if (r < ab) {
            vb = 1;
          } else if (r < abc) {
            ub = 1;
          } else {
            ub = 1;
            vb = 1;
          }
          u = (u << 1) | ub;
          v = (v << 1) | vb;
        }
        pairs[e] = (u << 32) | v;
      }
    });
    Csr g = csr_from_pairs(n, pairs, threads, directed != 0);
    pairs.clear();
    pairs.shrink_to_fit();
    if (permute) g = relabel(g, random_permutation(n, s_perm), threads);
    return publish(g);
  } catch (...) {
    return nullptr;
  }
}

// side x side 4-neighbour grid, vertex (x,y) = y*side + x. Each of the
// 2*side*(side-1) grid edges is deleted independently with probability
// p_delete. If `permute`, vertices are relabelled by a random permutation.
void* gg_grid(int32_t side, double p_delete, uint64_t seed, int32_t permute, int32_t threads) {
  if (side < 1 || side > 46340 || p_delete < 0 || p_delete > 1) return nullptr;
  const int64_t s = side, n = s * s;
  const uint64_t s_del = substream(seed, 3), s_perm = substream(seed, 4);
  try {
    std::vector<uint64_t> pairs;
    pairs.reserve(2 * s * (s - 1));
    const int64_t nh = (s - 1) * s;  // horizontal edges first, then vertical
    for (int64_t y = 0; y < s; ++y)
      for (int64_t x = 0; x + 1 < s; ++x) {
        int64_t idx = y * (s - 1) + x;
        if (draw_unit(s_del, idx) >= p_delete) pairs.push_back((uint64_t(y * s + x) << 32) | uint64_t(y * s + x + 1));
      }
    for (int64_t y = 0; y + 1 < s; ++y)
      for (int64_t x = 0; x < s; ++x) {
        int64_t idx = nh + y * s + x;
        if (draw_unit(s_del, idx) >= p_delete) pairs.push_back((uint64_t(y * s + x) << 32) | uint64_t((y + 1) * s + x));
      }
    Csr g = csr_from_pairs(n, pairs, threads);
    if (permute) g = relabel(g, random_permutation(n, s_perm), threads);
    return publish(g);
  } catch (...) {
    return nullptr;
  }
}

// Erdos-Renyi style pair graph: `npairs` unordered pairs with both ends uniform
// on [0,n), symmetrised, self loops and duplicates dropped.
void* gg_erdos_renyi(int64_t n, int64_t npairs, uint64_t seed, int32_t threads) {
  if (n < 1 || n > INT32_MAX || npairs < 0) return nullptr;
  const uint64_t s_pair = substream(seed, 5);
  try {
    std::vector<uint64_t> pairs(npairs);
    parallel_for(npairs, threads, [&](int64_t lo, int64_t hi) {
      for (int64_t i = lo; i < hi; ++i) {
        uint64_t u = draw_below(s_pair, 2 * uint64_t(i), uint64_t(n));
        uint64_t v = draw_below(s_pair, 2 * uint64_t(i) + 1, uint64_t(n));
        pairs[i] = (u << 32) | v;
      }
    });
    return publish(csr_from_pairs(n, pairs, threads));
  } catch (...) {
    return nullptr;
  }
}

// Builds a graph from caller-supplied undirected pairs (same canonicalisation
// as the generators). Used for hand-made test graphs.
void* gg_from_pairs(int64_t n, int64_t npairs, const int32_t* us, const int32_t* vs) {
  return gg_directed_from_pairs(n, npairs, us, vs, 0);
}

// CSR of the arcs us[i] -> vs[i] when `directed` (sorted rows, self loops and
// duplicate arcs dropped), else of the undirected pairs as above.
void* gg_directed_from_pairs(int64_t n, int64_t npairs, const int32_t* us, const int32_t* vs, int32_t directed) {
  if (n < 1 || n > INT32_MAX || npairs < 0) return nullptr;
  try {
    std::vector<uint64_t> pairs(npairs);
    for (int64_t i = 0; i < npairs; ++i) {
      if (us[i] < 0 || us[i] >= n || vs[i] < 0 || vs[i] >= n) return nullptr;
      pairs[i] = (uint64_t(uint32_t(us[i])) << 32) | uint64_t(uint32_t(vs[i]));
    }
    return publish(csr_from_pairs(n, pairs, 1, directed != 0));
  } catch (...) {
    return nullptr;
  }
}

// Relabels an existing CSR by a random permutation of stream `seed`; writes the
// permutation (old id -> new id) to perm_out if non-NULL.
void* gg_permute(int64_t n, const int32_t* rp, const int32_t* col, uint64_t seed, int32_t* perm_out, int32_t threads) {
  try {
    Csr g;
    g.n = n;
    g.rp.assign(rp, rp + n + 1);
    g.col.assign(col, col + rp[n]);
    std::vector<int32_t> p = random_permutation(n, substream(seed, 6));
    if (perm_out) std::memcpy(perm_out, p.data(), sizeof(int32_t) * n);
    return publish(relabel(g, p, threads));
  } catch (...) {
    return nullptr;
  }
}

// Samples `count` source vertices from stream `seed`. If nonzero_degree, only
// vertices with at least one neighbour are eligible. If distinct, sources are
// drawn without replacement (partial Fisher-Yates over the eligible list, in
// ascending vertex order); otherwise independently with replacement.
// Returns the number written (0 if no vertex is eligible, or count exceeds the
// eligible set when distinct).
int64_t gg_sources(int64_t n, const int32_t* rp, int64_t count, uint64_t seed, int32_t nonzero_degree,
                   int32_t distinct, int32_t* out) {
  const uint64_t s_src = substream(seed, 7);
  std::vector<int32_t> elig;
  elig.reserve(n);
  for (int64_t v = 0; v < n; ++v)
    if (!nonzero_degree || rp[v + 1] > rp[v]) elig.push_back(static_cast<int32_t>(v));
  const int64_t ne = static_cast<int64_t>(elig.size());
  if (ne == 0) return 0;
  if (distinct) {
    if (count > ne) return 0;
    for (int64_t i = 0; i < count; ++i) {
      int64_t j = i + static_cast<int64_t>(draw_below(s_src, i, static_cast<uint64_t>(ne - i)));
      std::swap(elig[i], elig[j]);
      out[i] = elig[i];
    }
  } else {
    for (int64_t i = 0; i < count; ++i) out[i] = elig[draw_below(s_src, i, static_cast<uint64_t>(ne))];
  }
  return count;
}

}  // extern "C"
