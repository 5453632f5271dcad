// Host-side preprocessing declarations (host_build.cpp).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace blest {

struct Bvss {
  int64_t nsets = 0, nvss = 0, nslices = 0;
  bool wide = false;
  std::vector<uint32_t> slice_ptr;  // N_s + 1
  std::vector<int64_t> real_ptrs;   // N_s + 1 (VSS offsets, realPtrs)
  std::vector<uint32_t> slices32;   // (row << 8) | mask, sigma = 8
  std::vector<uint64_t> slices64;   // (row << 32) | mask
  std::vector<uint64_t> degmask;    // per set: bit b = vertex s*sigma+b has degree > 0
};

// O(m log d) check of a simple CSR (sorted rows, no duplicates or self
// loops; symmetric unless the graph is directed); *why explains a failure.
bool validate_csr(int64_t n, int64_t m, const int32_t* rp, const int32_t* col, std::string* why,
                  bool symmetric = true);

// CSR of the transposed graph (in-arcs), rows sorted.
void transpose_csr(int64_t n, const int32_t* rp, const int32_t* col, std::vector<int32_t>& rpt,
                   std::vector<int32_t>& colt);

// CSR of the undirected graph underlying a directed one (union of out- and
// in-arcs per vertex), rows sorted and deduplicated.
void symmetrize_csr(int64_t n, const int32_t* rp, const int32_t* col, std::vector<int32_t>& rps,
                    std::vector<int32_t>& cols);

// Heavy-tailed degree distribution test used to pick the reordering.
bool is_scale_free_like(int64_t n, const int32_t* rp);

// Reverse Cuthill-McKee order: result[new id] = old id.
std::vector<int32_t> rcm_order(int64_t n, const int32_t* rp, const int32_t* col);

// JaccardWithWindows (Alg. "JaccardWithWindows", Section "Increasing
// Compression Ratio"): within each window of `window` consecutive ids, slice
// sets of sigma columns are filled greedily, each seeded by the
// highest-degree unassigned column and grown by the candidate maximising
// inter / (|R| + deg - inter). Result: new_of_old (the algorithm's inverse
// permutation), every id staying inside its window. Ties go to the smaller
// id; a window whose width is not a multiple of sigma ends with a partial set.
std::vector<int32_t> jaccard_order(int64_t n, const int32_t* rp, const int32_t* col, int sigma, int64_t window);

// Relabels a CSR: vertex old_of_new[i] becomes i.
void permute_csr(int64_t n, const int32_t* rp, const int32_t* col, const std::vector<int32_t>& old_of_new,
                 std::vector<int32_t>& new_of_old, std::vector<int32_t>& rp2, std::vector<int32_t>& col2);

bool build_bvss(int64_t n, const int32_t* rp, const int32_t* col, int sigma, int tau, bool wide, Bvss* out);

// Update divergence (Section "Boosting Cache Locality"): a VSS of tau slices
// is a (tau / theta) x theta matrix whose slice j sits in column j mod theta;
// a column's divergence is the population standard deviation of the row ids
// of its slices (every stored slice has a nonzero mask), a VSS's divergence
// the mean over its non-empty columns, and U_div the mean over all N_v VSSs.
// theta = tau / 32 (the paper's 32 x 4 matrix at tau = 128). 0 without VSSs.
double update_divergence(const Bvss& b, int tau);

// The paper's dispatch (Section "Ablation Studies"): graphs with U_div above
// this threshold use lazy vertex updates (Alg. 3), the others Alg. 2.
constexpr double kEagerMaxUdiv = 25000.0;

// Panel-blocked copy of a sigma = 8, 32-bit BVSS for dense top-down levels.
// Rows are cut into panels of 2^rb consecutive rows; a panel's slices are
// listed set by set (ascending set, then row) in chunks of kPanelChunk. A
// chunk records the set of its first slice (base); each slice word is
//   (row - panel start) << (32 - rb) | (set - base) << 8 | mask.
// A chunk is closed early (and padded with zero words, which never hit) so
// that set - base stays below 2^(24 - rb) and (base mod 8) + (set - base)
// stays below 512: the frontier words of a chunk's sets then lie in one
// 512-byte window that a wave loads with one 8-byte load per lane.
constexpr int kPanelChunk = 256;
struct Panels {
  int rb = 0;                     // log2 rows per panel (0: no panel copy)
  int64_t npanels = 0, nchunks = 0;
  std::vector<uint32_t> words;    // nchunks * kPanelChunk
  std::vector<uint32_t> base;     // nchunks
  std::vector<uint32_t> ptr;      // npanels + 1: chunk range of each panel
};

// log2 of the panel height for an n-vertex graph traversed by `workgroups`
// persistent workgroups: about one panel per workgroup, within [5, 15].
int panel_log2_rows(int64_t n, int64_t workgroups);

// rb = log2 rows per panel, in [5, 15]. Returns false (and builds nothing)
// for 64-bit slices, an empty BVSS or n > 2^24.
bool build_panels(int64_t n, const Bvss& b, int rb, Panels* out);

}  // namespace blest
