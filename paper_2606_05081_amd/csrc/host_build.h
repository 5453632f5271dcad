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

// O(m log d) check of an undirected simple CSR; *why explains a failure.
bool validate_csr(int64_t n, int64_t m, const int32_t* rp, const int32_t* col, std::string* why);

// Heavy-tailed degree distribution test used to pick the reordering.
bool is_scale_free_like(int64_t n, const int32_t* rp);

// Reverse Cuthill-McKee order: result[new id] = old id.
std::vector<int32_t> rcm_order(int64_t n, const int32_t* rp, const int32_t* col);

// Relabels a CSR: vertex old_of_new[i] becomes i.
void permute_csr(int64_t n, const int32_t* rp, const int32_t* col, const std::vector<int32_t>& old_of_new,
                 std::vector<int32_t>& new_of_old, std::vector<int32_t>& rp2, std::vector<int32_t>& col2);

bool build_bvss(int64_t n, const int32_t* rp, const int32_t* col, int sigma, int tau, bool wide, Bvss* out);

}  // namespace blest
