// Sparse voxel octree from finest-level occupancy (Sec. 3.2; App. A.1), in
// the canonical layout: voxels of each depth sorted by Morton code, children
// of consecutive parents contiguous, corners of each feature level sorted by
// the Morton code of their lattice point.  This is the paper's
// initialisation pass that precomputes each voxel's corner pointers
// (Sec. 3.4).  Host code: it runs once per model, before any GPU work.
#include <algorithm>
#include <cstring>
#include <utility>
#include <vector>

#include "ngl_common.h"

namespace {

// Spread the low 21 bits of v so that bit b lands at bit 3b.
inline uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | v << 32) & 0x1f00000000ffffull;
  v = (v | v << 16) & 0x1f0000ff0000ffull;
  v = (v | v << 8) & 0x100f00f00f00f00full;
  v = (v | v << 4) & 0x10c30c30c30c30c3ull;
  v = (v | v << 2) & 0x1249249249249249ull;
  return v;
}

inline uint64_t compact3(uint64_t v) {
  v &= 0x1249249249249249ull;
  v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
  v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
  v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
  v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
  v = (v ^ (v >> 32)) & 0x1fffffull;
  return v;
}

inline uint64_t morton(uint64_t x, uint64_t y, uint64_t z) { return spread3(x) | spread3(y) << 1 | spread3(z) << 2; }

struct Tree {
  int L = 0, D = 0;
  std::vector<uint64_t> code[NGL_MAX_DEPTH];         // sorted voxel codes per depth
  std::vector<uint64_t> corner_code[NGL_MAX_LODS];   // sorted lattice codes per level
  std::vector<std::pair<uint64_t, uint32_t>> slots[NGL_MAX_LODS];  // (lattice code, 8*v+j), sorted
};

int build(const int32_t* ijk, int64_t n, int32_t L, Tree& t, bool want_slots) {
  NGL_REQUIRE(L >= 1 && L <= NGL_MAX_LODS, "num_lods %d outside 1..%d", L, NGL_MAX_LODS);
  NGL_REQUIRE(n >= 0, "negative cell count");
  NGL_REQUIRE(n == 0 || ijk != nullptr, "ijk is null");
  t.L = L;
  t.D = L + 1;
  const int64_t res = int64_t(1) << t.D;
  auto& fin = t.code[t.D];
  fin.resize(size_t(n));
  for (int64_t k = 0; k < n; ++k) {
    int32_t x = ijk[3 * k], y = ijk[3 * k + 1], z = ijk[3 * k + 2];
    NGL_REQUIRE(x >= 0 && y >= 0 && z >= 0 && x < res && y < res && z < res,
                "cell %lld = (%d,%d,%d) outside [0,%lld)^3", (long long)k, x, y, z, (long long)res);
    fin[size_t(k)] = morton(uint64_t(x), uint64_t(y), uint64_t(z));
  }
  std::sort(fin.begin(), fin.end());
  fin.erase(std::unique(fin.begin(), fin.end()), fin.end());
  // Parent closure: shifting a sorted code list keeps it sorted.
  for (int d = t.D - 1; d >= 0; --d) {
    const auto& ch = t.code[d + 1];
    auto& pa = t.code[d];
    pa.clear();
    for (uint64_t c : ch)
      if (pa.empty() || pa.back() != (c >> 3)) pa.push_back(c >> 3);
  }
  for (int l = 1; l <= L; ++l) {
    const auto& vc = t.code[l + 1];
    std::vector<std::pair<uint64_t, uint32_t>> s;
    s.reserve(vc.size() * 8);
    for (size_t v = 0; v < vc.size(); ++v) {
      uint64_t c = vc[v];
      uint64_t x = compact3(c), y = compact3(c >> 1), z = compact3(c >> 2);
      for (uint32_t j = 0; j < 8; ++j)
        s.emplace_back(morton(x + (j & 1), y + (j >> 1 & 1), z + (j >> 2 & 1)), uint32_t(8 * v + j));
    }
    std::sort(s.begin(), s.end());
    auto& cc = t.corner_code[l - 1];
    cc.clear();
    for (auto& e : s)
      if (cc.empty() || cc.back() != e.first) cc.push_back(e.first);
    if (want_slots) t.slots[l - 1] = std::move(s);
  }
  return NGL_OK;
}

}  // namespace

extern "C" {

int ngl_octree_plan(const int32_t* ijk, int64_t n, int32_t num_lods, int64_t* nvox, int64_t* ncorner) {
  NGL_REQUIRE(nvox && ncorner, "output count arrays are null");
  Tree t;
  int rc = build(ijk, n, num_lods, t, false);
  if (rc != NGL_OK) return rc;
  for (int d = 0; d <= t.D; ++d) nvox[d] = int64_t(t.code[d].size());
  for (int l = 0; l < t.L; ++l) ncorner[l] = int64_t(t.corner_code[l].size());
  return NGL_OK;
}

int ngl_octree_fill(const int32_t* ijk, int64_t n, int32_t num_lods, const ngl_octree_host* out) {
  NGL_REQUIRE(out != nullptr, "output struct is null");
  Tree t;
  int rc = build(ijk, n, num_lods, t, true);
  if (rc != NGL_OK) return rc;
  for (int d = 0; d <= t.D; ++d) {
    const auto& c = t.code[d];
    const size_t nv = c.size();
    if (out->cell[d])
      for (size_t v = 0; v < nv; ++v)
        out->cell[d][v] = uint32_t(compact3(c[v]) | compact3(c[v] >> 1) << 10 | compact3(c[v] >> 2) << 20);
    if (out->parent[d]) {
      if (d == 0) {
        for (size_t v = 0; v < nv; ++v) out->parent[d][v] = -1;
      } else {
        // merge walk: parents are sorted and every child's parent exists
        const auto& pc = t.code[d - 1];
        size_t p = 0;
        for (size_t v = 0; v < nv; ++v) {
          while (pc[p] != (c[v] >> 3)) ++p;
          out->parent[d][v] = int32_t(p);
        }
      }
    }
    if (out->child_mask[d] || out->first_child[d]) {
      std::vector<uint8_t> mask(nv, 0);
      std::vector<int32_t> first(nv, -1);
      if (d < t.D) {
        const auto& cc = t.code[d + 1];
        size_t p = 0;
        for (size_t k = 0; k < cc.size(); ++k) {
          while (c[p] != (cc[k] >> 3)) ++p;
          if (first[p] < 0) first[p] = int32_t(k);
          mask[p] |= uint8_t(1u << (cc[k] & 7));
        }
      }
      if (out->child_mask[d]) std::memcpy(out->child_mask[d], mask.data(), nv);
      if (out->first_child[d]) std::memcpy(out->first_child[d], first.data(), nv * sizeof(int32_t));
    }
  }
  for (int l = 1; l <= t.L; ++l) {
    const auto& s = t.slots[l - 1];
    if (out->corners[l - 1]) {
      int32_t idx = -1;
      uint64_t prev = ~uint64_t(0);
      for (auto& e : s) {
        if (e.first != prev) { ++idx; prev = e.first; }
        out->corners[l - 1][e.second] = idx;
      }
    }
    if (out->corner_adj_off[l - 1] || out->corner_adj[l - 1]) {
      // slots are sorted by (corner code, 8v+j): a CSR of corner -> 8v+j
      int32_t idx = -1;
      uint64_t prev = ~uint64_t(0);
      for (size_t k = 0; k < s.size(); ++k) {
        if (s[k].first != prev) {
          ++idx;
          prev = s[k].first;
          if (out->corner_adj_off[l - 1]) out->corner_adj_off[l - 1][idx] = int32_t(k);
        }
        if (out->corner_adj[l - 1]) out->corner_adj[l - 1][k] = int32_t(s[k].second);
      }
      if (out->corner_adj_off[l - 1]) out->corner_adj_off[l - 1][idx + 1] = int32_t(s.size());
    }
    if (out->corner_cell[l - 1]) {
      const auto& cc = t.corner_code[l - 1];
      for (size_t k = 0; k < cc.size(); ++k) {
        out->corner_cell[l - 1][3 * k] = int32_t(compact3(cc[k]));
        out->corner_cell[l - 1][3 * k + 1] = int32_t(compact3(cc[k] >> 1));
        out->corner_cell[l - 1][3 * k + 2] = int32_t(compact3(cc[k] >> 2));
      }
    }
  }
  return NGL_OK;
}

}  // extern "C"
