// Sparse voxel octree from finest-level occupancy on the device (Sec. 3.2;
// App. A.1): the same canonical layout as the host build, bit for bit.
//   1. Morton codes of the occupied cells, radix sort, unique -> depth D.
//   2. Parent closure: depth d is the unique list of depth d+1 codes >> 3
//      (sorted children give sorted parents); a child's parent index is the
//      running count of new parents, a parent's first child the position of
//      its first child, its mask the OR of its (at most 8) children's octants.
//   3. Per feature level, the 8 lattice corners of every voxel as
//      (corner code, 8v + j) pairs, stably sorted by code: the unique codes
//      are the level's corners, each pair's rank its corner index, and the
//      sorted pairs are the corner -> (voxel, slot) adjacency.
// Sizes stay on the device; arrays are caller-allocated to upper bounds.
#include "ngl_common.h"
#include "ngl_device.h"
#include "ngl_sort.h"

#include <algorithm>

namespace ngl {

__device__ inline uint32_t spread3_u32(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ inline uint32_t compact3_u32(uint32_t v) {
  v &= 0x09249249u;
  v = (v ^ (v >> 2)) & 0x030C30C3u;
  v = (v ^ (v >> 4)) & 0x0300F00Fu;
  v = (v ^ (v >> 8)) & 0x030000FFu;
  v = (v ^ (v >> 16)) & 0x000003FFu;
  return v;
}

__device__ inline uint32_t morton3_u32(uint32_t x, uint32_t y, uint32_t z) {
  return spread3_u32(x) | spread3_u32(y) << 1 | spread3_u32(z) << 2;
}

// Keys of the occupied cells; cells outside [0, res)^3 get the key 2^31
// (sorted last and dropped) and are counted in *bad.
static __global__ __launch_bounds__(kBlock) void k_oct_keys(const int32_t* __restrict__ ijk, int64_t n, int res,
                                                            uint32_t* key, uint32_t* val, int64_t* bad) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= n) return;
  const int32_t x = ijk[3 * k], y = ijk[3 * k + 1], z = ijk[3 * k + 2];
  const bool ok = x >= 0 && y >= 0 && z >= 0 && x < res && y < res && z < res;
  key[k] = ok ? morton3_u32(uint32_t(x), uint32_t(y), uint32_t(z)) : 0x80000000u;
  val[k] = uint32_t(k);
  if (!ok) atomicAdd(reinterpret_cast<unsigned long long*>(bad), 1ull);
}

// New-run flags of a sorted list (after shifting each entry right by
// `shift` bits); entries >= limit (invalid keys) are never new.  n is read
// from *n_dev when given.
static __global__ __launch_bounds__(kBlock) void k_oct_flags(const uint32_t* __restrict__ c, int64_t n_max,
                                                             const int64_t* n_dev, int shift, uint32_t limit,
                                                             uint32_t* flag, uint32_t* pos) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t n = n_dev ? *n_dev : n_max;
  if (i >= n_max) return;
  uint32_t f = 0;
  if (i < n && c[i] < limit) f = (i == 0 || (c[i] >> shift) != (c[i - 1] >> shift)) ? 1u : 0u;
  flag[i] = f;
  pos[i] = f;  // scanned in place next
}

// After the exclusive scan of the flags (pos) and their total (*cnt32):
// out_code[pos] = c >> shift for new entries; first[pos] = i; parent[i] =
// index of i's run (nullable arrays are skipped).  *count = total.
static __global__ __launch_bounds__(kBlock) void k_oct_compact(const uint32_t* __restrict__ c, int64_t n_max,
                                                               const int64_t* n_dev, int shift, uint32_t limit,
                                                               const uint32_t* __restrict__ pos,
                                                               const uint32_t* __restrict__ flag, uint32_t* out_code,
                                                               int32_t* first, int32_t* parent,
                                                               const uint32_t* cnt32, int64_t* count) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t n = n_dev ? *n_dev : n_max;
  if (i == 0) *count = int64_t(*cnt32);
  if (i >= n || c[i] >= limit) return;
  const uint32_t p = pos[i] + flag[i] - 1u;  // index of this entry's run
  if (flag[i]) {
    out_code[p] = c[i] >> shift;
    if (first) first[p] = int32_t(i);
  }
  if (parent) parent[i] = int32_t(p);
}

// Per voxel of depth d: packed cell; child mask from its children's
// octants (children [first[v], first[v+1]) of the depth d+1 codes).  At
// the finest depth (no children) mask 0 and first child -1 where asked.
static __global__ __launch_bounds__(kBlock) void k_oct_cells(const uint32_t* __restrict__ code,
                                                             const int64_t* __restrict__ nv, int64_t n_max,
                                                             const int32_t* __restrict__ first,
                                                             const uint32_t* __restrict__ child_code,
                                                             const int64_t* __restrict__ nchild, uint32_t* cell,
                                                             uint8_t* mask, int32_t* leaf_first) {
  const int64_t v = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (v >= n_max || v >= *nv) return;
  const uint32_t c = code[v];
  cell[v] = compact3_u32(c) | compact3_u32(c >> 1) << 10 | compact3_u32(c >> 2) << 20;
  if (!first) {
    if (mask) mask[v] = 0;
    if (leaf_first) leaf_first[v] = -1;
    return;
  }
  if (mask) {
    const int64_t b = first[v];
    const int64_t e = v + 1 < *nv ? int64_t(first[v + 1]) : *nchild;
    uint32_t mk = 0;
    for (int64_t k = b; k < e; ++k) mk |= 1u << (child_code[k] & 7u);
    mask[v] = uint8_t(mk);
  }
}

// (corner code, 8v + j) for every voxel v of a level (depth l+1).
static __global__ __launch_bounds__(kBlock) void k_oct_corner_keys(const uint32_t* __restrict__ code,
                                                                   const int64_t* __restrict__ nv, int64_t n_max,
                                                                   uint32_t* key, uint32_t* val) {
  const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= 8 * n_max) return;
  const int64_t v = e >> 3;
  const uint32_t j = uint32_t(e & 7);
  if (v >= *nv) {
    key[e] = 0xffffffffu;
    val[e] = uint32_t(e);
    return;
  }
  const uint32_t c = code[v];
  const uint32_t x = compact3_u32(c), y = compact3_u32(c >> 1), z = compact3_u32(c >> 2);
  key[e] = morton3_u32(x + (j & 1u), y + ((j >> 1) & 1u), z + ((j >> 2) & 1u));
  val[e] = uint32_t(e);
}

// Corner tables from the sorted pairs: corners[8v + j] = corner index,
// corner_cell, adjacency CSR (offsets at run starts, entries = 8v + j).
static __global__ __launch_bounds__(kBlock) void k_oct_corner_out(const uint32_t* __restrict__ key,
                                                                  const uint32_t* __restrict__ val, int64_t m_max,
                                                                  const int64_t* __restrict__ nv,
                                                                  const uint32_t* __restrict__ pos,
                                                                  const uint32_t* __restrict__ flag,
                                                                  const uint32_t* __restrict__ ncorner32,
                                                                  int32_t* corners, int32_t* corner_cell,
                                                                  int32_t* adj_off, int32_t* adj, int64_t* ncorner) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t m = 8 * (*nv);
  if (i == 0) {
    *ncorner = int64_t(*ncorner32);
    if (adj_off) adj_off[*ncorner32] = int32_t(m);
  }
  if (i >= m_max || i >= m) return;
  const uint32_t ci = pos[i] + flag[i] - 1u;
  corners[val[i]] = int32_t(ci);
  if (adj) adj[i] = int32_t(val[i]);
  if (flag[i]) {
    if (adj_off) adj_off[ci] = int32_t(i);
    if (corner_cell) {
      const uint32_t c = key[i];
      corner_cell[3 * ci] = int32_t(compact3_u32(c));
      corner_cell[3 * ci + 1] = int32_t(compact3_u32(c >> 1));
      corner_cell[3 * ci + 2] = int32_t(compact3_u32(c >> 2));
    }
  }
}

static __global__ void k_oct_init(int64_t* bad, int32_t* parent0) {
  if (threadIdx.x == 0) {
    *bad = 0;
    parent0[0] = -1;
  }
}

static __global__ void k_oct_copy_count(const uint32_t* src, int64_t* dst) {
  if (threadIdx.x == 0) *dst = int64_t(*src);
}

struct OctWS {
  uint32_t* key[2];
  uint32_t* val[2];
  uint32_t* flag;
  uint32_t* pos;
  uint32_t* hist;
  uint32_t* cnt32;   // [4]
  uint32_t* code[NGL_MAX_DEPTH];
  size_t bytes = 0;
};

static OctWS oct_carve(void* base, int64_t n, int D) {
  OctWS w;
  char* p = static_cast<char*>(base);
  size_t off = 0;
  auto take = [&](size_t b) -> void* {
    void* r = p ? p + off : nullptr;
    off += (b + 255) & ~size_t(255);
    return r;
  };
  const int64_t m = 8 * std::max<int64_t>(n, 1);  // largest sorted list (corner pairs)
  for (int k = 0; k < 2; ++k) {
    w.key[k] = static_cast<uint32_t*>(take(4 * size_t(m)));
    w.val[k] = static_cast<uint32_t*>(take(4 * size_t(m)));
  }
  w.flag = static_cast<uint32_t*>(take(4 * size_t(m)));
  w.pos = static_cast<uint32_t*>(take(4 * size_t(m)));
  w.hist = static_cast<uint32_t*>(take(4 * 256 * 512));
  w.cnt32 = static_cast<uint32_t*>(take(16));
  for (int d = 0; d <= D; ++d) w.code[d] = static_cast<uint32_t*>(take(4 * size_t(std::max<int64_t>(n, 1))));
  w.bytes = off;
  return w;
}

static int sort_grid_for(int64_t n) { return int(std::min<int64_t>(512, std::max<int64_t>(1, (n + 1023) / 1024))); }

}  // namespace ngl

extern "C" {

int ngl_octree_build_device_workspace(int64_t n, int32_t num_lods, size_t* bytes) {
  NGL_REQUIRE(bytes != nullptr && n >= 0 && n < (int64_t(1) << 28), "bad arguments");
  NGL_REQUIRE(num_lods >= 1 && num_lods <= NGL_MAX_LODS, "num_lods %d outside 1..%d", num_lods, NGL_MAX_LODS);
  *bytes = ngl::oct_carve(nullptr, n, num_lods + 1).bytes;
  return NGL_OK;
}

int ngl_octree_build_device(const int32_t* ijk, int64_t n, int32_t num_lods, const ngl_octree_device* out,
                            void* ws, size_t ws_bytes, void* stream) {
  using namespace ngl;
  NGL_REQUIRE(out != nullptr, "output struct is null");
  NGL_REQUIRE(n >= 0 && n < (int64_t(1) << 28), "cell count out of range");
  NGL_REQUIRE(num_lods >= 1 && num_lods <= NGL_MAX_LODS, "num_lods %d outside 1..%d", num_lods, NGL_MAX_LODS);
  NGL_REQUIRE(n == 0 || ijk != nullptr, "ijk is null");
  const int L = num_lods, D = L + 1;
  OctWS w = oct_carve(ws, n, D);
  NGL_REQUIRE(ws != nullptr && ws_bytes >= w.bytes, "workspace too small: %zu < %zu bytes", ws_bytes, w.bytes);
  NGL_REQUIRE(out->nvox && out->ncorner && out->bad, "count arrays are null");
  for (int d = 0; d <= D; ++d) {
    NGL_REQUIRE(out->cell[d] && out->parent[d], "cell or parent array of depth %d is null", d);
    if (d < D) NGL_REQUIRE(out->child_mask[d] && out->first_child[d], "child arrays of depth %d are null", d);
  }
  for (int l = 1; l <= L; ++l)
    NGL_REQUIRE((out->corner_adj_off[l - 1] == nullptr) == (out->corner_adj[l - 1] == nullptr),
                "corner adjacency of level %d needs both arrays or neither", l);
  for (int l = 1; l <= L; ++l) NGL_REQUIRE(out->corners[l - 1], "corners of level %d are null", l);
  hipStream_t s = (hipStream_t)stream;
  const int64_t nn = std::max<int64_t>(n, 1);
  const unsigned g1 = unsigned((nn + kBlock - 1) / kBlock);
  k_oct_init<<<1, 64, 0, s>>>(out->bad, out->parent[0]);
  // 1. finest depth: keys, sort, unique
  if (n > 0) k_oct_keys<<<g1, kBlock, 0, s>>>(ijk, n, 1 << D, w.key[0], w.val[0], out->bad);
  int cur = 0;
  if (n > 0) cur = radix_sort_pairs(w.key, w.val, n, 32, sort_grid_for(n), w.hist, s);
  const uint32_t* sorted = w.key[cur];
  k_oct_flags<<<g1, kBlock, 0, s>>>(sorted, n, nullptr, 0, 0x80000000u, w.flag, w.pos);
  k_scan_inplace<<<1, 1024, 0, s>>>(w.pos, n, w.cnt32);
  k_oct_compact<<<g1, kBlock, 0, s>>>(sorted, n, nullptr, 0, 0x80000000u, w.pos, w.flag, w.code[D], nullptr, nullptr,
                                      w.cnt32, out->nvox + D);
  // 2. parent closure, deepest first
  for (int d = D - 1; d >= 0; --d) {
    k_oct_flags<<<g1, kBlock, 0, s>>>(w.code[d + 1], n, out->nvox + d + 1, 3, 0xffffffffu, w.flag, w.pos);
    k_scan_inplace<<<1, 1024, 0, s>>>(w.pos, n, w.cnt32);
    k_oct_compact<<<g1, kBlock, 0, s>>>(w.code[d + 1], n, out->nvox + d + 1, 3, 0xffffffffu, w.pos, w.flag,
                                        w.code[d], out->first_child[d], out->parent[d + 1], w.cnt32, out->nvox + d);
  }
  for (int d = 0; d <= D; ++d)
    k_oct_cells<<<g1, kBlock, 0, s>>>(w.code[d], out->nvox + d, n, d < D ? out->first_child[d] : nullptr,
                                      d < D ? w.code[d + 1] : nullptr, d < D ? out->nvox + d + 1 : nullptr,
                                      out->cell[d], out->child_mask[d], d < D ? nullptr : out->first_child[d]);
  // 3. corners per level; depth l+1 holds at most min(n, 8^(l+1)) voxels
  for (int l = 1; l <= L; ++l) {
    const int64_t nl = (l + 1) * 3 < 62 ? std::min<int64_t>(nn, int64_t(1) << (3 * (l + 1))) : nn;
    const int64_t m = 8 * nl;
    const unsigned g8 = unsigned((m + kBlock - 1) / kBlock);
    // all m entries are written (sentinels past the level's voxels)
    k_oct_corner_keys<<<g8, kBlock, 0, s>>>(w.code[l + 1], out->nvox + l + 1, nl, w.key[0], w.val[0]);
    const int bits = 3 * (l + 2);
    const int c = radix_sort_pairs(w.key, w.val, m, bits <= 32 ? bits : 32, sort_grid_for(m), w.hist, s);
    k_oct_flags<<<g8, kBlock, 0, s>>>(w.key[c], m, nullptr, 0, 0xffffffffu, w.flag, w.pos);
    k_scan_inplace<<<1, 1024, 0, s>>>(w.pos, m, w.cnt32);
    k_oct_corner_out<<<g8, kBlock, 0, s>>>(w.key[c], w.val[c], m, out->nvox + l + 1, w.pos, w.flag, w.cnt32,
                                           out->corners[l - 1], out->corner_cell[l - 1], out->corner_adj_off[l - 1],
                                           out->corner_adj[l - 1], out->ncorner + l - 1);
  }
  NGL_LAUNCHED();
  return NGL_OK;
}

}  // extern "C"
