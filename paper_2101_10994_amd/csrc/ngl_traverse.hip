// Primary rays and the breadth-first ray-octree intersection (Sec. 3.4,
// Alg. 1; subroutines of App. C) on gfx950.
//
// Per depth, two launches over the current list of ray-voxel pairs:
//   k_decide_count  Decide (FP32 slab tests) and a per-block sum
//   k_child_emit    each block sums the block sums before its own (its
//   / k_root_emit   offset of the ExclusiveSum), scans its decisions, then
//                   Subdivide (children front to back) or Compactify
// so the global ExclusiveSum is reduce-then-scan with the block partition
// fixed by (list size, grid).  Lists live in caller workspace, sizes stay
// on the device: no host synchronisation between depths.
#include "ngl_common.h"
#include "ngl_device.h"

namespace ngl {

constexpr int kTravGrid = 2048;  // blocks per pass; each owns a contiguous chunk

// ---------------------------------------------------------------------------
// Camera rays
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_camera(float ex, float ey, float ez, float fx, float fy, float fz,
                                                   float rx, float ry, float rz, float ux, float uy, float uz,
                                                   float sxs, float sys, int W, int H, float* __restrict__ o,
                                                   float* __restrict__ d) {
  const int64_t R = int64_t(W) * H;
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= R) return;
  const int row = int(i / W), col = int(i - int64_t(row) * W);
  const float sx = (2.0f * (float(col) + 0.5f) / float(W) - 1.0f) * sxs;
  const float sy = (1.0f - 2.0f * (float(row) + 0.5f) / float(H)) * sys;
  const float vx = fx + sx * rx + sy * ux;
  const float vy = fy + sx * ry + sy * uy;
  const float vz = fz + sx * rz + sy * uz;
  const float n = sqrtf(vx * vx + vy * vy + vz * vz);
  o[i] = ex;
  o[R + i] = ey;
  o[2 * R + i] = ez;
  d[i] = vx / n;
  d[R + i] = vy / n;
  d[2 * R + i] = vz / n;
}

// Correctly rounded reciprocal direction per ray, reused by every depth.
__global__ __launch_bounds__(kBlock) void k_ray_inv(const float* __restrict__ d, int64_t R, float* __restrict__ inv) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= R) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) inv[a * R + i] = __fdiv_rn(1.0f, d[a * R + i]);
}

// ---------------------------------------------------------------------------
// Traversal
// ---------------------------------------------------------------------------
// Lists hold only pairs whose box the ray hits.  The root pass decides the
// root for every ray; the pass from depth d decides every occupied child of
// each hit pair (the Decide of depth d+1, evaluated while subdividing), so
// D = number of hit children, and Subdivide writes exactly those children
// front to back at the exclusive-sum offset.  The final list equals the one
// produced by deciding all occupied children at the next depth first.
struct Level {
  const float* o;         // [3][R]
  const float* inv;       // [3][R]
  int64_t R;
  const int32_t* ray_in;  // hit pairs at `depth` (unused by the root pass)
  const int32_t* vox_in;
  const int64_t* n_in;    // device list size
  uint8_t* hmask;         // [cap] hit-children mask per input pair (child passes)
  int depth;              // depth of the input list (root pass: 0)
  bool final_out;         // the produced list is at the target depth
  int64_t cap;
  uint32_t* bsum;         // [kTravGrid] block sums
  int64_t* n_out;         // device size of the produced list
  int64_t* counts;        // [0] final pair count, [1] largest list needed
  int32_t* ray_out;
  int32_t* vox_out;
  float* tin_out;         // target depth only
  float* tout_out;
};

// Contiguous chunk of the list owned by block b (multiple of the block size).
__device__ inline void chunk_of(int64_t n, int64_t& begin, int64_t& end) {
  int64_t chunk = (n + kTravGrid - 1) / kTravGrid;
  chunk = (chunk + kBlock - 1) / kBlock * kBlock;
  begin = int64_t(blockIdx.x) * chunk;
  end = begin + chunk < n ? begin + chunk : n;
}

__device__ inline void load_ray(const Level& L, int32_t ray, float o[3], float inv[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    o[a] = L.o[a * L.R + ray];
    inv[a] = L.inv[a * L.R + ray];
  }
}

// Decide for the root: 1 if the ray hits [-1,1]^3.
__device__ inline uint32_t decide_root(const Level& L, int64_t t, float& tin, float& tout) {
  float o[3], inv[3], lo[3], hi[3];
  load_ray(L, int32_t(t), o, inv);
  box_of(0u, 0, lo, hi);
  return slab_f32(o, inv, lo, hi, tin, tout) ? 1u : 0u;
}

__device__ inline uint32_t wave_incl_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

// Inclusive scan of four 16-bit counters packed in one word (no carries:
// every partial sum stays below 2^16).
__device__ inline uint64_t wave_incl_scan4(uint64_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint64_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

__device__ inline uint32_t field16(uint64_t x, int u) { return uint32_t(x >> (16 * u)) & 0xffffu; }

__device__ inline int64_t list_size(const Level& L, bool root) {
  if (root) return L.R;
  const int64_t n = *L.n_in;
  return n < L.cap ? n : L.cap;
}

// Each thread takes kTravU pairs of a block chunk at a time, kBlock apart
// (coalesced), and issues every load of the group before its first use.
constexpr int kTravU = 4;

// Inputs of the child Decide of pair t (ray, voxel and its cell record).
struct PairIn {
  int32_t ray, vox, fc;
  uint32_t cell, mask;
  float o[3], inv[3];
};

__device__ inline void load_pairs(const ngl_model& md, const Level& L, const int64_t (&t)[kTravU],
                                  const bool (&live)[kTravU], PairIn (&p)[kTravU]) {
#pragma unroll
  for (int u = 0; u < kTravU; ++u) {
    p[u].ray = live[u] ? L.ray_in[t[u]] : 0;
    p[u].vox = live[u] ? L.vox_in[t[u]] : 0;
  }
  const int d = L.depth;
#pragma unroll
  for (int u = 0; u < kTravU; ++u) {
    if (live[u]) {
      load_ray(L, p[u].ray, p[u].o, p[u].inv);
      p[u].cell = md.cell[d][p[u].vox];
      p[u].mask = md.child_mask[d][p[u].vox];
      p[u].fc = md.first_child[d][p[u].vox];
    }
  }
}

// Bit ch of the result: child ch exists and the ray hits its box.
__device__ inline uint32_t hit_children(const PairIn& p, int d) {
  return ChildSlabs(p.o, p.inv, p.cell, d).hit_mask(p.mask);
}

template <bool ROOT>
__global__ __launch_bounds__(kBlock) void k_decide_count(ngl_model md, Level L) {
  const int64_t n = list_size(L, ROOT);
  int64_t begin, end;
  chunk_of(n, begin, end);
  uint32_t local = 0;
  for (int64_t base = begin + threadIdx.x; base < end; base += kTravU * kBlock) {
    int64_t t[kTravU];
    bool live[kTravU];
#pragma unroll
    for (int u = 0; u < kTravU; ++u) {
      t[u] = base + u * kBlock;
      live[u] = t[u] < end;
    }
    if constexpr (ROOT) {
#pragma unroll
      for (int u = 0; u < kTravU; ++u) {
        float ti, to;
        if (live[u]) local += decide_root(L, t[u], ti, to);
      }
    } else {
      PairIn p[kTravU];
      load_pairs(md, L, t, live, p);
#pragma unroll
      for (int u = 0; u < kTravU; ++u) {
        if (live[u]) {
          const uint32_t hm = hit_children(p[u], L.depth);
          L.hmask[t[u]] = uint8_t(hm);
          local += uint32_t(__popc(hm));
        }
      }
    }
  }
  __shared__ uint32_t part[kBlock / 64];
  const uint32_t w = wave_incl_scan(local);
  if ((threadIdx.x & 63) == 63) part[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kBlock / 64; ++k) s += part[k];
    L.bsum[blockIdx.x] = s;
  }
}

// Block offset of the ExclusiveSum: the sum of the block sums before this
// block; the last block also reports the list size.
__device__ inline int64_t block_offset(const Level& L) {
  __shared__ uint64_t red[kBlock / 64];
  uint64_t v = 0;
  for (int b = threadIdx.x; b < int(blockIdx.x); b += kBlock) v += L.bsum[b];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t o = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) o += red[w];
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    const int64_t total = int64_t(o) + int64_t(L.bsum[blockIdx.x]);
    *L.n_out = total;
    if (total > L.counts[1]) L.counts[1] = total;
    if (L.final_out) L.counts[0] = total;
  }
  return int64_t(o);
}

// Block-wide exclusive scan of kTravU counts per thread (pair (u, thread) in
// list order u*kBlock + thread): start of each pair within the group and
// the group total.
__device__ inline void group_scan(const uint32_t (&D)[kTravU], uint32_t (&start)[kTravU], uint32_t& total) {
  __shared__ uint64_t part[kBlock / 64];
  uint64_t packed = 0;
#pragma unroll
  for (int u = 0; u < kTravU; ++u) packed |= uint64_t(D[u]) << (16 * u);
  const uint64_t incl = wave_incl_scan4(packed);
  if ((threadIdx.x & 63) == 63) part[threadIdx.x >> 6] = incl;
  __syncthreads();
  uint64_t pre = 0, tile = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    const uint64_t s = part[w];
    if (w < int(threadIdx.x >> 6)) pre += s;
    tile += s;
  }
  __syncthreads();
  uint32_t before = 0;
#pragma unroll
  for (int u = 0; u < kTravU; ++u) {
    start[u] = before + field16(pre, u) + field16(incl, u) - D[u];
    before += field16(tile, u);
  }
  total = before;
}

// Root pass: Compactify the rays that hit the root (at most one output per
// input, so the writes are already in order).
__global__ __launch_bounds__(kBlock) void k_root_emit(ngl_model md, Level L) {
  const int64_t n = list_size(L, true);
  int64_t begin, end;
  chunk_of(n, begin, end);
  int64_t offset = block_offset(L);
  const int64_t cap = L.cap;
  for (int64_t base = begin; base < end; base += kTravU * kBlock) {
    uint32_t D[kTravU], start[kTravU], total;
    float ti[kTravU], to[kTravU];
#pragma unroll
    for (int u = 0; u < kTravU; ++u) {
      const int64_t t = base + u * kBlock + threadIdx.x;
      D[u] = t < end ? decide_root(L, t, ti[u], to[u]) : 0u;
    }
    group_scan(D, start, total);
#pragma unroll
    for (int u = 0; u < kTravU; ++u) {
      const int64_t k = offset + start[u];
      if (D[u] && k < cap) {
        L.ray_out[k] = int32_t(base + u * kBlock + threadIdx.x);
        L.vox_out[k] = 0;
        if (L.final_out) {
          L.tin_out[k] = ti[u];
          L.tout_out[k] = to[u];
        }
      }
    }
    offset += total;
  }
}

// Child passes: Subdivide.  The hit children of a group of kTravU*kBlock
// pairs fill a contiguous output range; the pairs' records go to LDS and
// each thread then produces outputs j = thread, thread + kBlock, ... of the
// range: its pair is the last one whose start is <= j (binary search over
// the group's starts), its child the (j - start)-th hit child in front-to-
// back order (child = visit ^ oct).  Consecutive threads write consecutive
// outputs.
__global__ __launch_bounds__(kBlock) void k_child_emit(ngl_model md, Level L) {
  constexpr int G = kTravU * kBlock;
  __shared__ uint16_t s_start[G];
  __shared__ int32_t s_ray[G];
  __shared__ int32_t s_fc[G];
  __shared__ uint32_t s_cell[G];
  __shared__ uint32_t s_info[G];  // visit-order hit bits | child mask << 8 | oct << 16
  const int64_t n = list_size(L, false);
  int64_t begin, end;
  chunk_of(n, begin, end);
  int64_t offset = block_offset(L);
  const int64_t cap = L.cap;
  const int d = L.depth;
  const float step = 2.0f / float(1 << d);
  for (int64_t base = begin; base < end; base += G) {
    uint32_t D[kTravU], hm[kTravU], start[kTravU], total;
    int32_t ray[kTravU], vox[kTravU];
#pragma unroll
    for (int u = 0; u < kTravU; ++u) {
      const int64_t t = base + u * kBlock + threadIdx.x;
      hm[u] = t < end ? L.hmask[t] : 0u;
      D[u] = uint32_t(__popc(hm[u]));
      ray[u] = D[u] ? L.ray_in[t] : 0;
      vox[u] = D[u] ? L.vox_in[t] : 0;
    }
    uint32_t cell[kTravU], mask[kTravU];
    int32_t fc[kTravU];
    float o[kTravU][3];
#pragma unroll
    for (int u = 0; u < kTravU; ++u) {
      if (D[u]) {
        cell[u] = md.cell[d][vox[u]];
        mask[u] = md.child_mask[d][vox[u]];
        fc[u] = md.first_child[d][vox[u]];
#pragma unroll
        for (int a = 0; a < 3; ++a) o[u][a] = L.o[a * L.R + ray[u]];
      }
    }
    group_scan(D, start, total);
#pragma unroll
    for (int u = 0; u < kTravU; ++u) {
      const int i = u * kBlock + threadIdx.x;
      s_start[i] = uint16_t(start[u]);
      if (D[u]) {
        const int ijk[3] = {cell_x(cell[u]), cell_y(cell[u]), cell_z(cell[u])};
        int oct = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float centre = -1.0f + (float(ijk[a]) + 0.5f) * step;  // exact dyadic
          oct |= (o[u][a] > centre ? 1 : 0) << a;
        }
        uint32_t order = 0;  // bit r: the child visited r-th is hit
#pragma unroll
        for (int r = 0; r < 8; ++r) order |= ((hm[u] >> (r ^ oct)) & 1u) << r;
        s_ray[i] = ray[u];
        s_fc[i] = fc[u];
        s_cell[i] = cell[u];
        s_info[i] = order | mask[u] << 8 | uint32_t(oct) << 16;
      }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < int(total); j += kBlock) {
      int i = 0;
#pragma unroll
      for (int w = G / 2; w >= 1; w >>= 1)
        if (s_start[i + w] <= j) i += w;
      const uint32_t info = s_info[i];
      uint32_t v = info & 0xffu;
      for (int q = j - int(s_start[i]); q > 0; --q) v &= v - 1u;
      const int ch = __builtin_ctz(v) ^ int(info >> 16);
      const uint32_t m = (info >> 8) & 0xffu;
      const int64_t k = offset + j;
      if (k < cap) {
        const int32_t r = s_ray[i];
        L.ray_out[k] = r;
        L.vox_out[k] = s_fc[i] + __popc(m & ((1u << ch) - 1u));
        if (L.final_out) {
          float oo[3], inv[3], a0, a1;
          load_ray(L, r, oo, inv);
          ChildSlabs::one(oo, inv, s_cell[i], d, ch, a0, a1);
          L.tin_out[k] = a0;
          L.tout_out[k] = a1;
        }
      }
    }
    __syncthreads();
    offset += total;
  }
}

// ray_off[r] = first index of the final list whose ray is >= r (r = 0..R).
__global__ __launch_bounds__(kBlock) void k_ray_offsets(const int32_t* __restrict__ ray, const int64_t* counts,
                                                        int64_t cap, int64_t R, int32_t* __restrict__ ray_off) {
  const int64_t r = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (r > R) return;
  int64_t n = counts[0];
  n = n < cap ? n : cap;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (ray[mid] < r) lo = mid + 1;
    else hi = mid;
  }
  ray_off[r] = int32_t(lo);
}

__global__ void k_counts_init(int64_t* counts, int64_t value) {
  if (threadIdx.x == 0) {
    counts[0] = value;
    counts[1] = value;
  }
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

struct TravWS {
  float* inv;
  int32_t* ray[2];
  int32_t* vox[2];
  uint8_t* hmask;
  uint32_t* bsum;
  int64_t* nlev;
  size_t bytes;
};

static TravWS carve(void* base, int64_t R, int64_t cap) {
  TravWS w{};
  char* p = static_cast<char*>(base);
  size_t off = 0;
  auto take = [&](size_t b) {
    char* q = p ? p + off : nullptr;
    off += align256(b);
    return q;
  };
  w.inv = reinterpret_cast<float*>(take(sizeof(float) * 3 * size_t(R)));
  for (int k = 0; k < 2; ++k) {
    w.ray[k] = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * size_t(cap)));
    w.vox[k] = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * size_t(cap)));
  }
  w.hmask = reinterpret_cast<uint8_t*>(take(size_t(cap)));
  w.bsum = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * kTravGrid));
  w.nlev = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * (NGL_MAX_DEPTH + 1)));
  w.bytes = off;
  return w;
}

}  // namespace ngl

extern "C" {

int ngl_camera_rays(const float* eye, const float* target, const float* up, float fov_y_deg, int32_t width,
                    int32_t height, float* o, float* d, void* stream) {
  NGL_REQUIRE(eye && target && up, "camera vectors are null");
  NGL_REQUIRE(width > 0 && height > 0, "image size must be positive");
  NGL_REQUIRE(fov_y_deg > 0.0f && fov_y_deg < 180.0f, "fov must be in (0, 180)");
  NGL_REQUIRE(o && d, "ray buffers are null");
  double f[3], r[3], u[3], n = 0;
  for (int a = 0; a < 3; ++a) {
    f[a] = double(target[a]) - double(eye[a]);
    n += f[a] * f[a];
  }
  NGL_REQUIRE(n > 0, "eye and target coincide");
  n = std::sqrt(n);
  for (int a = 0; a < 3; ++a) f[a] /= n;
  r[0] = f[1] * up[2] - f[2] * up[1];
  r[1] = f[2] * up[0] - f[0] * up[2];
  r[2] = f[0] * up[1] - f[1] * up[0];
  n = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  NGL_REQUIRE(n > 0, "up is parallel to the view direction");
  for (int a = 0; a < 3; ++a) r[a] /= n;
  u[0] = r[1] * f[2] - r[2] * f[1];
  u[1] = r[2] * f[0] - r[0] * f[2];
  u[2] = r[0] * f[1] - r[1] * f[0];
  const double th = std::tan(double(fov_y_deg) * M_PI / 360.0);
  const double aspect = double(width) / double(height);
  const int64_t R = int64_t(width) * height;
  const unsigned grid = unsigned((R + ngl::kBlock - 1) / ngl::kBlock);
  ngl::k_camera<<<grid, ngl::kBlock, 0, (hipStream_t)stream>>>(
      eye[0], eye[1], eye[2], float(f[0]), float(f[1]), float(f[2]), float(r[0]), float(r[1]), float(r[2]),
      float(u[0]), float(u[1]), float(u[2]), float(th * aspect), float(th), width, height, o, d);
  NGL_LAUNCHED();
  return NGL_OK;
}

int ngl_trace_octree_workspace(int64_t R, int64_t pair_capacity, size_t* bytes) {
  NGL_REQUIRE(bytes && R >= 0 && pair_capacity >= 0, "invalid workspace query");
  *bytes = ngl::carve(nullptr, R, pair_capacity).bytes;
  return NGL_OK;
}

int ngl_trace_octree(const ngl_model* m, const float* o, const float* d, int64_t R, int32_t target_depth,
                     int64_t pair_capacity, void* ws, size_t ws_bytes, int32_t* pair_ray, int32_t* pair_vox,
                     float* t_in, float* t_out, int32_t* ray_off, int64_t* counts, void* stream) {
  using namespace ngl;
  int rc = check_model(m, false);
  if (rc) return rc;
  NGL_REQUIRE(R >= 0 && R < (int64_t(1) << 31), "ray count out of range");
  NGL_REQUIRE(target_depth >= 0 && target_depth <= m->num_lods + 1, "target_depth %d outside 0..%d", target_depth,
              m->num_lods + 1);
  NGL_REQUIRE(pair_capacity >= 0 && pair_capacity < (int64_t(1) << 31), "pair_capacity out of range");
  NGL_REQUIRE(counts && ray_off, "counts or ray_off is null");
  NGL_REQUIRE(R == 0 || (o && d), "ray buffers are null");
  NGL_REQUIRE(pair_capacity == 0 || (pair_ray && pair_vox && t_in && t_out), "pair buffers are null");
  TravWS w = carve(ws, R, pair_capacity);
  NGL_REQUIRE(ws != nullptr && ws_bytes >= w.bytes, "workspace too small: %zu < %zu bytes", ws_bytes, w.bytes);
  hipStream_t s = (hipStream_t)stream;
  k_counts_init<<<1, 64, 0, s>>>(counts, 0);
  if (R == 0 || m->nvox[0] == 0) {
    const int64_t n = R + 1;
    k_fill_i32<<<unsigned((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(ray_off, n, 0);
    NGL_LAUNCHED();
    return NGL_OK;
  }
  const unsigned rgrid = unsigned((R + kBlock - 1) / kBlock);
  k_ray_inv<<<rgrid, kBlock, 0, s>>>(d, R, w.inv);
  // root pass, then one pass per depth d = 0..target-1 producing depth d+1
  for (int step = -1; step < target_depth; ++step) {
    const bool root = step < 0;
    const int out_depth = root ? 0 : step + 1;
    Level L{};
    L.o = o;
    L.inv = w.inv;
    L.R = R;
    if (!root) {
      L.ray_in = w.ray[step & 1];
      L.vox_in = w.vox[step & 1];
      L.n_in = w.nlev + step;
      L.depth = step;
    }
    L.hmask = w.hmask;
    L.final_out = out_depth == target_depth;
    L.cap = pair_capacity;
    L.bsum = w.bsum;
    L.n_out = w.nlev + out_depth;
    L.counts = counts;
    if (L.final_out) {
      L.ray_out = pair_ray;
      L.vox_out = pair_vox;
      L.tin_out = t_in;
      L.tout_out = t_out;
    } else {
      L.ray_out = w.ray[out_depth & 1];
      L.vox_out = w.vox[out_depth & 1];
    }
    if (root) {
      k_decide_count<true><<<kTravGrid, kBlock, 0, s>>>(*m, L);
      k_root_emit<<<kTravGrid, kBlock, 0, s>>>(*m, L);
    } else {
      k_decide_count<false><<<kTravGrid, kBlock, 0, s>>>(*m, L);
      k_child_emit<<<kTravGrid, kBlock, 0, s>>>(*m, L);
    }
  }
  k_ray_offsets<<<unsigned((R + 1 + kBlock - 1) / kBlock), kBlock, 0, s>>>(pair_ray, counts, pair_capacity, R,
                                                                            ray_off);
  NGL_LAUNCHED();
  return NGL_OK;
}

}  // extern "C"
