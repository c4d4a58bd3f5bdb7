// Primary rays and the breadth-first ray-octree intersection (Sec. 3.4,
// Alg. 1; subroutines of App. C) on gfx950.
//
// Per depth, two launches over the current list of ray-voxel pairs:
//   k_decide_count  Decide (FP32 slab tests) and a per-block sum
//   k_decide_emit   each block sums the block sums before its own (its
//                   offset of the ExclusiveSum), scans its decisions, then
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

// Decide for the occupied children of hit pair (ray, vox) at depth d: bit c
// of the result is set iff child c exists and the ray hits its box.
__device__ inline uint32_t decide_children(const ngl_model& md, int d, const float o[3], const float inv[3],
                                           int32_t vox, uint32_t* cmask, int32_t* fc) {
  const uint32_t c = md.cell[d][vox];
  const uint32_t m = md.child_mask[d][vox];
  *cmask = m;
  *fc = md.first_child[d][vox];
  uint32_t hm = 0;
  const ChildSlabs S(o, inv, c, d);
#pragma unroll
  for (int ch = 0; ch < 8; ++ch) {
    float ti, to;
    if ((m >> ch & 1u) && S.test(ch, ti, to)) hm |= 1u << ch;
  }
  return hm;
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

__device__ inline int64_t list_size(const Level& L, bool root) {
  if (root) return L.R;
  const int64_t n = *L.n_in;
  return n < L.cap ? n : L.cap;
}

template <bool ROOT>
__global__ __launch_bounds__(kBlock) void k_decide_count(ngl_model md, Level L) {
  const int64_t n = list_size(L, ROOT);
  int64_t begin, end;
  chunk_of(n, begin, end);
  uint32_t local = 0;
  for (int64_t t = begin + threadIdx.x; t < end; t += kBlock) {
    if constexpr (ROOT) {
      float ti, to;
      local += decide_root(L, t, ti, to);
    } else {
      float o[3], inv[3];
      load_ray(L, L.ray_in[t], o, inv);
      uint32_t cm;
      int32_t fc;
      const uint32_t hm = decide_children(md, L.depth, o, inv, L.vox_in[t], &cm, &fc);
      L.hmask[t] = uint8_t(hm);
      local += uint32_t(__popc(hm));
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

template <bool ROOT>
__global__ __launch_bounds__(kBlock) void k_decide_emit(ngl_model md, Level L) {
  const int64_t n = list_size(L, ROOT);
  int64_t begin, end;
  chunk_of(n, begin, end);
  __shared__ uint32_t part[kBlock / 64];
  // this block's offset: the sum of the block sums before it; the last block
  // also reports the list size
  int64_t offset;
  {
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
    offset = int64_t(o);
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
      const int64_t total = offset + int64_t(L.bsum[blockIdx.x]);
      *L.n_out = total;
      if (total > L.counts[1]) L.counts[1] = total;
      if (L.final_out) L.counts[0] = total;
    }
  }
  const int64_t cap = L.cap;
  for (int64_t base = begin; base < end; base += kBlock) {
    const int64_t t = base + threadIdx.x;
    uint32_t D = 0, hm = 0;
    float ti = 0.0f, to = 0.0f;
    if (t < end) {
      if constexpr (ROOT) {
        D = decide_root(L, t, ti, to);
      } else {
        hm = L.hmask[t];
        D = uint32_t(__popc(hm));
      }
    }
    const uint32_t incl = wave_incl_scan(D);
    if ((threadIdx.x & 63) == 63) part[threadIdx.x >> 6] = incl;
    __syncthreads();
    uint32_t pre = 0, tile = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      const uint32_t s = part[w];
      if (w < int(threadIdx.x >> 6)) pre += s;
      tile += s;
    }
    __syncthreads();
    if (D) {
      int64_t k = offset + pre + incl - D;
      if constexpr (ROOT) {
        // Compactify (root pass): keep the rays that hit the root
        if (k < cap) {
          L.ray_out[k] = int32_t(t);
          L.vox_out[k] = 0;
          if (L.final_out) {
            L.tin_out[k] = ti;
            L.tout_out[k] = to;
          }
        }
      } else {
        // Subdivide: hit children front to back, child = q XOR oct
        const int32_t ray = L.ray_in[t];
        const int32_t vox = L.vox_in[t];
        float o[3], inv[3];
        load_ray(L, ray, o, inv);
        const int d = L.depth;
        const uint32_t c = md.cell[d][vox];
        const uint32_t m = md.child_mask[d][vox];
        const int32_t fc = md.first_child[d][vox];
        const float step = 2.0f / float(1 << d);
        const int ijk[3] = {cell_x(c), cell_y(c), cell_z(c)};
        int oct = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float centre = -1.0f + (float(ijk[a]) + 0.5f) * step;  // exact dyadic
          oct |= (o[a] > centre ? 1 : 0) << a;
        }
        const ChildSlabs S(o, inv, c, d);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int ch = q ^ oct;
          if (hm >> ch & 1u) {
            if (k < cap) {
              L.ray_out[k] = ray;
              L.vox_out[k] = fc + __popc(m & ((1u << ch) - 1u));
              if (L.final_out) {
                float a0, a1;
                S.test(ch, a0, a1);
                L.tin_out[k] = a0;
                L.tout_out[k] = a1;
              }
            }
            ++k;
          }
        }
      }
    }
    offset += tile;
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
      k_decide_emit<true><<<kTravGrid, kBlock, 0, s>>>(*m, L);
    } else {
      k_decide_count<false><<<kTravGrid, kBlock, 0, s>>>(*m, L);
      k_decide_emit<false><<<kTravGrid, kBlock, 0, s>>>(*m, L);
    }
  }
  k_ray_offsets<<<unsigned((R + 1 + kBlock - 1) / kBlock), kBlock, 0, s>>>(pair_ray, counts, pair_capacity, R,
                                                                            ray_off);
  NGL_LAUNCHED();
  return NGL_OK;
}

}  // extern "C"
