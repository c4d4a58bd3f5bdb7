// Device helpers shared by the gfx950 kernels: exact point location, octree
// descent, the FP32 slab predicate, corner-feature rows and the FP32
// decoder.  Everything here is __device__ inline; each .hip file is a
// self-contained code object.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "ngl.h"

namespace ngl {

constexpr int kBlock = 256;

// Pointers read through the scalar cache: the decoder weights are uniform
// across a wavefront, so loads from this address space become s_load.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

template <typename T>
__device__ inline cptr<T> as_const(const void* p) {
  return (cptr<T>)(p);
}

// ---------------------------------------------------------------------------
// Feature rows (16-byte vector loads; FP32, FP16 or BF16 storage)
// ---------------------------------------------------------------------------
struct F32 {};
struct F16 {};
struct BF16 {};

// F<M, FT, XYZ>::run(md, args...) for the model's feature dtype and position
// input (M is fixed by the caller's translation unit).
template <template <int, typename, bool> class F, int M, typename... Args>
inline int dispatch_ft(const ngl_model& md, Args... args) {
  switch (md.feat_dtype) {
    case NGL_F32: return md.with_xyz ? F<M, F32, true>::run(md, args...) : F<M, F32, false>::run(md, args...);
    case NGL_F16: return md.with_xyz ? F<M, F16, true>::run(md, args...) : F<M, F16, false>::run(md, args...);
    default: return md.with_xyz ? F<M, BF16, true>::run(md, args...) : F<M, BF16, false>::run(md, args...);
  }
}

__device__ inline float bf16_to_f32(uint32_t bits16) { return __uint_as_float(bits16 << 16); }
__device__ inline float f16_to_f32(uint32_t bits16) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)bits16);
}

// acc[k] += w * row[k] for row `c` of a [n][M] feature table (below 4 GiB:
// rows are addressed by a 32-bit byte offset, as in load_slice).
template <int M, typename FT>
__device__ inline void axpy_row(const void* base, int c, float w, float* acc) {
  if constexpr (std::is_same<FT, F32>::value) {
    const float4* r = reinterpret_cast<const float4*>(static_cast<const char*>(base) + uint32_t(c) * uint32_t(M * 4));
#pragma unroll
    for (int q = 0; q < M / 4; ++q) {
      const float4 v = r[q];
      acc[4 * q + 0] = fmaf(w, v.x, acc[4 * q + 0]);
      acc[4 * q + 1] = fmaf(w, v.y, acc[4 * q + 1]);
      acc[4 * q + 2] = fmaf(w, v.z, acc[4 * q + 2]);
      acc[4 * q + 3] = fmaf(w, v.w, acc[4 * q + 3]);
    }
  } else {
    const uint4* r = reinterpret_cast<const uint4*>(static_cast<const char*>(base) + uint32_t(c) * uint32_t(M * 2));
#pragma unroll
    for (int q = 0; q < M / 8; ++q) {
      uint4 v = r[q];
      uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        float lo, hi;
        if constexpr (std::is_same<FT, BF16>::value) {
          lo = bf16_to_f32(wv[h] & 0xffffu);
          hi = bf16_to_f32(wv[h] >> 16);
        } else {
          lo = f16_to_f32(wv[h] & 0xffffu);
          hi = f16_to_f32(wv[h] >> 16);
        }
        acc[8 * q + 2 * h] = fmaf(w, lo, acc[8 * q + 2 * h]);
        acc[8 * q + 2 * h + 1] = fmaf(w, hi, acc[8 * q + 2 * h + 1]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Exact point location
// ---------------------------------------------------------------------------
// Half-open cell [lo, hi) of resolution r (power of two, <= 1024) containing
// x in [-1, 1]; x = +1 lies in the last cell.  The FP32 estimate is within
// one cell of the answer; one comparison against the exact dyadic bounds
// corrects it.
__device__ inline int cell_of(float x, int r) {
  const float step = 2.0f / float(r);  // exact: r is a power of two
  int i = int(floorf((x + 1.0f) * (0.5f * float(r))));
  i = min(max(i, 0), r - 1);
  if (x < -1.0f + float(i) * step) {
    i = max(i - 1, 0);
  } else if (i < r - 1 && x >= -1.0f + float(i + 1) * step) {
    i = i + 1;
  }
  return i;
}

// a[i] for a runtime i without dynamic register indexing.
template <int N>
__device__ inline int pick(const int* a, int i) {
  int r = a[0];
#pragma unroll
  for (int k = 1; k < N; ++k) r = (k == i) ? a[k] : r;
  return r;
}

__device__ inline bool in_box(float x, float y, float z) {
  return x >= -1.0f && x <= 1.0f && y >= -1.0f && y <= 1.0f && z >= -1.0f && z <= 1.0f;
}

__device__ inline uint32_t pack_cell(int x, int y, int z) { return uint32_t(x) | uint32_t(y) << 10 | uint32_t(z) << 20; }
__device__ inline int cell_x(uint32_t c) { return int(c & 1023u); }
__device__ inline int cell_y(uint32_t c) { return int(c >> 10 & 1023u); }
__device__ inline int cell_z(uint32_t c) { return int(c >> 20 & 1023u); }

// Descend from the root to depth `depth` along the cell (cx,cy,cz) given at
// that depth; vox[l-1] receives the voxel of feature level l (depth l+1)
// for l = 1..depth-1, or -1 once a voxel is absent.  *last receives the
// voxel at `depth` (or -1), and *at receives the voxel of level `want`
// (or -1), without indexing vox at run time.
template <int MAXL>
__device__ inline void descend(const ngl_model& md, int cx, int cy, int cz, int depth, int* vox, int* last = nullptr,
                               int want = -1, int* at = nullptr) {
  int v = 0;
  bool alive = md.nvox[0] > 0;
  int vl = -1, va = -1;
#pragma unroll
  for (int d = 0; d < MAXL + 1; ++d) {
    if (d < depth) {
      if (alive) {
        const int s = depth - 1 - d;
        const int c = ((cx >> s) & 1) | ((cy >> s) & 1) << 1 | ((cz >> s) & 1) << 2;
        const uint32_t mask = md.child_mask[d][v];
        if (mask >> c & 1u) {
          v = md.first_child[d][v] + __popc(mask & ((1u << c) - 1u));
        } else {
          alive = false;
        }
      }
      const int cur = alive ? v : -1;
      if (d >= 1) vox[d - 1] = cur;
      if (d == depth - 1) vl = cur;
      if (d == want) va = cur;
    }
  }
  if (last) *last = vl;
  if (at) *at = va;
}

// ---------------------------------------------------------------------------
// FP32 slab predicate (closed box, t >= 0).  Evaluated operation by
// operation exactly as stated in the library header so that hit lists are
// reproducible bit for bit.
// ---------------------------------------------------------------------------
__device__ inline bool slab_f32(const float o[3], const float inv[3], const float lo[3], const float hi[3],
                                float& t_in, float& t_out) {
#pragma clang fp contract(off)
  float tmin = -__builtin_inff(), tmax = __builtin_inff();
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (__builtin_isinf(inv[a])) {
      ok = ok && (lo[a] <= o[a] && o[a] <= hi[a]);
    } else {
      const float d0 = lo[a] - o[a];
      const float d1 = hi[a] - o[a];
      const float t0 = d0 * inv[a];
      const float t1 = d1 * inv[a];
      const float nr = t0 < t1 ? t0 : t1;
      const float fr = t0 < t1 ? t1 : t0;
      tmin = nr > tmin ? nr : tmin;
      tmax = fr < tmax ? fr : tmax;
    }
  }
  const float t0c = tmin > 0.0f ? tmin : 0.0f;
  t_in = t0c;
  t_out = tmax;
  return ok && (tmax >= t0c);
}

// Slab tests of the eight children of cell c (packed) at `depth` against one
// ray.  The children's boxes along axis a are bounded by three planes
// p_k = -1 + (2 c_a + k) 2^-depth, k = 0, 1, 2 (exact dyadic values, the
// same expressions box_of gives for the child cells), so the plane
// distances (p_k - o_a) inv_a are formed once per axis.  An axis the ray
// runs parallel to (infinite inv) enters as the interval (-inf, +inf) for
// the half holding the origin and (+inf, -inf) for the other: the first
// leaves both running bounds unchanged, the second makes the child a miss,
// which is what slab_f32's separate containment test decides.  Every child
// then takes slab_f32's compare-and-select steps in slab_f32's order
// (x, then y, then z), the x-y part shared by the two children that have
// it, so each hit child's t_in and t_out are the same bits as slab_f32 on
// its own box.
struct ChildSlabs {
  float nr[3][2], fr[3][2];  // entry and exit distance per axis and child bit
  __device__ ChildSlabs(const float o[3], const float inv[3], uint32_t c, int depth) {
#pragma clang fp contract(off)
    const float step = 2.0f / float(1 << (depth + 1));
    const int ijk[3] = {cell_x(c), cell_y(c), cell_z(c)};
    bool inf[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      // p0 + step and p0 + 2 step are exact (multiples of step within [-1, 1])
      const float p0 = -1.0f + float(2 * ijk[a]) * step;
      const float p[3] = {p0, p0 + step, p0 + 2.0f * step};
      float t[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) t[k] = (p[k] - o[a]) * inv[a];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const float t0 = t[b], t1 = t[b + 1];
        nr[a][b] = t0 < t1 ? t0 : t1;
        fr[a][b] = t0 < t1 ? t1 : t0;
      }
      inf[a] = __builtin_isinf(inv[a]);
    }
    if (__builtin_expect(inf[0] || inf[1] || inf[2], 0)) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (inf[a]) {
          const float p0 = -1.0f + float(2 * ijk[a]) * step;
          const float p[3] = {p0, p0 + step, p0 + 2.0f * step};
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            const bool inside = p[b] <= o[a] && o[a] <= p[b + 1];
            nr[a][b] = inside ? -__builtin_inff() : __builtin_inff();
            fr[a][b] = inside ? __builtin_inff() : -__builtin_inff();
          }
        }
      }
    }
  }
  // All eight children: bit ch of the result is set when bit ch of `mask`
  // is and the ray hits child ch (ch = bx | by << 1 | bz << 2); t_in and
  // t_out are written for every child and meaningful for the hit ones.
  __device__ uint32_t hits(uint32_t mask, float t_in[8], float t_out[8]) const {
#pragma clang fp contract(off)
    float mn[2][2], mx[2][2];
#pragma unroll
    for (int bx = 0; bx < 2; ++bx) {
      const float n0 = nr[0][bx] > -__builtin_inff() ? nr[0][bx] : -__builtin_inff();
      const float f0 = fr[0][bx] < __builtin_inff() ? fr[0][bx] : __builtin_inff();
#pragma unroll
      for (int by = 0; by < 2; ++by) {
        mn[bx][by] = nr[1][by] > n0 ? nr[1][by] : n0;
        mx[bx][by] = fr[1][by] < f0 ? fr[1][by] : f0;
      }
    }
    uint32_t hm = 0;
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) {
      const int bx = ch & 1, by = (ch >> 1) & 1, bz = ch >> 2;
      const float tmin = nr[2][bz] > mn[bx][by] ? nr[2][bz] : mn[bx][by];
      const float tmax = fr[2][bz] < mx[bx][by] ? fr[2][bz] : mx[bx][by];
      const float t0c = tmin > 0.0f ? tmin : 0.0f;
      t_in[ch] = t0c;
      t_out[ch] = tmax;
      hm |= ((mask >> ch) & uint32_t(tmax >= t0c)) << ch;
    }
    return hm;
  }
  // Child ch alone, the same steps and bits as hits() gives for it.
  __device__ static bool one(const float o[3], const float inv[3], uint32_t c, int depth, int ch, float& t_in,
                             float& t_out) {
#pragma clang fp contract(off)
    const float step = 2.0f / float(1 << (depth + 1));
    const int ijk[3] = {cell_x(c), cell_y(c), cell_z(c)};
    float tmin = -__builtin_inff(), tmax = __builtin_inff();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float p0 = -1.0f + float(2 * ijk[a]) * step;
      const bool b = (ch >> a) & 1;
      const float lo = b ? p0 + step : p0;
      const float hi = b ? p0 + 2.0f * step : p0 + step;
      const float t0 = (lo - o[a]) * inv[a];
      const float t1 = (hi - o[a]) * inv[a];
      float n = t0 < t1 ? t0 : t1;
      float f = t0 < t1 ? t1 : t0;
      if (__builtin_isinf(inv[a])) {
        const bool inside = lo <= o[a] && o[a] <= hi;
        n = inside ? -__builtin_inff() : __builtin_inff();
        f = inside ? __builtin_inff() : -__builtin_inff();
      }
      tmin = n > tmin ? n : tmin;
      tmax = f < tmax ? f : tmax;
    }
    const float t0c = tmin > 0.0f ? tmin : 0.0f;
    t_in = t0c;
    t_out = tmax;
    return tmax >= t0c;
  }
  // The hit bits of hits() alone.  The running bounds start at -inf and
  // +inf and never become NaN, and a NaN distance leaves them unchanged in
  // both forms, so fmaxf/fminf give the same values as the selects up to
  // the sign of zero, which the final comparison does not see.
  __device__ uint32_t hit_mask(uint32_t mask) const {
    float mn[2][2], mx[2][2];
#pragma unroll
    for (int bx = 0; bx < 2; ++bx) {
      const float n0 = fmaxf(-__builtin_inff(), nr[0][bx]);
      const float f0 = fminf(__builtin_inff(), fr[0][bx]);
#pragma unroll
      for (int by = 0; by < 2; ++by) {
        mn[bx][by] = fmaxf(n0, nr[1][by]);
        mx[bx][by] = fminf(f0, fr[1][by]);
      }
    }
    uint32_t hm = 0;
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) {
      const int bx = ch & 1, by = (ch >> 1) & 1, bz = ch >> 2;
      const float tmin = fmaxf(mn[bx][by], nr[2][bz]);
      const float tmax = fminf(mx[bx][by], fr[2][bz]);
      hm |= ((mask >> ch) & uint32_t(tmax >= fmaxf(tmin, 0.0f))) << ch;
    }
    return hm;
  }
};

// Box of cell `c` (packed) at `depth`; exact dyadic bounds.
__device__ inline void box_of(uint32_t c, int depth, float lo[3], float hi[3]) {
  const float step = 2.0f / float(1 << depth);
  const int ijk[3] = {cell_x(c), cell_y(c), cell_z(c)};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = -1.0f + float(ijk[a]) * step;
    hi[a] = -1.0f + float(ijk[a] + 1) * step;
  }
}

// ---------------------------------------------------------------------------
// Trilinear interpolation of one level's corner features (Sec. 3.2)
// ---------------------------------------------------------------------------
// acc[k] += sum_j w_j(u) Z[corner(v, j)][k], u = local position of x in
// the cell (clamped to [0,1]).
// Local position of x in cell (cx, cy, cz) of level lvl, clamped to [0,1].
__device__ inline void cell_local(int lvl, int cx, int cy, int cz, const float x[3], float u[3]) {
  const int r = 4 << (lvl - 1);
  const float step = 2.0f / float(r);
  const float half_r = 0.5f * float(r);
  const int ci[3] = {cx, cy, cz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float lo = -1.0f + float(ci[a]) * step;
    u[a] = fminf(fmaxf((x[a] - lo) * half_r, 0.0f), 1.0f);
  }
}

// Trilinear weight of corner j (bit 0: +x, bit 1: +y, bit 2: +z).
__device__ inline float corner_weight(const float u[3], int j) {
  return ((j & 1) ? u[0] : 1.0f - u[0]) * ((j & 2) ? u[1] : 1.0f - u[1]) * ((j & 4) ? u[2] : 1.0f - u[2]);
}

template <int M, typename FT>
__device__ inline void interp_level(const ngl_model& md, int lvl, int v, int cx, int cy, int cz, const float x[3],
                                    float* acc) {
  float u[3];
  cell_local(lvl, cx, cy, cz, x, u);
  const int4* cp = reinterpret_cast<const int4*>(md.corners[lvl - 1] + size_t(v) * 8);
  const int4 c0 = cp[0], c1 = cp[1];
  const int cs[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
  for (int j = 0; j < 8; ++j) axpy_row<M, FT>(md.feat[lvl - 1], cs[j], corner_weight(u, j), acc);
}

// v[i] = row[off + i] as float, i < D: a D-wide slice of row `c`.
// Rows are addressed by a 32-bit byte offset from the table base (a level's
// table is below 4 GiB), which the loads take as a scalar base plus a
// vector offset.
template <int M, typename FT, int D>
__device__ inline void load_slice(const void* base, int c, int off, float* v) {
  if constexpr (std::is_same<FT, F32>::value) {
    const uint32_t ob = uint32_t(c) * uint32_t(M * 4) + uint32_t(off * 4);
    const float* r = reinterpret_cast<const float*>(static_cast<const char*>(base) + ob);
    if constexpr (D % 4 == 0) {
#pragma unroll
      for (int q = 0; q < D / 4; ++q) {
        const float4 f = reinterpret_cast<const float4*>(r)[q];
        v[4 * q] = f.x, v[4 * q + 1] = f.y, v[4 * q + 2] = f.z, v[4 * q + 3] = f.w;
      }
    } else if constexpr (D == 2) {
      const float2 f = *reinterpret_cast<const float2*>(r);
      v[0] = f.x, v[1] = f.y;
    } else {
#pragma unroll
      for (int i = 0; i < D; ++i) v[i] = r[i];
    }
  } else {
    const uint32_t ob = uint32_t(c) * uint32_t(M * 2) + uint32_t(off * 2);
    const uint16_t* r = reinterpret_cast<const uint16_t*>(static_cast<const char*>(base) + ob);
    uint32_t h[D];
    if constexpr (D % 8 == 0) {
#pragma unroll
      for (int q = 0; q < D / 8; ++q) {
        const uint4 f = reinterpret_cast<const uint4*>(r)[q];
        const uint32_t wv[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) h[8 * q + 2 * e] = wv[e] & 0xffffu, h[8 * q + 2 * e + 1] = wv[e] >> 16;
      }
    } else if constexpr (D == 4) {
      const uint2 f = *reinterpret_cast<const uint2*>(r);
      h[0] = f.x & 0xffffu, h[1] = f.x >> 16, h[2] = f.y & 0xffffu, h[3] = f.y >> 16;
    } else if constexpr (D == 2) {
      const uint32_t f = *reinterpret_cast<const uint32_t*>(r);
      h[0] = f & 0xffffu, h[1] = f >> 16;
    } else {
#pragma unroll
      for (int i = 0; i < D; ++i) h[i] = r[i];
    }
#pragma unroll
    for (int i = 0; i < D; ++i) v[i] = std::is_same<FT, BF16>::value ? bf16_to_f32(h[i]) : f16_to_f32(h[i]);
  }
}

// acc[i] += w * row[off + i], i < D: a D-wide slice of row `c`.
template <int M, typename FT, int D>
__device__ inline void axpy_slice(const void* base, int c, int off, float w, float* acc) {
  if constexpr (std::is_same<FT, F32>::value) {
    const float* r = reinterpret_cast<const float*>(static_cast<const char*>(base) + uint32_t(c) * uint32_t(M * 4) +
                                                    uint32_t(off * 4));
    float v[D];
    if constexpr (D % 4 == 0) {
#pragma unroll
      for (int q = 0; q < D / 4; ++q) {
        const float4 f = reinterpret_cast<const float4*>(r)[q];
        v[4 * q] = f.x, v[4 * q + 1] = f.y, v[4 * q + 2] = f.z, v[4 * q + 3] = f.w;
      }
    } else if constexpr (D == 2) {
      const float2 f = *reinterpret_cast<const float2*>(r);
      v[0] = f.x, v[1] = f.y;
    } else {
#pragma unroll
      for (int i = 0; i < D; ++i) v[i] = r[i];
    }
#pragma unroll
    for (int i = 0; i < D; ++i) acc[i] = fmaf(w, v[i], acc[i]);
  } else {
    const uint16_t* r = reinterpret_cast<const uint16_t*>(static_cast<const char*>(base) + uint32_t(c) * uint32_t(M * 2) +
                                                          uint32_t(off * 2));
    uint16_t h[D];
    if constexpr (D % 8 == 0) {
#pragma unroll
      for (int q = 0; q < D / 8; ++q) {
        const uint4 f = reinterpret_cast<const uint4*>(r)[q];
        const uint32_t wv[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) h[8 * q + 2 * e] = uint16_t(wv[e] & 0xffffu), h[8 * q + 2 * e + 1] = uint16_t(wv[e] >> 16);
      }
    } else if constexpr (D == 4) {
      const uint2 f = *reinterpret_cast<const uint2*>(r);
      h[0] = uint16_t(f.x & 0xffffu), h[1] = uint16_t(f.x >> 16), h[2] = uint16_t(f.y & 0xffffu), h[3] = uint16_t(f.y >> 16);
    } else if constexpr (D == 2) {
      const uint32_t f = *reinterpret_cast<const uint32_t*>(r);
      h[0] = uint16_t(f & 0xffffu), h[1] = uint16_t(f >> 16);
    } else {
#pragma unroll
      for (int i = 0; i < D; ++i) h[i] = r[i];
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const float f = std::is_same<FT, BF16>::value ? bf16_to_f32(h[i]) : f16_to_f32(h[i]);
      acc[i] = fmaf(w, f, acc[i]);
    }
  }
}

// interp_level_slice for a voxel that may be absent (v < 0): the loads use
// voxel 0 of the level (which exists) so that they need no branch, and an
// absent voxel leaves acc unchanged, as skipping the level does.
template <int M, typename FT, int D>
__device__ inline void interp_level_slice_sel(const ngl_model& md, int lvl, int v, int cx, int cy, int cz,
                                              const float x[3], int off, float* acc);

// The slice [off, off + D) of interp_level's accumulation, with the same
// weights and the same order of operations for every feature element.
template <int M, typename FT, int D>
__device__ inline void interp_level_slice(const ngl_model& md, int lvl, int v, int cx, int cy, int cz,
                                          const float x[3], int off, float* acc) {
  float u[3];
  cell_local(lvl, cx, cy, cz, x, u);
  const int4* cp = reinterpret_cast<const int4*>(md.corners[lvl - 1] + size_t(v) * 8);
  const int4 c0 = cp[0], c1 = cp[1];
  const int cs[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
  for (int j = 0; j < 8; ++j) axpy_slice<M, FT, D>(md.feat[lvl - 1], cs[j], off, corner_weight(u, j), acc);
}

template <int M, typename FT, int D>
__device__ inline void interp_level_slice_sel(const ngl_model& md, int lvl, int v, int cx, int cy, int cz,
                                              const float x[3], int off, float* acc) {
  float t[D];
#pragma unroll
  for (int i = 0; i < D; ++i) t[i] = acc[i];
  interp_level_slice<M, FT, D>(md, lvl, v >= 0 ? v : 0, cx, cy, cz, x, off, t);
#pragma unroll
  for (int i = 0; i < D; ++i) acc[i] = v >= 0 ? t[i] : acc[i];
}

// ---------------------------------------------------------------------------
// FP32 decoder f_theta_L([x, z]) = b2 + w2 . ReLU(W1 [x; z] + b1)  (Eq. 2)
// ---------------------------------------------------------------------------
template <int M, bool XYZ>
__device__ inline float decode_f32(const ngl_model& md, int L, const float x[3], const float* z) {
  constexpr int DIN = M + (XYZ ? 3 : 0);
  constexpr int OFF = XYZ ? 3 : 0;
  cptr<float> W1 = as_const<float>(md.W1[L - 1]);
  cptr<float> b1 = as_const<float>(md.b1[L - 1]);
  cptr<float> w2 = as_const<float>(md.w2[L - 1]);
  cptr<float> b2 = as_const<float>(md.b2);
  float out = b2[L - 1];
  const int H = md.hidden;
#pragma unroll 2
  for (int k = 0; k < H; ++k) {
    cptr<float> row = W1 + k * DIN;
    float a = b1[k];
    if constexpr (XYZ) {
      a = fmaf(row[0], x[0], a);
      a = fmaf(row[1], x[1], a);
      a = fmaf(row[2], x[2], a);
    }
#pragma unroll
    for (int i = 0; i < M; ++i) a = fmaf(row[OFF + i], z[i], a);
    out = fmaf(w2[k], fmaxf(a, 0.0f), out);
  }
  return out;
}

}  // namespace ngl
