// Training forward+backward of Eq. 4 (Sec. 3.3) on gfx950.
//
// Feature gradients are accumulated without atomics, in a fixed order, so
// results are bitwise reproducible:
//   1. k_keys / radix sort: points are sorted by the Morton code of their
//      finest cell.  Canonical voxel indices are Morton ranks, so this order
//      groups the points of every voxel of every level contiguously.
//   2. k_point: per point (in sorted order) the level sum z_L, each decoder's
//      forward pass, the upstream gradient g_L, dz_L = W1_z^T (g_L w2 . 1[a>0])
//      and the suffix sums dpsi_l = sum_{L>=l} dz_L (Eq. 2 reversed).
//   3. k_dec_grad / k_dec_reduce: decoder gradients as per-block partial sums
//      over fixed point ranges, reduced in block order.
//   4. per level: k_rec_count / scan / k_rec_write reduce fixed tiles of 64
//      sorted points into per-(voxel, tile) records of sum_p w_j(p) dpsi_l(p);
//      k_vox_reduce sums each voxel's records; k_corner gathers, for every
//      corner, the partials of the (voxel, slot) pairs that share it.
#include "ngl_common.h"

#include <algorithm>
#include <cmath>
#include "ngl_device.h"
#include "ngl_sort.h"

namespace ngl {

constexpr int kSortGrid = 256;  // most blocks of the radix-sort passes
constexpr int kDecGrid = 204;   // most blocks per LOD of the decoder-gradient pass (5 LODs fill 256 CUs x 4)

// Grids sized to the batch (small batches of the fitting loop would
// otherwise pay for the full grids): at least 1024 keys per sort block and
// 64 points (one tile) per decoder-gradient block.  Deterministic for a
// given P.
inline int sort_grid(int64_t P) { return int(std::min<int64_t>(kSortGrid, std::max<int64_t>(1, (P + 1023) / 1024))); }
inline int dec_grid(int64_t P) { return int(std::min<int64_t>(kDecGrid, std::max<int64_t>(1, (P + 63) / 64))); }
constexpr int kTile = 64;       // sorted points per record tile (one wavefront)
// Batches below this many points run the per-point stage with a wavefront
// per point (k_point_wave): a lane per point would leave most of the chip
// idle and each lane's serial decoder work would set the step time.
constexpr int64_t kPointWaveMax = 16384;

__device__ inline uint32_t spread3_10(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// ---------------------------------------------------------------------------
// 1. sort keys and a stable LSD radix sort (8-bit digits)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_keys(const float* __restrict__ xs, int64_t P, int D,
                                                 uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
  const int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (p >= P) return;
  const float x = xs[p], y = xs[P + p], z = xs[2 * P + p];
  uint32_t k = 1u << (3 * D);  // outside the box: after every cell
  if (in_box(x, y, z)) {
    const int r = 1 << D;
    k = spread3_10(cell_of(x, r)) | spread3_10(cell_of(y, r)) << 1 | spread3_10(cell_of(z, r)) << 2;
  }
  key[p] = k;
  val[p] = uint32_t(p);
}

// ---------------------------------------------------------------------------
// 2. per point: forward over all LODs, upstream gradient, dz, suffix sums
// ---------------------------------------------------------------------------
struct PointArgs {
  const float* xs;
  int64_t P;
  const uint32_t* sidx;     // sorted position -> point
  const float* target;      // training: [P] (original order)
  const float* grad;        // backward only: [L][P] (original order)
  float inv_p;
  float lod_w[NGL_MAX_LODS];  // training: weight of each LOD's loss term
  float* sdf_all;           // nullable [L][P] (original order)
  float* zrows;             // [L][P][M] z_L in sorted order
  float* drows;             // [L][P][M] dpsi_l in sorted order
  float* gs;                // [L][P] g_L in sorted order
  int32_t* vox_s;           // [L][P] voxel per level in sorted order
  float* loss_part;         // [grid]
};

template <int M, bool XYZ, bool TRAIN>
__global__ __launch_bounds__(kBlock) void k_point(ngl_model md, PointArgs A) {
  const int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t P = A.P;
  float lossacc = 0.0f;
  if (p < P) {
    const int64_t id = A.sidx[p];
    const float x[3] = {A.xs[id], A.xs[P + id], A.xs[2 * P + id]};
    const int Lm = md.num_lods;
    int vox[NGL_MAX_LODS];
    int cx = 0, cy = 0, cz = 0;
    if (in_box(x[0], x[1], x[2])) {
      const int r = 1 << (Lm + 1);
      cx = cell_of(x[0], r);
      cy = cell_of(x[1], r);
      cz = cell_of(x[2], r);
      descend<NGL_MAX_LODS>(md, cx, cy, cz, Lm + 1, vox);
    } else {
#pragma unroll
      for (int l = 0; l < NGL_MAX_LODS; ++l) vox[l] = -1;
    }
    constexpr int OFF = XYZ ? 3 : 0;
    constexpr int DIN = M + OFF;
    const int H = md.hidden;
    float z[M];
#pragma unroll
    for (int k = 0; k < M; ++k) z[k] = 0.0f;
    const float tgt = TRAIN ? A.target[id] : 0.0f;
#pragma unroll
    for (int l = 1; l <= NGL_MAX_LODS; ++l) {
      if (l > Lm) break;
      const int s = Lm - l;
      if (vox[l - 1] >= 0) interp_level<M, F32>(md, l, vox[l - 1], cx >> s, cy >> s, cz >> s, x, z);
      A.vox_s[int64_t(l - 1) * P + p] = vox[l - 1];
      float4* zr = reinterpret_cast<float4*>(A.zrows + (int64_t(l - 1) * P + p) * M);
#pragma unroll
      for (int q = 0; q < M / 4; ++q) zr[q] = make_float4(z[4 * q], z[4 * q + 1], z[4 * q + 2], z[4 * q + 3]);
      // decoder L = l: forward, keeping the ReLU pattern
      cptr<float> W1 = as_const<float>(md.W1[l - 1]);
      cptr<float> b1 = as_const<float>(md.b1[l - 1]);
      cptr<float> w2 = as_const<float>(md.w2[l - 1]);
      float out = as_const<float>(md.b2)[l - 1];
      uint32_t mask[NGL_MAX_HIDDEN / 32];
#pragma unroll
      for (int q = 0; q < NGL_MAX_HIDDEN / 32; ++q) mask[q] = 0;
      for (int kb = 0; kb < H; kb += 32) {
        uint32_t mword = 0;
        const int nk = H - kb < 32 ? H - kb : 32;  // H is a multiple of 16
#pragma unroll 2
        for (int kk = 0; kk < nk; ++kk) {
          const int k = kb + kk;
          cptr<float> row = W1 + k * DIN;
          float a = b1[k];
          if constexpr (XYZ) {
            a = fmaf(row[0], x[0], a);
            a = fmaf(row[1], x[1], a);
            a = fmaf(row[2], x[2], a);
          }
#pragma unroll
          for (int i = 0; i < M; ++i) a = fmaf(row[OFF + i], z[i], a);
          mword |= (a > 0.0f ? 1u : 0u) << kk;
          out = fmaf(w2[k], fmaxf(a, 0.0f), out);
        }
#pragma unroll
        for (int q = 0; q < NGL_MAX_HIDDEN / 32; ++q)
          if (q == kb / 32) mask[q] = mword;
      }
      float g;
      if constexpr (TRAIN) {
        const float wres = A.lod_w[l - 1] * (out - tgt);
        lossacc = fmaf(wres, out - tgt, lossacc);
        g = 2.0f * wres * A.inv_p;
      } else {
        g = A.grad[int64_t(l - 1) * P + id];
      }
      if (A.sdf_all) A.sdf_all[int64_t(l - 1) * P + id] = out;
      A.gs[int64_t(l - 1) * P + p] = g;
      // dz = W1_z^T (g w2 . 1[a > 0])
      float dz[M];
#pragma unroll
      for (int i = 0; i < M; ++i) dz[i] = 0.0f;
      for (int kb = 0; kb < H; kb += 32) {
        uint32_t mword = 0;
#pragma unroll
        for (int q = 0; q < NGL_MAX_HIDDEN / 32; ++q)
          if (q == kb / 32) mword = mask[q];
        const int nk = H - kb < 32 ? H - kb : 32;
#pragma unroll 2
        for (int kk = 0; kk < nk; ++kk) {
          const int k = kb + kk;
          const float ga = (mword >> kk & 1u) ? g * w2[k] : 0.0f;
          cptr<float> row = W1 + k * DIN + OFF;
#pragma unroll
          for (int i = 0; i < M; ++i) dz[i] = fmaf(row[i], ga, dz[i]);
        }
      }
      float4* dr = reinterpret_cast<float4*>(A.drows + (int64_t(l - 1) * P + p) * M);
#pragma unroll
      for (int q = 0; q < M / 4; ++q) dr[q] = make_float4(dz[4 * q], dz[4 * q + 1], dz[4 * q + 2], dz[4 * q + 3]);
    }
    // dpsi_l = sum_{L >= l} dz_L, from the finest level down
    float acc[M];
    {
      const float4* dr = reinterpret_cast<const float4*>(A.drows + (int64_t(Lm - 1) * P + p) * M);
#pragma unroll
      for (int q = 0; q < M / 4; ++q) {
        const float4 v = dr[q];
        acc[4 * q] = v.x;
        acc[4 * q + 1] = v.y;
        acc[4 * q + 2] = v.z;
        acc[4 * q + 3] = v.w;
      }
    }
    for (int l = Lm - 1; l >= 1; --l) {
      float4* dr = reinterpret_cast<float4*>(A.drows + (int64_t(l - 1) * P + p) * M);
#pragma unroll
      for (int q = 0; q < M / 4; ++q) {
        const float4 v = dr[q];
        acc[4 * q] += v.x;
        acc[4 * q + 1] += v.y;
        acc[4 * q + 2] += v.z;
        acc[4 * q + 3] += v.w;
        dr[q] = make_float4(acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]);
      }
    }
  }
  if constexpr (TRAIN) {
    // block sum of the squared residuals in a fixed order
    __shared__ float part[kBlock / 64];
    float v = lossacc;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      float s = 0.0f;
#pragma unroll
      for (int q = 0; q < kBlock / 64; ++q) s += part[q];
      A.loss_part[blockIdx.x] = s;
    }
  }
}

// Small batches (fewer points than lanes to keep busy): one wavefront per
// sorted point, the same quantities as k_point.  Lanes split each level's
// gather (lane = corner j * 8 + slice: 8 corners x M/8 features), the
// decoders' hidden units (unit k = lane + 64 u) and the adjoint
// (lane = output i + M * part, parts summing strided unit ranges); the
// partial sums are combined by fixed butterflies, so results are
// deterministic.  The squared residual of each point goes to loss_part[p].
__device__ inline void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int M, bool XYZ, bool TRAIN>
__global__ __launch_bounds__(kBlock) void k_point_wave(ngl_model md, PointArgs A) {
  constexpr int OFF = XYZ ? 3 : 0;
  constexpr int DIN = M + OFF;
  constexpr int FE = M / 8;        // gather: features per lane (8 lanes per corner row)
  constexpr int KP = 64 / M;       // adjoint: lanes per output
  constexpr int UMAX = NGL_MAX_HIDDEN / 64;
  __shared__ float zsh[kBlock / 64][M];
  __shared__ float gash[kBlock / 64][NGL_MAX_HIDDEN];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t p = int64_t(blockIdx.x) * (kBlock / 64) + w;
  const int64_t P = A.P;
  if (p >= P) return;  // wave-uniform: no block-wide barrier below
  const int64_t id = A.sidx[p];
  const float x[3] = {A.xs[id], A.xs[P + id], A.xs[2 * P + id]};
  const int Lm = md.num_lods;
  const int H = md.hidden;
  int vox[NGL_MAX_LODS];
  int cx = 0, cy = 0, cz = 0;
  if (in_box(x[0], x[1], x[2])) {
    const int r = 1 << (Lm + 1);
    cx = cell_of(x[0], r);
    cy = cell_of(x[1], r);
    cz = cell_of(x[2], r);
    descend<NGL_MAX_LODS>(md, cx, cy, cz, Lm + 1, vox);
  } else {
#pragma unroll
    for (int l = 0; l < NGL_MAX_LODS; ++l) vox[l] = -1;
  }
  const float tgt = TRAIN ? A.target[id] : 0.0f;
  const int j = lane >> 3, sl = lane & 7;        // gather: corner, slice
  const int oi = lane % M, part = lane / M;      // adjoint: output, part
  float zl[FE];                                  // this lane's slice of z_L
#pragma unroll
  for (int e = 0; e < FE; ++e) zl[e] = 0.0f;
  float dzl[NGL_MAX_LODS];                       // dz_L[oi] (part 0 lanes)
  float lossacc = 0.0f;
#pragma unroll
  for (int l = 1; l <= NGL_MAX_LODS; ++l) {
    dzl[l - 1] = 0.0f;
    if (l > Lm) continue;
    const int s = Lm - l;
    // psi_l: corner j's slice weighted, summed over the 8 corners
    if (vox[l - 1] >= 0) {
      float u[3];
      cell_local(l, cx >> s, cy >> s, cz >> s, x, u);
      const int c = md.corners[l - 1][int64_t(vox[l - 1]) * 8 + j];
      const float wj = corner_weight(u, j);
      const float* row = static_cast<const float*>(md.feat[l - 1]) + int64_t(c) * M + sl * FE;
      float t[FE];
#pragma unroll
      for (int e = 0; e < FE; ++e) t[e] = wj * row[e];
#pragma unroll
      for (int off = 8; off < 64; off <<= 1)
#pragma unroll
        for (int e = 0; e < FE; ++e) t[e] += __shfl_xor(t[e], off, 64);
#pragma unroll
      for (int e = 0; e < FE; ++e) zl[e] += t[e];
    }
    if (lane == 0) A.vox_s[int64_t(l - 1) * P + p] = vox[l - 1];
    if (lane < 8) {
#pragma unroll
      for (int e = 0; e < FE; ++e) zsh[w][sl * FE + e] = zl[e];
    }
    wave_sync_lds();
    float z[M];
#pragma unroll
    for (int q = 0; q < M; ++q) z[q] = zsh[w][q];
    if (lane < M) A.zrows[(int64_t(l - 1) * P + p) * M + lane] = zsh[w][lane];
    // decoder L = l, units k = lane + 64 u
    const float* W1 = static_cast<const float*>(md.W1[l - 1]);
    const float* b1 = md.b1[l - 1];
    const float* w2 = md.w2[l - 1];
    float part_out = 0.0f;
    float ga[UMAX];
#pragma unroll
    for (int uu = 0; uu < UMAX; ++uu) {
      ga[uu] = 0.0f;
      const int k = lane + 64 * uu;
      if (k < H) {
        const float* rw = W1 + k * DIN;
        float a = b1[k];
        if constexpr (XYZ) {
          a = fmaf(rw[0], x[0], a);
          a = fmaf(rw[1], x[1], a);
          a = fmaf(rw[2], x[2], a);
        }
#pragma unroll
        for (int i = 0; i < M; ++i) a = fmaf(rw[OFF + i], z[i], a);
        part_out = fmaf(w2[k], fmaxf(a, 0.0f), part_out);
        ga[uu] = a > 0.0f ? w2[k] : 0.0f;  // times g below
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) part_out += __shfl_xor(part_out, off, 64);
    const float out = md.b2[l - 1] + part_out;
    float g;
    if constexpr (TRAIN) {
      const float wres = A.lod_w[l - 1] * (out - tgt);
      lossacc = fmaf(wres, out - tgt, lossacc);
      g = 2.0f * wres * A.inv_p;
    } else {
      g = A.grad[int64_t(l - 1) * P + id];
    }
    if (lane == 0) {
      if (A.sdf_all) A.sdf_all[int64_t(l - 1) * P + id] = out;
      A.gs[int64_t(l - 1) * P + p] = g;
    }
    // dz = W1_z^T (g w2 . 1[a > 0]): ga to LDS, lane (oi, part) sums units
    // part, part + KP, ...
#pragma unroll
    for (int uu = 0; uu < UMAX; ++uu) {
      const int k = lane + 64 * uu;
      if (k < H) gash[w][k] = g * ga[uu];
    }
    wave_sync_lds();
    float d = 0.0f;
    for (int k = part; k < H; k += KP) d = fmaf(W1[k * DIN + OFF + oi], gash[w][k], d);
#pragma unroll
    for (int off = M; off < 64; off <<= 1) d += __shfl_xor(d, off, 64);
    dzl[l - 1] = d;
    wave_sync_lds();  // zsh and gash are rewritten by the next level
  }
  // dpsi_l = sum_{L >= l} dz_L, from the finest level down
  if (lane < M) {
    float acc = 0.0f;
#pragma unroll
    for (int l = NGL_MAX_LODS; l >= 1; --l) {
      if (l > Lm) continue;
      acc = l == Lm ? dzl[l - 1] : acc + dzl[l - 1];
      A.drows[(int64_t(l - 1) * P + p) * M + lane] = acc;
    }
  }
  if constexpr (TRAIN) {
    if (lane == 0) A.loss_part[p] = lossacc;
  }
}

__global__ __launch_bounds__(kBlock) void k_loss_reduce(const float* __restrict__ part, int n, float inv_p,
                                                        float* __restrict__ loss) {
  __shared__ float sp[kBlock];
  float s = 0.0f;
  for (int i = threadIdx.x; i < n; i += kBlock) s += part[i];
  sp[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int i = 0; i < kBlock; ++i) t += sp[i];
    *loss = t * inv_p;
  }
}

// ---------------------------------------------------------------------------
// 3. decoder gradients: fixed per-block partial sums, then a fixed reduction
// ---------------------------------------------------------------------------
struct DecArgs {
  const float* xs;
  int64_t P;
  const uint32_t* sidx;
  const float* zrows;
  const float* gs;
  float* part;      // [L][kDecGrid][PH][H][din+2] (the first gridDim.x blocks)
  float* part_b2;   // [L][kDecGrid]
};

template <int M, bool XYZ>
__global__ __launch_bounds__(kBlock) void k_dec_grad(ngl_model md, DecArgs A) {
  constexpr int OFF = XYZ ? 3 : 0;
  constexpr int DIN = M + OFF;
  constexpr int DP = (DIN + 3) / 4 * 4;  // staged row, padded to whole 16-byte vectors
  __shared__ __align__(16) float in_s[kTile][DP];
  __shared__ float g_s[kTile];
  const int L = blockIdx.y + 1;
  const int H = md.hidden;
  const int PH = kBlock / H;
  const int k = threadIdx.x % H;
  const int ph = threadIdx.x / H;
  const int64_t P = A.P;
  cptr<float> W1 = as_const<float>(md.W1[L - 1]);
  float w[DP];
#pragma unroll
  for (int i = 0; i < DP; ++i) w[i] = i < DIN ? W1[k * DIN + i] : 0.0f;
  const float bk = as_const<float>(md.b1[L - 1])[k];
  const float w2k = as_const<float>(md.w2[L - 1])[k];
  float acc[DP];
#pragma unroll
  for (int i = 0; i < DP; ++i) acc[i] = 0.0f;
  float ab1 = 0.0f, aw2 = 0.0f, ab2 = 0.0f;
  int64_t chunk = (P + gridDim.x - 1) / gridDim.x;
  chunk = (chunk + kTile - 1) / kTile * kTile;
  const int64_t begin = int64_t(blockIdx.x) * chunk;
  const int64_t end = begin + chunk < P ? begin + chunk : P;
  for (int64_t base = begin; base < end; base += kTile) {
    for (int e = threadIdx.x; e < kTile * DP; e += kBlock) {
      const int pp = e / DP, i = e % DP;
      const int64_t p = base + pp;
      float v = 0.0f;
      if (p < end && i < DIN) {
        if (i < OFF) v = A.xs[int64_t(i) * P + A.sidx[p]];
        else v = A.zrows[(int64_t(L - 1) * P + p) * M + (i - OFF)];
      }
      in_s[pp][i] = v;
    }
    if (threadIdx.x < kTile) {
      const int64_t p = base + threadIdx.x;
      g_s[threadIdx.x] = p < end ? A.gs[int64_t(L - 1) * P + p] : 0.0f;
    }
    __syncthreads();
    for (int pp = ph; pp < kTile; pp += PH) {
      float in[DP];
#pragma unroll
      for (int q = 0; q < DP / 4; ++q) {
        const float4 v = reinterpret_cast<const float4*>(in_s[pp])[q];
        in[4 * q] = v.x;
        in[4 * q + 1] = v.y;
        in[4 * q + 2] = v.z;
        in[4 * q + 3] = v.w;
      }
      float a = bk;
#pragma unroll
      for (int i = 0; i < DIN; ++i) a = fmaf(w[i], in[i], a);
      const float g = g_s[pp];
      aw2 = fmaf(g, fmaxf(a, 0.0f), aw2);
      const float ga = a > 0.0f ? g * w2k : 0.0f;
      ab1 += ga;
#pragma unroll
      for (int i = 0; i < DIN; ++i) acc[i] = fmaf(ga, in[i], acc[i]);
    }
    if (threadIdx.x == 0)
      for (int pp = 0; pp < kTile; ++pp) ab2 += g_s[pp];
    __syncthreads();
  }
  float* dst = A.part + ((((int64_t(L - 1) * kDecGrid + blockIdx.x) * PH + ph) * H + k) * (DIN + 2));
#pragma unroll
  for (int i = 0; i < DIN; ++i) dst[i] = acc[i];
  dst[DIN] = ab1;
  dst[DIN + 1] = aw2;
  if (threadIdx.x == 0) A.part_b2[int64_t(L - 1) * kDecGrid + blockIdx.x] = ab2;
}

struct DecOut {
  float* dW1[NGL_MAX_LODS];
  float* db1[NGL_MAX_LODS];
  float* dw2[NGL_MAX_LODS];
  float* db2;
};

// Each wavefront sums one output entry's nblk * PH partials: lane i takes
// the partials i, i + 64, ... in order, then a fixed butterfly adds the
// lanes (a fixed order, so the result is reproducible).  The extra
// wavefront of block 0 sums db2.
__global__ __launch_bounds__(kBlock) void k_dec_reduce(const float* __restrict__ part,
                                                       const float* __restrict__ part_b2, int H, int din, int PH,
                                                       int nblk, DecOut O) {
  const int L = blockIdx.y + 1;
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);  // entry of [H][din+2]
  const int W = din + 2;
  const int n = nblk * PH;
  if (e < H * W) {
    const int k = e / W, i = e % W;
    float s = 0.0f;
    for (int j = lane; j < n; j += 64) {
      const int b = j / PH, ph = j % PH;
      s += part[(((int64_t(L - 1) * kDecGrid + b) * PH + ph) * H + k) * W + i];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
      if (i < din) O.dW1[L - 1][k * din + i] = s;
      else if (i == din) O.db1[L - 1][k] = s;
      else O.dw2[L - 1][k] = s;
    }
  } else if (e == H * W) {
    float s = 0.0f;
    for (int b = lane; b < nblk; b += 64) s += part_b2[int64_t(L - 1) * kDecGrid + b];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) O.db2[L - 1] = s;
  }
}

// ---------------------------------------------------------------------------
// 4. feature gradients of one level: tile records, voxel sums, corner gather
// ---------------------------------------------------------------------------
struct LevelArgs {
  const float* xs;
  int64_t P;
  int lvl;
  const uint32_t* sidx;
  const int32_t* vox_s;   // [P] this level, sorted order
  const float* drows;     // [P][M] this level, sorted order
  uint32_t* rec_cnt;      // [ntiles] counts, then exclusive offsets
  uint32_t* rec_total;    // [1]
  int32_t* rec_key;       // [maxrec] voxel of each record (ascending)
  float* recs;            // [maxrec][8][M]
  int64_t maxrec;
  float* vpart;           // [nv][8][M]
};

// Records of a tile: one per run of equal (existing) voxels.
__global__ __launch_bounds__(64) void k_rec_count(LevelArgs A) {
  const int64_t p = int64_t(blockIdx.x) * kTile + threadIdx.x;
  const int32_t v = p < A.P ? A.vox_s[p] : -1;
  const int32_t prev = (threadIdx.x > 0 && p < A.P) ? A.vox_s[p - 1] : -1;
  const bool head = v >= 0 && v != prev;
  const uint64_t heads = __ballot(head);
  if (threadIdx.x == 0) A.rec_cnt[blockIdx.x] = uint32_t(__popcll(heads));
}

// STAGE (small batches, few tiles in flight): the tile's dpsi rows are
// loaded into LDS together before the sequential pass.
template <int M, bool STAGE>
__global__ __launch_bounds__(64) void k_rec_write(ngl_model md, LevelArgs A) {
  __shared__ float w_s[kTile][8];
  __shared__ int32_t v_s[kTile];
  __shared__ uint32_t r_s[kTile];
  __shared__ float d_s[STAGE ? kTile * M : 1];
  const int lane = threadIdx.x;
  const int64_t p = int64_t(blockIdx.x) * kTile + lane;
  const int lvl = A.lvl;
  // phase A, lane = point: voxel, trilinear weights and record slot
  const int32_t v = p < A.P ? A.vox_s[p] : -1;
  const int32_t prev = (lane > 0 && p < A.P) ? A.vox_s[p - 1] : -1;
  const bool head = v >= 0 && v != prev;
  const uint64_t heads = __ballot(head);
  const uint32_t rec = A.rec_cnt[blockIdx.x] + uint32_t(__popcll(heads & ((2ull << lane) - 1ull))) - 1u;
  float wj[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) wj[j] = 0.0f;
  if (v >= 0) {
    const int64_t id = A.sidx[p];
    const float x[3] = {A.xs[id], A.xs[A.P + id], A.xs[2 * A.P + id]};
    const uint32_t c = md.cell[lvl + 1][v];
    const int ci[3] = {cell_x(c), cell_y(c), cell_z(c)};
    const int r = 4 << (lvl - 1);
    const float step = 2.0f / float(r);
    const float half_r = 0.5f * float(r);
    float u[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = fminf(fmaxf((x[a] - (-1.0f + float(ci[a]) * step)) * half_r, 0.0f), 1.0f);
#pragma unroll
    for (int j = 0; j < 8; ++j)
      wj[j] = ((j & 1) ? u[0] : 1.0f - u[0]) * ((j & 2) ? u[1] : 1.0f - u[1]) * ((j & 4) ? u[2] : 1.0f - u[2]);
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) w_s[lane][j] = wj[j];
  v_s[lane] = v;
  r_s[lane] = rec;
  const int n = int(A.P - int64_t(blockIdx.x) * kTile < kTile ? A.P - int64_t(blockIdx.x) * kTile : kTile);
  if constexpr (STAGE) {
    const float* src = A.drows + int64_t(blockIdx.x) * kTile * M;
#pragma unroll
    for (int q = 0; q < M; ++q) {
      const int e = lane + 64 * q;
      if (e < n * M) d_s[e] = src[e];
    }
  }
  __syncthreads();
  // phase B, lane = (channel, slot group): sequential over the tile's points
  constexpr int SG = 64 / M;      // slot groups
  constexpr int SPL = 8 / SG;     // slots per lane
  const int ch = lane % M;
  const int sg = lane / M;
  float acc[SPL];
#pragma unroll
  for (int s = 0; s < SPL; ++s) acc[s] = 0.0f;
  for (int i = 0; i < n; ++i) {
    const int32_t vi = v_s[i];
    if (vi < 0) continue;
    const float row = STAGE ? d_s[i * M + ch] : A.drows[(int64_t(blockIdx.x) * kTile + i) * M + ch];
#pragma unroll
    for (int s = 0; s < SPL; ++s) acc[s] = fmaf(w_s[i][sg * SPL + s], row, acc[s]);
    if (i == n - 1 || v_s[i + 1] != vi) {
      const uint32_t r = r_s[i];
      if (int64_t(r) < A.maxrec) {
#pragma unroll
        for (int s = 0; s < SPL; ++s) A.recs[(int64_t(r) * 8 + sg * SPL + s) * M + ch] = acc[s];
        if (lane == 0) A.rec_key[r] = vi;
      }
#pragma unroll
      for (int s = 0; s < SPL; ++s) acc[s] = 0.0f;
    }
  }
}

// Sum of each voxel's records (ascending record order), one wavefront per voxel.
template <int M>
__global__ __launch_bounds__(64) void k_vox_reduce(LevelArgs A, int64_t nv) {
  const int64_t v = blockIdx.x;
  if (v >= nv) return;
  const int64_t nrec = *A.rec_total < A.maxrec ? *A.rec_total : A.maxrec;
  int64_t lo = 0, hi = nrec;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (A.rec_key[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  constexpr int PER = 8 * M / 64;
  float acc[PER];
#pragma unroll
  for (int s = 0; s < PER; ++s) acc[s] = 0.0f;
  // the voxel's records are [lo, hi); eight are loaded at a time and added
  // in ascending order
  hi = nrec;
  {
    int64_t a = lo;
    while (a < hi) {
      const int64_t mid = (a + hi) >> 1;
      if (A.rec_key[mid] <= v) a = mid + 1;
      else hi = mid;
    }
  }
  int64_t r = lo;
  for (; r + 8 <= hi; r += 8) {
    float t[8][PER];
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int s = 0; s < PER; ++s) t[k][s] = A.recs[(r + k) * 8 * M + s * 64 + threadIdx.x];
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int s = 0; s < PER; ++s) acc[s] += t[k][s];
  }
  for (; r < hi; ++r) {
#pragma unroll
    for (int s = 0; s < PER; ++s) acc[s] += A.recs[r * 8 * M + s * 64 + threadIdx.x];
  }
#pragma unroll
  for (int s = 0; s < PER; ++s) A.vpart[v * 8 * M + s * 64 + threadIdx.x] = acc[s];
}

// dZ_l[c][ch] = sum over (v, j) sharing corner c of vpart[v][j][ch].
template <int M>
__global__ __launch_bounds__(kBlock) void k_corner(const int32_t* __restrict__ adj_off,
                                                   const int32_t* __restrict__ adj,
                                                   const float* __restrict__ vpart, int64_t nc,
                                                   float* __restrict__ dfeat) {
  const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= nc * M) return;
  const int64_t c = e / M;
  const int ch = int(e % M);
  float s = 0.0f;
  for (int a = adj_off[c]; a < adj_off[c + 1]; ++a) s += vpart[int64_t(adj[a]) * M + ch];
  dfeat[e] = s;
}

__global__ __launch_bounds__(kBlock) void k_zero(float* p, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

struct TrainWS {
  uint32_t* key[2];
  uint32_t* val[2];
  uint32_t* hist;
  float* zrows;
  float* drows;
  float* gs;
  int32_t* vox_s;
  float* loss_part;
  float* dec_part;
  float* dec_b2;
  uint32_t* rec_cnt;
  uint32_t* rec_total;
  int32_t* rec_key;
  float* recs;
  float* vpart;
  int64_t maxrec;
  int64_t ntiles;
  size_t bytes;
};

static TrainWS carve(const ngl_model& m, int64_t P, void* base) {
  TrainWS w{};
  char* b = static_cast<char*>(base);
  size_t off = 0;
  auto take = [&](size_t n) {
    char* q = b ? b + off : nullptr;
    off += align256(n);
    return q;
  };
  const int L = m.num_lods, M = m.feat_dim, H = m.hidden, din = M + (m.with_xyz ? 3 : 0);
  const int PH = H > 0 ? kBlock / H : 1;
  int64_t nvmax = 0;
  for (int l = 1; l <= L; ++l) nvmax = m.nvox[l + 1] > nvmax ? m.nvox[l + 1] : nvmax;
  w.ntiles = (P + kTile - 1) / kTile;
  w.maxrec = nvmax + w.ntiles;
  for (int k = 0; k < 2; ++k) {
    w.key[k] = reinterpret_cast<uint32_t*>(take(4 * size_t(P)));
    w.val[k] = reinterpret_cast<uint32_t*>(take(4 * size_t(P)));
  }
  w.hist = reinterpret_cast<uint32_t*>(take(4 * 256 * size_t(kSortGrid)));
  w.zrows = reinterpret_cast<float*>(take(4 * size_t(L) * size_t(P) * size_t(M)));
  w.drows = reinterpret_cast<float*>(take(4 * size_t(L) * size_t(P) * size_t(M)));
  w.gs = reinterpret_cast<float*>(take(4 * size_t(L) * size_t(P)));
  w.vox_s = reinterpret_cast<int32_t*>(take(4 * size_t(L) * size_t(P)));
  w.loss_part = reinterpret_cast<float*>(take(4 * size_t(P < kPointWaveMax ? P + 1 : (P + kBlock - 1) / kBlock + 1)));
  w.dec_part = reinterpret_cast<float*>(take(4 * size_t(L) * kDecGrid * PH * size_t(H) * size_t(din + 2)));
  w.dec_b2 = reinterpret_cast<float*>(take(4 * size_t(L) * kDecGrid));
  w.rec_cnt = reinterpret_cast<uint32_t*>(take(4 * size_t(w.ntiles + 1)));
  w.rec_total = reinterpret_cast<uint32_t*>(take(4));
  w.rec_key = reinterpret_cast<int32_t*>(take(4 * size_t(w.maxrec)));
  w.recs = reinterpret_cast<float*>(take(4 * 8 * size_t(M) * size_t(w.maxrec)));
  w.vpart = reinterpret_cast<float*>(take(4 * 8 * size_t(M) * size_t(nvmax)));
  w.bytes = off;
  return w;
}

static int check_train(const ngl_model* m) {
  int rc = check_model(m, true);
  if (rc) return rc;
  if (m->feat_dtype != NGL_F32 || m->w_dtype != NGL_F32)
    NGL_FAIL(NGL_E_UNSUPPORTED, "training needs FP32 features and FP32 decoder weights");
  if (kBlock % m->hidden != 0) NGL_FAIL(NGL_E_UNSUPPORTED, "training needs hidden to divide %d", kBlock);
  if (m->feat_dim != 8 && m->feat_dim != 16 && m->feat_dim != 32 && m->feat_dim != 64)
    NGL_FAIL(NGL_E_UNSUPPORTED, "feat_dim %d not compiled", m->feat_dim);
  for (int l = 1; l <= m->num_lods; ++l)
    NGL_REQUIRE(m->ncorner[l - 1] == 0 || (m->corner_adj_off[l - 1] && (m->nvox[l + 1] == 0 || m->corner_adj[l - 1])),
                "corner adjacency of level %d is null (needed for training)", l);
  return NGL_OK;
}

template <int M, bool XYZ>
static int run_train(const ngl_model& md, const float* x, const float* target, const float* grad, int64_t P,
                     const float* lod_weight, float* loss, float* sdf_all, float* const* dfeat, float* const* dW1,
                     float* const* db1, float* const* dw2, float* db2, const TrainWS& w, hipStream_t s) {
  const int Lm = md.num_lods;
  const int D = Lm + 1;
  const unsigned pgrid = unsigned((P + kBlock - 1) / kBlock);
  // 1. sort by finest-cell Morton code (3D+1 key bits)
  k_keys<<<pgrid, kBlock, 0, s>>>(x, P, D, w.key[0], w.val[0]);
  const int bits = 3 * D + 1;
  const int sgrid = sort_grid(P);
  int cur = 0;
  for (int shift = 0; shift < bits; shift += 8) {
    k_radix_hist<<<sgrid, kBlock, 0, s>>>(w.key[cur], P, shift, w.hist);
    k_scan_inplace<<<1, 1024, 0, s>>>(w.hist, int64_t(256) * sgrid, nullptr);
    k_radix_scatter<<<sgrid, kBlock, 0, s>>>(w.key[cur], w.val[cur], w.key[cur ^ 1], w.val[cur ^ 1], P, shift,
                                                 w.hist);
    cur ^= 1;
  }
  const uint32_t* sidx = w.val[cur];
  // 2. per point
  PointArgs A{};
  A.xs = x;
  A.P = P;
  A.sidx = sidx;
  A.target = target;
  A.grad = grad;
  A.inv_p = 1.0f / float(P);
  for (int l = 0; l < NGL_MAX_LODS; ++l) A.lod_w[l] = lod_weight && l < Lm ? lod_weight[l] : 1.0f;
  A.sdf_all = sdf_all;
  A.zrows = w.zrows;
  A.drows = w.drows;
  A.gs = w.gs;
  A.vox_s = w.vox_s;
  A.loss_part = w.loss_part;
  if (P < kPointWaveMax) {
    // small batches: one wavefront per point
    const unsigned wgrid = unsigned((P + kBlock / 64 - 1) / (kBlock / 64));
    if (target) {
      k_point_wave<M, XYZ, true><<<wgrid, kBlock, 0, s>>>(md, A);
      if (loss) k_loss_reduce<<<1, kBlock, 0, s>>>(w.loss_part, int(P), 1.0f / float(P), loss);
    } else {
      k_point_wave<M, XYZ, false><<<wgrid, kBlock, 0, s>>>(md, A);
    }
  } else if (target) {
    k_point<M, XYZ, true><<<pgrid, kBlock, 0, s>>>(md, A);
    if (loss) k_loss_reduce<<<1, kBlock, 0, s>>>(w.loss_part, int(pgrid), 1.0f / float(P), loss);
  } else {
    k_point<M, XYZ, false><<<pgrid, kBlock, 0, s>>>(md, A);
  }
  // 3. decoder gradients
  DecArgs B{x, P, sidx, w.zrows, w.gs, w.dec_part, w.dec_b2};
  const int dgrid = dec_grid(P);
  k_dec_grad<M, XYZ><<<dim3(dgrid, Lm), kBlock, 0, s>>>(md, B);
  DecOut O{};
  for (int l = 0; l < Lm; ++l) {
    O.dW1[l] = dW1[l];
    O.db1[l] = db1[l];
    O.dw2[l] = dw2[l];
  }
  O.db2 = db2;
  const int din = M + (XYZ ? 3 : 0);
  const int H = md.hidden;
  const int waves = kBlock / 64;
  k_dec_reduce<<<dim3(unsigned((H * (din + 2) + 1 + waves - 1) / waves), Lm), kBlock, 0, s>>>(
      w.dec_part, w.dec_b2, H, din, kBlock / H, dgrid, O);
  // 4. feature gradients, level by level
  for (int l = 1; l <= Lm; ++l) {
    const int64_t nc = md.ncorner[l - 1];
    const int64_t nv = md.nvox[l + 1];
    if (nc == 0) continue;
    LevelArgs C{};
    C.xs = x;
    C.P = P;
    C.lvl = l;
    C.sidx = sidx;
    C.vox_s = w.vox_s + int64_t(l - 1) * P;
    C.drows = w.drows + int64_t(l - 1) * P * M;
    C.rec_cnt = w.rec_cnt;
    C.rec_total = w.rec_total;
    C.rec_key = w.rec_key;
    C.recs = w.recs;
    C.maxrec = w.maxrec;
    C.vpart = w.vpart;
    k_rec_count<<<unsigned(w.ntiles), 64, 0, s>>>(C);
    k_scan_inplace<<<1, 1024, 0, s>>>(w.rec_cnt, w.ntiles, w.rec_total);
    if (P < kPointWaveMax) k_rec_write<M, true><<<unsigned(w.ntiles), 64, 0, s>>>(md, C);
    else k_rec_write<M, false><<<unsigned(w.ntiles), 64, 0, s>>>(md, C);
    k_vox_reduce<M><<<unsigned(nv), 64, 0, s>>>(C, nv);
    k_corner<M><<<unsigned((nc * M + kBlock - 1) / kBlock), kBlock, 0, s>>>(md.corner_adj_off[l - 1],
                                                                            md.corner_adj[l - 1], w.vpart, nc,
                                                                            dfeat[l - 1]);
  }
  NGL_LAUNCHED();
  return NGL_OK;
}

static int zero_grads(const ngl_model& md, float* loss, float* const* dfeat, float* const* dW1, float* const* db1,
                      float* const* dw2, float* db2, hipStream_t s) {
  const int din = md.feat_dim + (md.with_xyz ? 3 : 0);
  auto z = [&](float* p, int64_t n) {
    if (p && n > 0) k_zero<<<unsigned((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(p, n);
  };
  z(loss, 1);
  z(db2, md.num_lods);
  for (int l = 0; l < md.num_lods; ++l) {
    z(dfeat[l], md.ncorner[l] * md.feat_dim);
    z(dW1[l], int64_t(md.hidden) * din);
    z(db1[l], md.hidden);
    z(dw2[l], md.hidden);
  }
  NGL_LAUNCHED();
  return NGL_OK;
}

static int train_entry(const ngl_model* m, const float* x, const float* target, const float* grad, int64_t P,
                       const float* lod_weight, float* loss, float* sdf_all, float* const* dfeat, float* const* dW1, float* const* db1,
                       float* const* dw2, float* db2, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_train(m);
  if (rc) return rc;
  NGL_REQUIRE(P >= 0 && P < (int64_t(1) << 31), "point count out of range");
  NGL_REQUIRE(dfeat && dW1 && db1 && dw2 && db2, "gradient buffers are null");
  for (int l = 0; l < m->num_lods; ++l)
    NGL_REQUIRE((dfeat[l] || m->ncorner[l] == 0) && dW1[l] && db1[l] && dw2[l], "gradient buffer of LOD %d is null",
                l + 1);
  hipStream_t s = (hipStream_t)stream;
  if (P == 0) return zero_grads(*m, loss, dfeat, dW1, db1, dw2, db2, s);
  NGL_REQUIRE(x != nullptr, "x is null");
  NGL_REQUIRE(target || grad, "target or upstream gradient is null");
  TrainWS w = carve(*m, P, ws);
  NGL_REQUIRE(ws != nullptr && ws_bytes >= w.bytes, "workspace too small: %zu < %zu bytes", ws_bytes, w.bytes);
  const ngl_model& md = *m;
#define NGL_TRAIN_CALL(M_, X_) \
  return run_train<M_, X_>(md, x, target, grad, P, lod_weight, loss, sdf_all, dfeat, dW1, db1, dw2, db2, w, s)
#define NGL_TRAIN_M(M_)          \
  if (md.with_xyz) NGL_TRAIN_CALL(M_, true); \
  else NGL_TRAIN_CALL(M_, false);
  switch (md.feat_dim) {
    case 8: NGL_TRAIN_M(8);
    case 16: NGL_TRAIN_M(16);
    case 32: NGL_TRAIN_M(32);
    default: NGL_TRAIN_M(64);
  }
#undef NGL_TRAIN_M
#undef NGL_TRAIN_CALL
}

}  // namespace ngl

extern "C" {

int ngl_train_workspace(const ngl_model* m, int64_t P, size_t* bytes) {
  int rc = ngl::check_train(m);
  if (rc) return rc;
  NGL_REQUIRE(bytes && P >= 0, "invalid workspace query");
  *bytes = ngl::carve(*m, P, nullptr).bytes;
  return NGL_OK;
}

int ngl_backward_all_lods(const ngl_model* m, const float* x, int64_t P, const float* grad_sdf, float* const* dfeat,
                          float* const* dW1, float* const* db1, float* const* dw2, float* db2, void* ws,
                          size_t ws_bytes, void* stream) {
  NGL_REQUIRE(P == 0 || grad_sdf != nullptr, "grad_sdf is null");
  return ngl::train_entry(m, x, nullptr, grad_sdf, P, nullptr, nullptr, nullptr, dfeat, dW1, db1, dw2, db2, ws,
                          ws_bytes, stream);
}

int ngl_train_fwd_bwd(const ngl_model* m, const float* x, const float* target, int64_t P, float* loss,
                      float* sdf_all, float* const* dfeat, float* const* dW1, float* const* db1, float* const* dw2,
                      float* db2, void* ws, size_t ws_bytes, void* stream) {
  NGL_REQUIRE(P == 0 || target != nullptr, "target is null");
  NGL_REQUIRE(loss != nullptr, "loss is null");
  return ngl::train_entry(m, x, target, nullptr, P, nullptr, loss, sdf_all, dfeat, dW1, db1, dw2, db2, ws, ws_bytes,
                          stream);
}

int ngl_train_fwd_bwd_lods(const ngl_model* m, const float* x, const float* target, int64_t P,
                           const float* lod_weight, float* loss, float* sdf_all, float* const* dfeat,
                           float* const* dW1, float* const* db1, float* const* dw2, float* db2, void* ws,
                           size_t ws_bytes, void* stream) {
  NGL_REQUIRE(P == 0 || target != nullptr, "target is null");
  NGL_REQUIRE(loss != nullptr && lod_weight != nullptr, "loss or lod_weight is null");
  NGL_REQUIRE(m != nullptr, "model is null");
  for (int l = 0; l < m->num_lods && l < NGL_MAX_LODS; ++l)
    NGL_REQUIRE(std::isfinite(lod_weight[l]) && lod_weight[l] >= 0.0f, "lod_weight[%d] must be finite and >= 0", l);
  return ngl::train_entry(m, x, target, nullptr, P, lod_weight, loss, sdf_all, dfeat, dW1, db1, dw2, db2, ws,
                          ws_bytes, stream);
}

}  // extern "C"
