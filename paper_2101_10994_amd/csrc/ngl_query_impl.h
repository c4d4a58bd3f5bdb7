// SDF query kernels (Sec. 3.2, Eq. 2; continuous LOD, Eq. 3), finite-
// difference normals (App. A.4) and their launchers, shared by the per-width
// translation units ngl_query_m{8,16,32,64}.hip and the entry points in
// ngl_query.hip.
#pragma once

#include "ngl_common.h"
#include "ngl_device.h"
#include "ngl_mfma.h"

namespace ngl {

// Locate x at feature levels 1..Lp: vox[l-1] (or -1) and the level's cell;
// *vlast = voxel of level Lp, *vnext = voxel of level `next` (both or -1).
template <int MAXL>
__device__ inline void locate(const ngl_model& md, const float x[3], int Lp, int* vox, int* cx, int* cy, int* cz,
                              int* vlast, int next = -1, int* vnext = nullptr) {
  const int Dp = Lp + 1;
  if (!in_box(x[0], x[1], x[2])) {
#pragma unroll
    for (int l = 0; l < MAXL; ++l) vox[l] = -1;
    *cx = *cy = *cz = 0;
    *vlast = -1;
    if (vnext) *vnext = -1;
    return;
  }
  const int r = 1 << Dp;
  *cx = cell_of(x[0], r);
  *cy = cell_of(x[1], r);
  *cz = cell_of(x[2], r);
  descend<MAXL>(md, *cx, *cy, *cz, Dp, vox, vlast, next, vnext);
}

template <int M, typename FT, bool XYZ>
__global__ __launch_bounds__(kBlock) void k_query(ngl_model md, const float* __restrict__ xs, int64_t P, int lod,
                                                  float alpha, const float* __restrict__ alpha_pp,
                                                  float* __restrict__ sdf, uint8_t* __restrict__ valid,
                                                  int32_t* __restrict__ vox_out) {
  const int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (p >= P) return;
  const float x[3] = {xs[p], xs[P + p], xs[2 * P + p]};
  const bool blend = alpha_pp != nullptr || alpha > 0.0f;
  const int Lp = blend ? lod + 1 : lod;
  const float a = alpha_pp ? alpha_pp[p] : alpha;
  int vox[NGL_MAX_LODS];
  int cx, cy, cz, vlast, vn;
  locate<NGL_MAX_LODS>(md, x, Lp, vox, &cx, &cy, &cz, &vlast, lod + 1, &vn);
  float z[M];
#pragma unroll
  for (int k = 0; k < M; ++k) z[k] = 0.0f;
  // Level loops are unrolled over the compile-time maximum so that the
  // per-level arrays stay in registers.
#pragma unroll
  for (int l = 1; l <= NGL_MAX_LODS; ++l)
    if (l <= lod && vox[l - 1] >= 0) interp_level<M, FT>(md, l, vox[l - 1], cx >> (Lp - l), cy >> (Lp - l), cz >> (Lp - l), x, z);
  float out = decode_f32<M, XYZ>(md, lod, x, z);
  if (blend) {
    // z_{L+1} = z_L + psi_{L+1}
    if (vn >= 0) interp_level<M, FT>(md, lod + 1, vn, cx, cy, cz, x, z);
    out = (1.0f - a) * out + a * decode_f32<M, XYZ>(md, lod + 1, x, z);
  }
  sdf[p] = out;
  if (valid) valid[p] = vlast >= 0 ? 1 : 0;
  if (vox_out) {
#pragma unroll
    for (int l = 1; l <= NGL_MAX_LODS; ++l)
      if (l <= Lp) vox_out[int64_t(l - 1) * P + p] = vox[l - 1];
  }
}

// All discrete LODs: the level sum is shared, one decoder per LOD.
template <int M, typename FT, bool XYZ>
__global__ __launch_bounds__(kBlock) void k_query_all(ngl_model md, const float* __restrict__ xs, int64_t P,
                                                      float* __restrict__ sdf_all) {
  const int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (p >= P) return;
  const float x[3] = {xs[p], xs[P + p], xs[2 * P + p]};
  const int Lm = md.num_lods;
  int vox[NGL_MAX_LODS];
  int cx, cy, cz, vlast;
  locate<NGL_MAX_LODS>(md, x, Lm, vox, &cx, &cy, &cz, &vlast);
  float z[M];
#pragma unroll
  for (int k = 0; k < M; ++k) z[k] = 0.0f;
#pragma unroll
  for (int l = 1; l <= NGL_MAX_LODS; ++l) {
    if (l <= Lm) {
      const int s = Lm - l;
      if (vox[l - 1] >= 0) interp_level<M, FT>(md, l, vox[l - 1], cx >> s, cy >> s, cz >> s, x, z);
      sdf_all[int64_t(l - 1) * P + p] = decode_f32<M, XYZ>(md, l, x, z);
    }
  }
}

// Matrix-core decoder (BF16 or FP32 form): the same location and gather per
// lane, then the first decoder layer for the wavefront's 64 points on the
// matrix cores.  Grid-stride over points so each block stages the decoder
// fragments in LDS once; inside the loop only wavefront-level LDS ordering
// is needed.
template <int M, typename FT, bool XYZ, int NW, class DEC>
__global__ __launch_bounds__(64 * NW) void k_query_mfma(ngl_model md, const float* __restrict__ xs, int64_t P,
                                                        int lod, float alpha, const float* __restrict__ alpha_pp,
                                                        float* __restrict__ sdf, uint8_t* __restrict__ valid,
                                                        int32_t* __restrict__ vox_out) {
  extern __shared__ __align__(16) char smem[];
  const int H = md.hidden;
  const bool blend = alpha_pp != nullptr || alpha > 0.0f;
  DecLds<DEC> S(smem, H, blend);
  DEC::load(md, lod, S.frag0, S.w2s0);
  if (blend) DEC::load(md, lod + 1, S.frag1, S.w2s1);
  __syncthreads();
  const float b2a = md.b2[lod - 1];
  const float b2b = blend ? md.b2[lod] : 0.0f;
  const int Lp = blend ? lod + 1 : lod;
  for (int64_t base = int64_t(blockIdx.x) * (64 * NW); base < P; base += int64_t(gridDim.x) * (64 * NW)) {
    const int64_t p = base + threadIdx.x;
    const bool act = p < P;
    float x[3] = {0.0f, 0.0f, 0.0f};
    if (act) {
      x[0] = xs[p];
      x[1] = xs[P + p];
      x[2] = xs[2 * P + p];
    }
    int vox[NGL_MAX_LODS];
    int cx, cy, cz, vlast, vn;
    locate<NGL_MAX_LODS>(md, x, Lp, vox, &cx, &cy, &cz, &vlast, lod + 1, &vn);
    if (!act) {
#pragma unroll
      for (int l = 0; l < NGL_MAX_LODS; ++l) vox[l] = -1;
      vlast = vn = -1;
    }
    float z[M];
#pragma unroll
    for (int k = 0; k < M; ++k) z[k] = 0.0f;
#pragma unroll
    for (int l = 1; l <= NGL_MAX_LODS; ++l)
      if (l <= lod && vox[l - 1] >= 0)
        interp_level<M, FT>(md, l, vox[l - 1], cx >> (Lp - l), cy >> (Lp - l), cz >> (Lp - l), x, z);
    DEC::stage(S.stage, x, z);
    wave_lds_sync();
    float out = DEC::decode(S.frag0, S.w2s0, b2a, S.stage, H, __ballot(act));
    if (blend) {
      if (vn >= 0) interp_level<M, FT>(md, lod + 1, vn, cx, cy, cz, x, z);
      wave_lds_sync();
      DEC::stage(S.stage, x, z);
      wave_lds_sync();
      const float a = act ? (alpha_pp ? alpha_pp[p] : alpha) : 0.0f;
      out = (1.0f - a) * out + a * DEC::decode(S.frag1, S.w2s1, b2b, S.stage, H, __ballot(act));
    }
    wave_lds_sync();
    if (act) {
      sdf[p] = out;
      if (valid) valid[p] = vlast >= 0 ? 1 : 0;
      if (vox_out) {
#pragma unroll
        for (int l = 1; l <= NGL_MAX_LODS; ++l)
          if (l <= Lp) vox_out[int64_t(l - 1) * P + p] = vox[l - 1];
      }
    }
  }
}

// Cooperative gather: lanes locate their own points as above, then the
// wavefront gathers and decodes its 64 points one 16-point tile at a time
// (TileShape): the 4 lanes of group r serve point r of the tile, lane g
// loading the elements [g M/4, g M/4 + M/4) of every corner row, so a row
// (32 to 256 bytes) is read by 4 lanes together where one lane per point
// reads whole rows alone.  Every element is accumulated in the same order
// as interp_level and the staged decoder rows hold the same values, so the
// results are those of k_query_mfma bit for bit.  Only one tile's
// accumulators and staging rows are live at a time.
// One evaluation of the wavefront's located points: features of levels
// 1..lod, the decoder lod, and with `blend` the Eq. 3 mix (weight a, this
// lane's) with decoder lod+1 on z + the level lod+1 voxel vn.  rows: this
// wavefront's 16 staging rows.  Every lane must call it.
template <int M, typename FT, class DEC>
__device__ __forceinline__ float coop_eval(const ngl_model& md, const DecLds<DEC>& S, const float x[3],
                                           const int* vox, int cx, int cy, int cz, int vn, bool act, int lod, int Lp,
                                           bool blend, float a, float b2a, float b2b, const void* l1s = nullptr,
                                           bool l1 = false) {
  const uint64_t live = __ballot(act);  // tiles without an active point are skipped
  constexpr int D = TileShape<M>::D;
  const int lane = threadIdx.x & 63, r = lane >> 2, g = lane & 3;
  const int H = md.hidden;
  typename DEC::Stage* rows = S.stage;
  float mine = 0.0f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (((live >> (16 * t)) & 0xffffull) == 0) continue;
    const int q = 16 * t + r;  // the group's point
    float xq[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) xq[k] = __shfl(x[k], q, 64);
    const int qx = __shfl(cx, q, 64), qy = __shfl(cy, q, 64), qz = __shfl(cz, q, 64);
    float acc[D];
#pragma unroll
    for (int i = 0; i < D; ++i) acc[i] = 0.0f;
#pragma unroll
    for (int l = 1; l <= NGL_MAX_LODS; ++l)
      if (l <= lod && md.nvox[l + 1] > 0) {
        const int sh = Lp - l;
        tile_level<M, FT>(md, l, __shfl(act ? vox[l - 1] : -1, q, 64), xq, qx >> sh, qy >> sh, qz >> sh, g, acc,
                          l1s, l1);
      }
    DEC::template tile_slice<D>(rows, r, g * D, acc);
    if (g == 0) DEC::tile_rest(rows, r, xq);
    wave_lds_sync();
    const float p0 = DEC::tile(S.frag0, S.w2s0, rows, H);
    float out = b2a + p0;
    if (blend) {
      // z_{L+1} = z_L + psi_{L+1}
      wave_lds_sync();
      if (md.nvox[lod + 2] > 0) tile_level<M, FT>(md, lod + 1, __shfl(act ? vn : -1, q, 64), xq, qx, qy, qz, g, acc);
      DEC::template tile_slice<D>(rows, r, g * D, acc);
      wave_lds_sync();
      const float p1 = DEC::tile(S.frag1, S.w2s1, rows, H);
      out = (1.0f - a) * out + a * (b2b + p1);
    }
    wave_lds_sync();
    if ((lane >> 4) == t) mine = out;  // lane 16 t + j owns point 16 t + j
  }
  return mine;
}

template <int M, typename FT, bool XYZ, int NW, class DEC>
__global__ __launch_bounds__(64 * NW) void k_query_coop(ngl_model md, const float* __restrict__ xs, int64_t P,
                                                        int lod, float alpha, const float* __restrict__ alpha_pp,
                                                        float* __restrict__ sdf, uint8_t* __restrict__ valid,
                                                        int32_t* __restrict__ vox_out, bool l1) {
  extern __shared__ __align__(16) char smem[];
  const int H = md.hidden;
  const bool blend = alpha_pp != nullptr || alpha > 0.0f;
  DecLds<DEC> S(smem, H, blend, DEC::TILE_ELEMS);
  // level 1's table after the staging rows (when the launch reserved it)
  char* l1s = smem + DecLds<DEC>::fixed_bytes(H, blend) + NW * size_t(DEC::TILE_BYTES);
  DEC::load(md, lod, S.frag0, S.w2s0);
  if (blend) DEC::load(md, lod + 1, S.frag1, S.w2s1);
  if (l1) stage_l1<M, FT>(md, l1s);
  __syncthreads();
  const float b2a = md.b2[lod - 1];
  const float b2b = blend ? md.b2[lod] : 0.0f;
  const int Lp = blend ? lod + 1 : lod;
  for (int64_t base = int64_t(blockIdx.x) * (64 * NW); base < P; base += int64_t(gridDim.x) * (64 * NW)) {
    const int64_t p = base + threadIdx.x;
    const bool act = p < P;
    float x[3] = {0.0f, 0.0f, 0.0f};
    if (act) {
      x[0] = xs[p];
      x[1] = xs[P + p];
      x[2] = xs[2 * P + p];
    }
    int vox[NGL_MAX_LODS];
    int cx, cy, cz, vlast, vn;
    locate<NGL_MAX_LODS>(md, x, Lp, vox, &cx, &cy, &cz, &vlast, lod + 1, &vn);
    if (!act) {
#pragma unroll
      for (int l = 0; l < NGL_MAX_LODS; ++l) vox[l] = -1;
      vlast = vn = -1;
    }
    const float a = act ? (alpha_pp ? alpha_pp[p] : alpha) : 0.0f;
    const float out = coop_eval<M, FT, DEC>(md, S, x, vox, cx, cy, cz, vn, act, lod, Lp, blend, a, b2a, b2b, l1s,
                                            l1);
    if (act) {
      sdf[p] = out;
      if (valid) valid[p] = vlast >= 0 ? 1 : 0;
      if (vox_out) {
#pragma unroll
        for (int l = 1; l <= NGL_MAX_LODS; ++l)
          if (l <= Lp) vox_out[int64_t(l - 1) * P + p] = vox[l - 1];
      }
    }
  }
}

template <int M, typename FT, bool XYZ, int NW, class DEC>
static int launch_query_coop_nw(const ngl_model& md, const float* x, int64_t P, int lod, float alpha,
                                const float* app, float* sdf, uint8_t* valid, int32_t* vox, hipStream_t s,
                                size_t lds) {
  // Grid-stride over the points with one round of resident blocks (each
  // stages the decoder once), or at most NGL_OPT_QUERY_BLOCKS_PER_CU per CU.
  const void* kern = reinterpret_cast<const void*>(&k_query_coop<M, FT, XYZ, NW, DEC>);
  const int bpc = option(NGL_OPT_QUERY_BLOCKS_PER_CU);
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  // level 1's rows in LDS when the table fits beside the decoder
  const bool l1 = l1_bytes<M, FT>() > 0 && l1_fits(md) && lds + l1_bytes<M, FT>() <= 65536;
  if (l1) lds += l1_bytes<M, FT>();
  int64_t grid = (P + 64 * NW - 1) / (64 * NW);
  const int64_t cap = bpc > 0 ? int64_t(cus) * bpc : resident_grid(kern, 64 * NW, lds, 0);
  if (grid > cap) grid = cap;
  k_query_coop<M, FT, XYZ, NW, DEC><<<unsigned(grid), 64 * NW, lds, s>>>(md, x, P, lod, alpha, app, sdf, valid, vox,
                                                                          l1);
  NGL_LAUNCHED();
  return NGL_OK;
}

template <int M, typename FT, bool XYZ, class DEC>
static int launch_query_coop(const ngl_model& md, const float* x, int64_t P, int lod, float alpha, const float* app,
                             float* sdf, uint8_t* valid, int32_t* vox, hipStream_t s) {
  const bool blend = app != nullptr || alpha > 0.0f;
  const size_t fixed = DecLds<DEC>::fixed_bytes(md.hidden, blend);
  constexpr size_t R = DEC::TILE_BYTES;
  if (fixed + 4 * R <= 65536)
    return launch_query_coop_nw<M, FT, XYZ, 4, DEC>(md, x, P, lod, alpha, app, sdf, valid, vox, s, fixed + 4 * R);
  if (fixed + 2 * R <= 65536)
    return launch_query_coop_nw<M, FT, XYZ, 2, DEC>(md, x, P, lod, alpha, app, sdf, valid, vox, s, fixed + 2 * R);
  return launch_query_coop_nw<M, FT, XYZ, 1, DEC>(md, x, P, lod, alpha, app, sdf, valid, vox, s, fixed + R);
}

template <int M, typename FT, bool XYZ, int NW, class DEC>
static int launch_query_mfma_nw(const ngl_model& md, const float* x, int64_t P, int lod, float alpha,
                                const float* app, float* sdf, uint8_t* valid, int32_t* vox, hipStream_t s,
                                size_t lds) {
  int64_t grid = (P + 64 * NW - 1) / (64 * NW);
  if (grid > 4096) grid = 4096;
  k_query_mfma<M, FT, XYZ, NW, DEC><<<unsigned(grid), 64 * NW, lds, s>>>(md, x, P, lod, alpha, app, sdf, valid, vox);
  NGL_LAUNCHED();
  return NGL_OK;
}

template <int M, typename FT, bool XYZ, class DEC>
static int launch_query_mfma(const ngl_model& md, const float* x, int64_t P, int lod, float alpha, const float* app,
                             float* sdf, uint8_t* valid, int32_t* vox, hipStream_t s) {
  if (option(NGL_OPT_COOP_GATHER) == 1)
    return launch_query_coop<M, FT, XYZ, DEC>(md, x, P, lod, alpha, app, sdf, valid, vox, s);
  const bool blend = app != nullptr || alpha > 0.0f;
  const size_t fixed = DecLds<DEC>::fixed_bytes(md.hidden, blend);
  if (fixed + 4 * DEC::STAGE_BYTES <= 65536)
    return launch_query_mfma_nw<M, FT, XYZ, 4, DEC>(md, x, P, lod, alpha, app, sdf, valid, vox, s,
                                                    fixed + 4 * DEC::STAGE_BYTES);
  if (fixed + 2 * DEC::STAGE_BYTES <= 65536)
    return launch_query_mfma_nw<M, FT, XYZ, 2, DEC>(md, x, P, lod, alpha, app, sdf, valid, vox, s,
                                                    fixed + 2 * DEC::STAGE_BYTES);
  return launch_query_mfma_nw<M, FT, XYZ, 1, DEC>(md, x, P, lod, alpha, app, sdf, valid, vox, s,
                                                  fixed + DEC::STAGE_BYTES);
}

// Central-difference normals: six queries per point.  MFMA selects the
// matrix-core decoder (every lane joins each of the six decodes).
struct NormalArgs {
  const float* x;       // points [3][P], or null with rays below
  const float* o;
  const float* d;
  const float* t_hit;
  const uint8_t* status;
  int64_t P;
  int lod;
  float alpha;
  float h;
  float* normals;       // [3][P]
  bool l1;              // level 1's table staged in LDS (k_normals_coop)
};

template <int M, typename FT, bool XYZ>
__device__ inline void query_z(const ngl_model& md, const float x[3], int lod, bool blend, float* z, float* zn) {
  const int Lp = blend ? lod + 1 : lod;
  int vox[NGL_MAX_LODS];
  int cx, cy, cz, vlast, vn;
  locate<NGL_MAX_LODS>(md, x, Lp, vox, &cx, &cy, &cz, &vlast, lod + 1, &vn);
#pragma unroll
  for (int k = 0; k < M; ++k) z[k] = 0.0f;
#pragma unroll
  for (int l = 1; l <= NGL_MAX_LODS; ++l)
    if (l <= lod && vox[l - 1] >= 0)
      interp_level<M, FT>(md, l, vox[l - 1], cx >> (Lp - l), cy >> (Lp - l), cz >> (Lp - l), x, z);
  if (blend) {
#pragma unroll
    for (int k = 0; k < M; ++k) zn[k] = z[k];
    if (vn >= 0) interp_level<M, FT>(md, lod + 1, vn, cx, cy, cz, x, zn);
  }
}

template <int M, typename FT, bool XYZ, int NW, class DEC, bool MFMA>
__global__ __launch_bounds__(64 * NW) void k_normals(ngl_model md, NormalArgs A) {
  extern __shared__ __align__(16) char smem[];
  const int H = md.hidden;
  const bool blend = A.alpha > 0.0f;
  DecLds<DEC> S(smem, H, blend && MFMA);
  if constexpr (MFMA) {
    DEC::load(md, A.lod, S.frag0, S.w2s0);
    if (blend) DEC::load(md, A.lod + 1, S.frag1, S.w2s1);
    __syncthreads();
  }
  const float b2a = md.b2[A.lod - 1];
  const float b2b = blend ? md.b2[A.lod] : 0.0f;
  const int64_t P = A.P;
  for (int64_t base = int64_t(blockIdx.x) * (64 * NW); base < P; base += int64_t(gridDim.x) * (64 * NW)) {
    const int64_t p = base + threadIdx.x;
    bool act = p < P;
    float x0[3] = {0.0f, 0.0f, 0.0f};
    if (act) {
      if (A.status) {
        act = A.status[p] == NGL_RAY_HIT;
        const float t = A.t_hit[p];
#pragma unroll
        for (int a = 0; a < 3; ++a) x0[a] = fmaf(t, A.d[a * P + p], A.o[a * P + p]);
      } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) x0[a] = A.x[a * P + p];
      }
    }
    float g[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int a = e >> 1;
      const float sgn = (e & 1) ? -1.0f : 1.0f;
      float x[3] = {x0[0], x0[1], x0[2]};
      x[a] = x0[a] + sgn * A.h;
      float f;
      float z[M], zn[M];
      if (act) {
        query_z<M, FT, XYZ>(md, x, A.lod, blend, z, zn);
      } else {
#pragma unroll
        for (int k = 0; k < M; ++k) z[k] = zn[k] = 0.0f;
      }
      if constexpr (MFMA) {
        DEC::stage(S.stage, x, z);
        wave_lds_sync();
        f = DEC::decode(S.frag0, S.w2s0, b2a, S.stage, H, __ballot(act));
        if (blend) {
          wave_lds_sync();
          DEC::stage(S.stage, x, zn);
          wave_lds_sync();
          f = (1.0f - A.alpha) * f + A.alpha * DEC::decode(S.frag1, S.w2s1, b2b, S.stage, H, __ballot(act));
        }
        wave_lds_sync();
      } else {
        f = 0.0f;
        if (act) {
          f = decode_f32<M, XYZ>(md, A.lod, x, z);
          if (blend) f = (1.0f - A.alpha) * f + A.alpha * decode_f32<M, XYZ>(md, A.lod + 1, x, zn);
        }
      }
      g[a] += sgn * f;
    }
    if (p < P) {
      float n[3] = {0.0f, 0.0f, 0.0f};
      if (act) {
        const float inv2h = 0.5f / A.h;
        const float gx = g[0] * inv2h, gy = g[1] * inv2h, gz = g[2] * inv2h;
        const float len = sqrtf(gx * gx + gy * gy + gz * gz);
        if (len > 0.0f) {
          n[0] = gx / len;
          n[1] = gy / len;
          n[2] = gz / len;
        }
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) A.normals[a * P + p] = n[a];
    }
  }
}

// Matrix-core form: each block walks a contiguous range of the points and
// queues the active ones (rays that hit, or every point) in LDS, so its
// wavefronts only evaluate active points (a frame's misses get their zero
// normal on the way).  Each of the six probes is one cooperative,
// tile-wise evaluation (coop_eval), whose results are the bits of the
// one-lane-per-point form.
template <int M, typename FT, bool XYZ, int NW, class DEC>
__global__ __launch_bounds__(64 * NW) void k_normals_coop(ngl_model md, NormalArgs A) {
  constexpr int NB = 64 * NW;  // points evaluated per block pass
  extern __shared__ __align__(16) char smem[];
  __shared__ int32_t queue[2 * NB];
  __shared__ int qn;
  const int H = md.hidden;
  const int lod = A.lod;
  const bool blend = A.alpha > 0.0f;
  const int Lp = blend ? lod + 1 : lod;
  DecLds<DEC> S(smem, H, blend, DEC::TILE_ELEMS);
  char* l1s = smem + DecLds<DEC>::fixed_bytes(H, blend) + NW * size_t(DEC::TILE_BYTES);
  DEC::load(md, lod, S.frag0, S.w2s0);
  if (blend) DEC::load(md, lod + 1, S.frag1, S.w2s1);
  if (A.l1) stage_l1<M, FT>(md, l1s);
  if (threadIdx.x == 0) qn = 0;
  __syncthreads();
  const float b2a = md.b2[lod - 1];
  const float b2b = blend ? md.b2[lod] : 0.0f;
  const int64_t P = A.P;
  int64_t chunk = (P + gridDim.x - 1) / gridDim.x;
  chunk = (chunk + NB - 1) / NB * NB;
  const int64_t begin = int64_t(blockIdx.x) * chunk;
  const int64_t end = begin + chunk < P ? begin + chunk : P;
  int64_t pos = begin;
  for (;;) {
    // 1. queue active points until a full pass is available or the range ends
    while (qn < NB && pos < end) {
      const int64_t p = pos + threadIdx.x;
      bool act = false;
      if (p < end) {
        act = A.status ? A.status[p] == NGL_RAY_HIT : true;
        if (!act) {
#pragma unroll
          for (int a = 0; a < 3; ++a) A.normals[a * P + p] = 0.0f;
        }
      }
      const uint64_t m = __ballot(act);
      int base = 0;
      if ((threadIdx.x & 63) == 0 && m) base = atomicAdd(&qn, __popcll(m));
      base = __shfl(base, 0, 64);
      if (act) queue[base + __popcll(m & ((1ull << (threadIdx.x & 63)) - 1ull))] = int32_t(p);
      pos += NB;
      __syncthreads();
    }
    const int n = qn;
    if (n == 0) break;
    const int take = n < NB ? n : NB;
    // 2. evaluate the six probes of up to NB queued points
    const bool act = int(threadIdx.x) < take;
    const int64_t p = act ? queue[threadIdx.x] : 0;
    float x0[3] = {0.0f, 0.0f, 0.0f};
    if (act) {
      if (A.status) {
        const float t = A.t_hit[p];
#pragma unroll
        for (int a = 0; a < 3; ++a) x0[a] = fmaf(t, A.d[a * P + p], A.o[a * P + p]);
      } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) x0[a] = A.x[a * P + p];
      }
    }
    float g[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int a = e >> 1;
      const float sgn = (e & 1) ? -1.0f : 1.0f;
      float x[3] = {x0[0], x0[1], x0[2]};
      x[a] = x0[a] + sgn * A.h;
      int vox[NGL_MAX_LODS];
      int cx, cy, cz, vlast, vn;
      locate<NGL_MAX_LODS>(md, x, Lp, vox, &cx, &cy, &cz, &vlast, lod + 1, &vn);
      if (!act) {
#pragma unroll
        for (int l = 0; l < NGL_MAX_LODS; ++l) vox[l] = -1;
        vn = -1;
      }
      const float f = coop_eval<M, FT, DEC>(md, S, x, vox, cx, cy, cz, vn, act, lod, Lp, blend, A.alpha, b2a, b2b,
                                            l1s, A.l1);
      g[a] += sgn * f;
    }
    if (act) {
      float nrm[3] = {0.0f, 0.0f, 0.0f};
      const float inv2h = 0.5f / A.h;
      const float gx = g[0] * inv2h, gy = g[1] * inv2h, gz = g[2] * inv2h;
      const float len = sqrtf(gx * gx + gy * gy + gz * gz);
      if (len > 0.0f) {
        nrm[0] = gx / len;
        nrm[1] = gy / len;
        nrm[2] = gz / len;
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) A.normals[a * P + p] = nrm[a];
    }
    // 3. drop the evaluated points from the queue
    __syncthreads();
    const int rest = n - take;
    for (int i = threadIdx.x; i < rest; i += NB) queue[i] = queue[take + i];
    __syncthreads();
    if (threadIdx.x == 0) qn = rest;
    __syncthreads();
  }
}

template <int M, typename FT, bool XYZ, class DEC, bool MFMA, int NW>
static int launch_normals_nw(const ngl_model& md, const NormalArgs& A, hipStream_t s, size_t lds) {
  // one round of resident blocks looping over the points (each stages the
  // decoders once)
  const void* kern = reinterpret_cast<const void*>(&k_normals<M, FT, XYZ, NW, DEC, MFMA>);
  int64_t grid = (A.P + 64 * NW - 1) / (64 * NW);
  const int64_t cap = resident_grid(kern, 64 * NW, lds, 0);
  if (grid > cap) grid = cap;
  k_normals<M, FT, XYZ, NW, DEC, MFMA><<<unsigned(grid), 64 * NW, lds, s>>>(md, A);
  NGL_LAUNCHED();
  return NGL_OK;
}

template <int M, typename FT, bool XYZ, class DEC, bool MFMA>
static int launch_normals(const ngl_model& md, const NormalArgs& A, hipStream_t s) {
  const bool blend = A.alpha > 0.0f;
  if constexpr (!MFMA) {
    return launch_normals_nw<M, FT, XYZ, DEC, false, 2>(md, A, s, 0);
  } else {
    if (option(NGL_OPT_COOP_GATHER) == 0) {
      // one lane per point and probe (same results as the cooperative form)
      const size_t fixed = DecLds<DEC>::fixed_bytes(md.hidden, blend);
      if (fixed + 4 * DEC::STAGE_BYTES <= 65536)
        return launch_normals_nw<M, FT, XYZ, DEC, true, 4>(md, A, s, fixed + 4 * DEC::STAGE_BYTES);
      if (fixed + 2 * DEC::STAGE_BYTES <= 65536)
        return launch_normals_nw<M, FT, XYZ, DEC, true, 2>(md, A, s, fixed + 2 * DEC::STAGE_BYTES);
      return launch_normals_nw<M, FT, XYZ, DEC, true, 1>(md, A, s, fixed + DEC::STAGE_BYTES);
    }
    constexpr int NW = 4;
    size_t lds = DecLds<DEC>::fixed_bytes(md.hidden, blend) + NW * size_t(DEC::TILE_BYTES);
    NormalArgs B = A;
    B.l1 = l1_bytes<M, FT>() > 0 && l1_fits(md) && lds + l1_bytes<M, FT>() <= 65536;
    if (B.l1) lds += l1_bytes<M, FT>();
    const void* kern = reinterpret_cast<const void*>(&k_normals_coop<M, FT, XYZ, NW, DEC>);
    int64_t grid = (A.P + 64 * NW - 1) / (64 * NW);
    const int64_t cap = resident_grid(kern, 64 * NW, lds, 0);
    if (grid > cap) grid = cap;
    k_normals_coop<M, FT, XYZ, NW, DEC><<<unsigned(grid), 64 * NW, lds, s>>>(md, B);
    NGL_LAUNCHED();
    return NGL_OK;
  }
}

template <int M, typename FT, bool XYZ>
struct NormalOp {
  static int run(const ngl_model& md, const NormalArgs& A, hipStream_t s) {
    if (md.w_dtype == NGL_BF16) return launch_normals<M, FT, XYZ, DecBF16<M, XYZ>, true>(md, A, s);
    if (option(NGL_OPT_F32_DECODER) == 1) return launch_normals<M, FT, XYZ, DecF32<M, XYZ>, true>(md, A, s);
    return launch_normals<M, FT, XYZ, DecF32<M, XYZ>, false>(md, A, s);
  }
};

template <int M, typename FT, bool XYZ>
static int launch_query(const ngl_model& md, const float* x, int64_t P, int lod, float alpha, const float* app,
                        float* sdf, uint8_t* valid, int32_t* vox, hipStream_t s) {
  const unsigned grid = unsigned((P + kBlock - 1) / kBlock);
  k_query<M, FT, XYZ><<<grid, kBlock, 0, s>>>(md, x, P, lod, alpha, app, sdf, valid, vox);
  NGL_LAUNCHED();
  return NGL_OK;
}

template <int M, typename FT, bool XYZ>
static int launch_query_all(const ngl_model& md, const float* x, int64_t P, float* out, hipStream_t s) {
  const unsigned grid = unsigned((P + kBlock - 1) / kBlock);
  k_query_all<M, FT, XYZ><<<grid, kBlock, 0, s>>>(md, x, P, out);
  NGL_LAUNCHED();
  return NGL_OK;
}

template <int M, typename FT, bool XYZ>
struct QueryOp {
  static int run(const ngl_model& md, const float* x, int64_t P, int lod, float alpha, const float* app, float* sdf,
                 uint8_t* valid, int32_t* vox, hipStream_t s) {
    if (md.w_dtype == NGL_BF16)
      return launch_query_mfma<M, FT, XYZ, DecBF16<M, XYZ>>(md, x, P, lod, alpha, app, sdf, valid, vox, s);
    if (option(NGL_OPT_F32_DECODER) == 1)
      return launch_query_mfma<M, FT, XYZ, DecF32<M, XYZ>>(md, x, P, lod, alpha, app, sdf, valid, vox, s);
    return launch_query<M, FT, XYZ>(md, x, P, lod, alpha, app, sdf, valid, vox, s);
  }
};

template <int M, typename FT, bool XYZ>
struct QueryAllOp {
  static int run(const ngl_model& md, const float* x, int64_t P, float* out, hipStream_t s) {
    return launch_query_all<M, FT, XYZ>(md, x, P, out, s);
  }
};

// Per-width runners, defined in ngl_query_m<width>.hip.
#define NGL_QUERY_DECLARE(M_)                                                                       \
  int query_run_m##M_(const ngl_model& md, const float* x, int64_t P, int lod, float alpha,         \
                      const float* app, float* sdf, uint8_t* valid, int32_t* vox, hipStream_t s);   \
  int query_all_run_m##M_(const ngl_model& md, const float* x, int64_t P, float* out, hipStream_t s); \
  int normals_run_m##M_(const ngl_model& md, const NormalArgs& A, hipStream_t s);
NGL_QUERY_DECLARE(8)
NGL_QUERY_DECLARE(16)
NGL_QUERY_DECLARE(32)
NGL_QUERY_DECLARE(64)
#undef NGL_QUERY_DECLARE

#define NGL_QUERY_DEFINE(M_)                                                                        \
  int query_run_m##M_(const ngl_model& md, const float* x, int64_t P, int lod, float alpha,         \
                      const float* app, float* sdf, uint8_t* valid, int32_t* vox, hipStream_t s) {  \
    return dispatch_ft<QueryOp, M_>(md, x, P, lod, alpha, app, sdf, valid, vox, s);                 \
  }                                                                                                 \
  int query_all_run_m##M_(const ngl_model& md, const float* x, int64_t P, float* out, hipStream_t s) { \
    return dispatch_ft<QueryAllOp, M_>(md, x, P, out, s);                                           \
  }                                                                                                 \
  int normals_run_m##M_(const ngl_model& md, const NormalArgs& A, hipStream_t s) {                  \
    return dispatch_ft<NormalOp, M_>(md, A, s);                                                     \
  }

}  // namespace ngl
