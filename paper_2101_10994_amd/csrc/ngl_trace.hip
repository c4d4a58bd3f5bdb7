// Adaptive-stepping sphere tracing (Sec. 3.4, Fig. 3; stopping rules of
// App. A.4) on gfx950.  One lane per ray walks its front-to-back voxel list
// from the ray-octree intersection: outside the current voxel it jumps to
// the voxel's entry, inside it evaluates the SDF from that voxel and its
// ancestors and takes a sphere-tracing step.
#include "ngl_common.h"
#include "ngl_device.h"

namespace ngl {

// SDF at x from voxel `v` at depth Lp+1 and its ancestors (parents always
// exist).  Lp = lod, or lod+1 when blending with alpha > 0.
template <int M, typename FT, bool XYZ>
__device__ inline float sdf_in_voxel(const ngl_model& md, int v, int lod, float alpha, const float x[3]) {
  const bool blend = alpha > 0.0f;
  const int Lp = blend ? lod + 1 : lod;
  int vox[NGL_MAX_LODS];
  uint32_t cell[NGL_MAX_LODS];
#pragma unroll
  for (int l = NGL_MAX_LODS; l >= 1; --l) {
    if (l <= Lp) {
      vox[l - 1] = v;
      cell[l - 1] = md.cell[l + 1][v];
      v = md.parent[l + 1][v];
    }
  }
  float z[M];
#pragma unroll
  for (int k = 0; k < M; ++k) z[k] = 0.0f;
#pragma unroll
  for (int l = 1; l <= NGL_MAX_LODS; ++l)
    if (l <= lod) interp_level<M, FT>(md, l, vox[l - 1], cell_x(cell[l - 1]), cell_y(cell[l - 1]), cell_z(cell[l - 1]), x, z);
  float out = decode_f32<M, XYZ>(md, lod, x, z);
  if (blend) {
    const int vn = pick<NGL_MAX_LODS>(vox, lod);
    const uint32_t cn = uint32_t(pick<NGL_MAX_LODS>(reinterpret_cast<const int*>(cell), lod));
    interp_level<M, FT>(md, lod + 1, vn, cell_x(cn), cell_y(cn), cell_z(cn), x, z);
    out = (1.0f - alpha) * out + alpha * decode_f32<M, XYZ>(md, lod + 1, x, z);
  }
  return out;
}

template <int M, typename FT, bool XYZ, bool ANALYTIC>
__global__ __launch_bounds__(kBlock) void k_sphere_trace(ngl_model md, const float* __restrict__ o,
                                                         const float* __restrict__ d, int64_t R, int lod, float alpha,
                                                         const int32_t* __restrict__ pair_vox,
                                                         const float* __restrict__ t_in,
                                                         const float* __restrict__ t_out,
                                                         const int32_t* __restrict__ ray_off, ngl_trace_params prm,
                                                         float* __restrict__ t_hit, uint8_t* __restrict__ status,
                                                         int32_t* __restrict__ steps, int32_t* __restrict__ hit_vox) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= R) return;
  const float oo[3] = {o[i], o[R + i], o[2 * R + i]};
  const float dd[3] = {d[i], d[R + i], d[2 * R + i]};
  int p = ray_off[i];
  int e = ray_off[i + 1];
  bool bad = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) bad = bad || !__builtin_isfinite(oo[a]) || !__builtin_isfinite(dd[a]);
  float t = p < e ? t_in[p] : 0.0f;
  int k = 0;
  float prev = __builtin_inff();
  uint8_t st = NGL_RAY_MISS;
  int32_t hv = -1;
  if (bad) {
    st = NGL_RAY_INVALID;
  } else {
    for (;;) {
      while (p < e && t > t_out[p]) ++p;  // empty space: next voxel
      if (p == e) {
        st = NGL_RAY_MISS;
        break;
      }
      const float ti = t_in[p];
      if (t < ti) t = ti;  // outside the voxel: jump to its entry
      if (t > prm.t_far) {
        st = NGL_RAY_FAR;
        break;
      }
      if (k == prm.max_steps) {
        st = NGL_RAY_MAX_STEPS;
        break;
      }
      const float x[3] = {fmaf(t, dd[0], oo[0]), fmaf(t, dd[1], oo[1]), fmaf(t, dd[2], oo[2])};
      const int32_t v = pair_vox[p];
      if (!ANALYTIC && (v < 0 || int64_t(v) >= md.nvox[(alpha > 0.0f ? lod + 1 : lod) + 1])) {
        st = NGL_RAY_INVALID;  // hit list does not belong to this depth
        break;
      }
      float dist;
      if constexpr (ANALYTIC) {
        const float q0 = x[0] - prm.sphere[0], q1 = x[1] - prm.sphere[1], q2 = x[2] - prm.sphere[2];
        dist = sqrtf(q0 * q0 + q1 * q1 + q2 * q2) - prm.sphere[3];
      } else {
        dist = sdf_in_voxel<M, FT, XYZ>(md, v, lod, alpha, x);
      }
      ++k;
      if (dist < prm.delta) {
        st = NGL_RAY_HIT;
        hv = v;
        break;
      }
      if (prm.osc_check && fabsf(dist - prev) < 6.0f * prm.delta) {
        st = NGL_RAY_STALLED;
        break;
      }
      prev = dist;
      t += dist;
    }
  }
  t_hit[i] = t;
  status[i] = st;
  steps[i] = k;
  hit_vox[i] = hv;
}

template <int M, typename FT, bool XYZ>
struct TraceOp {
  static int run(const ngl_model& md, const float* o, const float* d, int64_t R, int lod, float alpha,
                 const int32_t* pv, const float* ti, const float* to, const int32_t* off, const ngl_trace_params& prm,
                 float* th, uint8_t* st, int32_t* steps, int32_t* hv, hipStream_t s) {
    const unsigned grid = unsigned((R + kBlock - 1) / kBlock);
    k_sphere_trace<M, FT, XYZ, false>
        <<<grid, kBlock, 0, s>>>(md, o, d, R, lod, alpha, pv, ti, to, off, prm, th, st, steps, hv);
    NGL_LAUNCHED();
    return NGL_OK;
  }
};

}  // namespace ngl

extern "C" {

int ngl_sphere_trace(const ngl_model* m, const float* o, const float* d, int64_t R, int32_t lod, float alpha,
                     const int32_t* pair_vox, const float* t_in, const float* t_out, const int32_t* ray_off,
                     const ngl_trace_params* params, float* t_hit, uint8_t* status, int32_t* steps,
                     int32_t* hit_vox, void* stream) {
  using namespace ngl;
  NGL_REQUIRE(params != nullptr, "params is null");
  const bool analytic = params->analytic != 0;
  int rc = check_model(m, !analytic);
  if (rc) return rc;
  NGL_REQUIRE(R >= 0 && R < (int64_t(1) << 31), "ray count out of range");
  NGL_REQUIRE(params->max_steps >= 0, "max_steps must be >= 0");
  NGL_REQUIRE(alpha >= 0.0f && alpha < 1.0f, "alpha must be in [0,1)");
  if (!analytic) {
    NGL_REQUIRE(lod >= 1 && lod <= m->num_lods, "lod %d outside 1..%d", lod, m->num_lods);
    NGL_REQUIRE(!(alpha > 0.0f) || lod < m->num_lods, "blending needs lod < num_lods");
  }
  if (R == 0) return NGL_OK;
  NGL_REQUIRE(o && d && ray_off && t_hit && status && steps && hit_vox, "null buffer");
  hipStream_t s = (hipStream_t)stream;
  if (analytic) {
    const unsigned grid = unsigned((R + kBlock - 1) / kBlock);
    k_sphere_trace<8, F32, true, true><<<grid, kBlock, 0, s>>>(*m, o, d, R, lod, alpha, pair_vox, t_in, t_out,
                                                                ray_off, *params, t_hit, status, steps, hit_vox);
    NGL_LAUNCHED();
    return NGL_OK;
  }
  if (m->w_dtype != NGL_F32) NGL_FAIL(NGL_E_UNSUPPORTED, "BF16 decoder weights are not supported by this call yet");
  const ngl_model& md = *m;
#define NGL_TRACE_ARGS md, o, d, R, int(lod), alpha, pair_vox, t_in, t_out, ray_off, *params, t_hit, status, steps, hit_vox, s
#define NGL_TRACE_XYZ(M_, FT_) \
  return md.with_xyz ? TraceOp<M_, FT_, true>::run(NGL_TRACE_ARGS) : TraceOp<M_, FT_, false>::run(NGL_TRACE_ARGS)
#define NGL_TRACE_FT(M_)                   \
  switch (md.feat_dtype) {                 \
    case NGL_F32: NGL_TRACE_XYZ(M_, F32);  \
    case NGL_F16: NGL_TRACE_XYZ(M_, F16);  \
    default: NGL_TRACE_XYZ(M_, BF16);      \
  }
  switch (md.feat_dim) {
    case 8: NGL_TRACE_FT(8);
    case 16: NGL_TRACE_FT(16);
    case 32: NGL_TRACE_FT(32);
    case 64: NGL_TRACE_FT(64);
    default: NGL_FAIL(NGL_E_UNSUPPORTED, "feat_dim %d not compiled (8, 16, 32, 64)", md.feat_dim);
  }
#undef NGL_TRACE_FT
#undef NGL_TRACE_XYZ
#undef NGL_TRACE_ARGS
}

}  // extern "C"
