// Adaptive-stepping sphere tracing (Sec. 3.4, Fig. 3; stopping rules of
// App. A.4) on gfx950.  Each ray walks its front-to-back voxel list from the
// ray-octree intersection: outside the current voxel it jumps to the voxel's
// entry, inside it evaluates the SDF from that voxel and its ancestors and
// takes a sphere-tracing step.
#include "ngl_common.h"
#include "ngl_device.h"
#include "ngl_mfma.h"

namespace ngl {

struct TraceArgs {
  const float* o;
  const float* d;
  int64_t R;
  int lod;
  float alpha;
  const int32_t* pair_vox;
  const float* t_in;
  const float* t_out;
  const int32_t* ray_off;
  ngl_trace_params prm;
  float* t_hit;
  uint8_t* status;
  int32_t* steps;
  int32_t* hit_vox;
  unsigned int* counter;  // work queue head (zeroed before the launch)
};

// Persistent sphere tracer.  Each wavefront keeps one ray per lane; a lane
// whose ray terminates takes the next ray from a global queue, so every step
// is evaluated on a compacted set of active rays.  Every ray ends after at
// most max_steps evaluations and one pass over its pairs, and the queue is
// finite, so every wavefront reaches the exit.
template <int M, typename FT, bool XYZ, bool ANALYTIC, bool MFMA, int NW>
__global__ __launch_bounds__(64 * NW) void k_sphere_trace(ngl_model md, TraceArgs A) {
  using S = MfmaShape<M, XYZ>;
  extern __shared__ __align__(16) char smem[];
  const int lane = threadIdx.x & 63;
  const int64_t R = A.R;
  const bool blend = A.alpha > 0.0f;
  const int lod = A.lod;
  const int Lp = blend ? lod + 1 : lod;
  const int64_t nv_t = ANALYTIC ? 0 : md.nvox[Lp + 1];
  int ray = -1, p = 0, e = 0, k = 0, cp = -1;
  bool ready = false;
  float t = 0.0f, prev = __builtin_inff();
  float oo[3] = {0.0f, 0.0f, 0.0f}, dd[3] = {0.0f, 0.0f, 0.0f};
  int vox[NGL_MAX_LODS];
  uint32_t cell[NGL_MAX_LODS];
#pragma unroll
  for (int l = 0; l < NGL_MAX_LODS; ++l) {
    vox[l] = 0;
    cell[l] = 0;
  }
  // decoder fragments (MFMA form): LOD lod, and lod+1 when blending
  const int H = md.hidden;
  uint4* frag0 = reinterpret_cast<uint4*>(smem);
  uint4* frag1 = frag0 + (MFMA ? (H / 16) * S::KS * 64 : 0);
  float* w2s0 = reinterpret_cast<float*>(frag1 + (MFMA && blend ? (H / 16) * S::KS * 64 : 0));
  float* w2s1 = w2s0 + H;
  uint16_t* stage = reinterpret_cast<uint16_t*>(w2s1 + H) + (threadIdx.x >> 6) * 64 * S::ROW;
  float b2a = 0.0f, b2b = 0.0f;
  if constexpr (MFMA) {
    load_frags<M, XYZ>(md, lod, frag0, w2s0);
    if (blend) load_frags<M, XYZ>(md, lod + 1, frag1, w2s1);
    __syncthreads();
    b2a = md.b2[lod - 1];
    b2b = blend ? md.b2[lod] : 0.0f;
  }
  bool exhausted = false;  // wave-uniform
  auto finish = [&](uint8_t st, int32_t hv) {
    A.t_hit[ray] = t;
    A.status[ray] = st;
    A.steps[ray] = k;
    A.hit_vox[ray] = hv;
    ray = -1;
    ready = false;
  };
  for (;;) {
    // 1. refill idle lanes and move every ray to an evaluable state
    for (int round = 0; round < 8; ++round) {
      const uint64_t need = __ballot(ray < 0);
      if (need && !exhausted) {
        const int n = __popcll(need);
        const int first = __ffsll((unsigned long long)need) - 1;
        unsigned int base = 0;
        if (lane == first) base = atomicAdd(A.counter, unsigned(n));
        base = __shfl(base, first, 64);
        if (int64_t(base) + n >= R) exhausted = true;
        if (ray < 0) {
          const int64_t my = int64_t(base) + __popcll(need & ((1ull << lane) - 1ull));
          if (my < R) {
            ray = int(my);
            p = A.ray_off[ray];
            e = A.ray_off[ray + 1];
            k = 0;
            cp = -1;
            prev = __builtin_inff();
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              oo[a] = A.o[a * R + ray];
              dd[a] = A.d[a * R + ray];
            }
            t = p < e ? A.t_in[p] : 0.0f;
            bool bad = false;
#pragma unroll
            for (int a = 0; a < 3; ++a) bad = bad || !__builtin_isfinite(oo[a]) || !__builtin_isfinite(dd[a]);
            if (bad) finish(NGL_RAY_INVALID, -1);
          }
        }
      }
      if (ray >= 0 && !ready) {
        while (p < e && t > A.t_out[p]) ++p;  // empty space: next voxel
        if (p == e) {
          finish(NGL_RAY_MISS, -1);
        } else {
          const float ti = A.t_in[p];
          if (t < ti) t = ti;  // outside the voxel: jump to its entry
          if (t > A.prm.t_far) finish(NGL_RAY_FAR, -1);
          else if (k == A.prm.max_steps) finish(NGL_RAY_MAX_STEPS, -1);
          else ready = true;
        }
      }
      const bool waiting = (ray < 0 && !exhausted) || (ray >= 0 && !ready);
      if (__ballot(waiting) == 0) break;
    }
    const bool act = ray >= 0 && ready;
    if (__ballot(act) == 0) {
      if (exhausted && __ballot(ray >= 0) == 0) break;
      continue;
    }
    // 2. one SDF evaluation per active lane
    float dist = 0.0f;
    int32_t v = -1;
    float x[3] = {0.0f, 0.0f, 0.0f};
    float z[M];
#pragma unroll
    for (int q = 0; q < M; ++q) z[q] = 0.0f;
    bool ok = false;  // this lane evaluates the model
    if (act) {
      x[0] = fmaf(t, dd[0], oo[0]);
      x[1] = fmaf(t, dd[1], oo[1]);
      x[2] = fmaf(t, dd[2], oo[2]);
      v = A.pair_vox[p];
      if constexpr (ANALYTIC) {
        const float q0 = x[0] - A.prm.sphere[0], q1 = x[1] - A.prm.sphere[1], q2 = x[2] - A.prm.sphere[2];
        dist = sqrtf(q0 * q0 + q1 * q1 + q2 * q2) - A.prm.sphere[3];
      } else {
        if (v < 0 || int64_t(v) >= nv_t) {
          finish(NGL_RAY_INVALID, -1);  // hit list does not belong to this depth
        } else {
          if (p != cp) {
            // ancestor chain of the pair's voxel (parents always exist)
            int w = v;
#pragma unroll
            for (int l = NGL_MAX_LODS; l >= 1; --l) {
              if (l <= Lp) {
                vox[l - 1] = w;
                cell[l - 1] = md.cell[l + 1][w];
                w = md.parent[l + 1][w];
              }
            }
            cp = p;
          }
#pragma unroll
          for (int l = 1; l <= NGL_MAX_LODS; ++l)
            if (l <= lod)
              interp_level<M, FT>(md, l, vox[l - 1], cell_x(cell[l - 1]), cell_y(cell[l - 1]), cell_z(cell[l - 1]), x, z);
          ok = true;
        }
      }
    }
    if constexpr (!ANALYTIC) {
      if constexpr (MFMA) {
        // every lane joins the wavefront's decode; idle lanes stage zeros
        stage_row<M, XYZ>(stage, x, z);
        wave_lds_sync();
        dist = wave_decode<M, XYZ>(frag0, w2s0, b2a, stage, H);
        if (blend) {
          // with alpha > 0 the pair voxel is the level lod+1 voxel
          if (ok) interp_level<M, FT>(md, lod + 1, v, cell_x(md.cell[Lp + 1][v]), cell_y(md.cell[Lp + 1][v]),
                                      cell_z(md.cell[Lp + 1][v]), x, z);
          wave_lds_sync();
          stage_row<M, XYZ>(stage, x, z);
          wave_lds_sync();
          dist = (1.0f - A.alpha) * dist + A.alpha * wave_decode<M, XYZ>(frag1, w2s1, b2b, stage, H);
        }
        wave_lds_sync();
      } else if (ok) {
        dist = decode_f32<M, XYZ>(md, lod, x, z);
        if (blend) {
          interp_level<M, FT>(md, lod + 1, v, cell_x(md.cell[Lp + 1][v]), cell_y(md.cell[Lp + 1][v]),
                              cell_z(md.cell[Lp + 1][v]), x, z);
          dist = (1.0f - A.alpha) * dist + A.alpha * decode_f32<M, XYZ>(md, lod + 1, x, z);
        }
      }
    }
    // 3. step
    if (act && ray >= 0) {
      ++k;
      if (dist < A.prm.delta) {
        finish(NGL_RAY_HIT, v);
      } else if (A.prm.osc_check && fabsf(dist - prev) < 6.0f * A.prm.delta) {
        finish(NGL_RAY_STALLED, -1);
      } else {
        prev = dist;
        t += dist;
        ready = false;
      }
    }
  }
}

__global__ void k_zero_counter(unsigned int* c) {
  if (threadIdx.x == 0) *c = 0u;
}

// Enough blocks to fill every CU at the kernel's occupancy (one value per
// instantiation, computed on first use).
template <int M, typename FT, bool XYZ, bool ANALYTIC, bool MFMA, int NW>
static int persistent_grid(size_t lds) {
  static int cached = 0;
  if (cached) return cached;
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1024;
  const void* kern = reinterpret_cast<const void*>(&k_sphere_trace<M, FT, XYZ, ANALYTIC, MFMA, NW>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, 64 * NW, lds) != hipSuccess || per < 1) per = 1;
  cached = cus * per;
  return cached;
}

template <int M, typename FT, bool XYZ, bool ANALYTIC, bool MFMA, int NW>
static int launch_trace_nw(const ngl_model& md, const TraceArgs& A, hipStream_t s, size_t lds) {
  k_zero_counter<<<1, 64, 0, s>>>(A.counter);
  int grid = persistent_grid<M, FT, XYZ, ANALYTIC, MFMA, NW>(lds);
  const int64_t need = (A.R + 64 * NW - 1) / (64 * NW);
  if (need < grid) grid = int(need);
  k_sphere_trace<M, FT, XYZ, ANALYTIC, MFMA, NW><<<grid, 64 * NW, lds, s>>>(md, A);
  NGL_LAUNCHED();
  return NGL_OK;
}

template <int M, typename FT, bool XYZ, bool ANALYTIC>
static int launch_trace(const ngl_model& md, const TraceArgs& A, hipStream_t s) {
  using S = MfmaShape<M, XYZ>;
  if (ANALYTIC || md.w_dtype != NGL_BF16) return launch_trace_nw<M, FT, XYZ, ANALYTIC, false, 4>(md, A, s, 0);
  const size_t fixed = size_t(S::frag_bytes(md.hidden)) * (A.alpha > 0.0f ? 2 : 1) + 2 * sizeof(float) * md.hidden;
  if (fixed + 4 * S::STAGE_BYTES <= 65536)
    return launch_trace_nw<M, FT, XYZ, false, true, 4>(md, A, s, fixed + 4 * S::STAGE_BYTES);
  if (fixed + 2 * S::STAGE_BYTES <= 65536)
    return launch_trace_nw<M, FT, XYZ, false, true, 2>(md, A, s, fixed + 2 * S::STAGE_BYTES);
  return launch_trace_nw<M, FT, XYZ, false, true, 1>(md, A, s, fixed + S::STAGE_BYTES);
}

template <int M, typename FT, bool XYZ>
struct TraceOp {
  static int run(const ngl_model& md, const TraceArgs& A, hipStream_t s) { return launch_trace<M, FT, XYZ, false>(md, A, s); }
};

}  // namespace ngl

extern "C" {

int ngl_sphere_trace_workspace(size_t* bytes) {
  NGL_REQUIRE(bytes != nullptr, "bytes is null");
  *bytes = 256;
  return NGL_OK;
}

int ngl_sphere_trace(const ngl_model* m, const float* o, const float* d, int64_t R, int32_t lod, float alpha,
                     const int32_t* pair_vox, const float* t_in, const float* t_out, const int32_t* ray_off,
                     const ngl_trace_params* params, float* t_hit, uint8_t* status, int32_t* steps,
                     int32_t* hit_vox, void* ws, size_t ws_bytes, void* stream) {
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
  NGL_REQUIRE(ws != nullptr && ws_bytes >= 256, "workspace too small: %zu < 256 bytes", ws_bytes);
  hipStream_t s = (hipStream_t)stream;
  TraceArgs A{o, d, R, int(lod), alpha, pair_vox, t_in, t_out, ray_off, *params, t_hit, status, steps, hit_vox,
              static_cast<unsigned int*>(ws)};
  if (analytic) return launch_trace<8, F32, true, true>(*m, A, s);
  const ngl_model& md = *m;
#define NGL_TRACE_XYZ(M_, FT_) \
  return md.with_xyz ? TraceOp<M_, FT_, true>::run(md, A, s) : TraceOp<M_, FT_, false>::run(md, A, s)
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
}

}  // extern "C"
