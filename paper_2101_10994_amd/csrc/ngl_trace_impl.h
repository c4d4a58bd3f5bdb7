// Sphere-tracing kernels and their launchers (Sec. 3.4, Fig. 3; stopping
// rules of App. A.4), shared by the per-width translation units
// ngl_trace_m{8,16,32,64}.hip and the entry points in ngl_trace.hip.
#pragma once

#include "ngl_common.h"
#include "ngl_device.h"
#include "ngl_mfma.h"

namespace ngl {

struct TraceArgs {
  const float* o;         // this view's rays, SoA [3][stride]
  const float* d;
  int64_t stride;         // SoA stride of o and d
  int64_t base;           // index of this view's first ray in the outputs
  int64_t R;              // rays of this view
  int lod;
  float alpha;
  const int32_t* pair_vox;  // this view's hit lists
  const float* t_in;
  const float* t_out;
  const int32_t* ray_off;   // [R+1]
  ngl_trace_params prm;
  float* t_hit;           // outputs indexed base + ray
  uint8_t* status;
  int32_t* steps;
  int32_t* hit_vox;
  unsigned int* counter;  // this view's work queue head (zeroed before the launch)
  unsigned int* live;     // nullable: rays of this view not yet finished
  uint64_t* done_clock;   // nullable: timestamp when the view's last ray ends
  // Per-ray LOD selection (all zero/null otherwise):
  int pair_depth;                     // depth of the hit lists (0: that of lod, +1 when blending)
  const int32_t* ray_ids;             // nullable: the queue serves these ray ids
  const unsigned int* bucket_counts;  // nullable: ray_ids is split into buckets of these sizes ...
  int bucket;                         // ... and this launch serves bucket `bucket`
  const float* alpha_pp;              // nullable: blend weight per ray (replaces alpha)
  const unsigned int* bucket_sizes;   // nullable: bucket b starts at the sum of these sizes below b
                                      // (bucket_counts then give each bucket's live entries)
  // Phased tracing (all zero/null otherwise): a ray about to take evaluation
  // number pause_at is parked (state saved, id appended to `parked`) so the
  // next launch can serve the long rays from a dense queue; `resume` starts
  // each queued ray from its parked state.
  int pause_at;
  bool resume;
  float* st_t;
  int32_t* st_p;
  int32_t* st_k;
  float* st_prev;
  int32_t* parked;
  unsigned int* parked_n;
  bool wide;  // host side: serve the queue with the wide (lanes-per-ray) kernel
  bool l1;    // level 1's table staged in LDS (k_sphere_trace, set by its launcher)
};

// The launch evaluates decoders lod and lod+1.
__host__ __device__ inline bool trace_blend(const TraceArgs& A) { return A.alpha > 0.0f || A.alpha_pp != nullptr; }

// Continuous LOD from a distance (Sec. 3.4, LOD Selection), in FP32 with
// every operation rounded in this order (the oracle's orc_lod_select):
// u = clamp((dist - d_near) / (d_far - d_near), 0, 1),
// L = lod_near + (lod_far - lod_near) * u clamped to the LODs' range,
// L* = floor(L), alpha = L - L*
// (L* = num_lods and alpha = 0 when L >= num_lods).
__device__ inline void lod_of_distance(const ngl_lod_select& s, int num_lods, float dist, float* Lc, int* Li,
                                       float* alpha) {
#pragma clang fp contract(off)
  float u = (dist - s.d_near) / (s.d_far - s.d_near);
  if (u < 0.0f) u = 0.0f;
  if (u > 1.0f) u = 1.0f;
  const float span = s.lod_far - s.lod_near;
  const float prod = span * u;
  float L = s.lod_near + prod;
  const float lo = fminf(s.lod_near, s.lod_far), hi = fmaxf(s.lod_near, s.lod_far);
  if (L < lo) L = lo;
  if (L > hi) L = hi;
  int li = int(floorf(L));
  float a = L - float(li);
  if (li >= num_lods) {
    li = num_lods;
    a = 0.0f;
  }
  *Lc = L;
  *Li = li;
  *alpha = a;
}

// Voxels of levels 1..Lp on the ancestor chain of pair voxel v (level
// Lpair; parents always exist) and the cell of the level-Lc voxel, Lc =
// min(Lp, Lpair); the cell of an ancestor at level l <= Lc is that cell's
// coordinates shifted right by Lc - l (cells nest).  With `known`, vox and
// cLc hold the chain of an earlier pair of the same ray, and the walk stops
// at the first ancestor already held: everything above it is the same.
__device__ __forceinline__ void ancestor_chain(const ngl_model& md, int v, int Lpair, int Lp, bool known, int* vox,
                                               uint32_t* cLc) {
  const int Lc = Lp < Lpair ? Lp : Lpair;
  int w = v;
#pragma unroll
  for (int l = NGL_MAX_LODS; l >= 1; --l) {
    if (l <= Lpair) {
      if (l <= Lp) {
        if (known && vox[l - 1] == w) break;
        vox[l - 1] = w;
        if (l == Lc) *cLc = md.cell[l + 1][w];
      }
      w = md.parent[l + 1][w];
    }
  }
}

// Packed cell at level l of the ancestor of the level-Lc cell c.
__device__ __forceinline__ uint32_t cell_at(uint32_t c, int Lc, int l) {
  const int sh = Lc - l;
  return pack_cell(cell_x(c) >> sh, cell_y(c) >> sh, cell_z(c) >> sh);
}

// Ray served at queue position q: with an image width W (a multiple of 8,
// the image a whole number of 8-row bands) the queue walks 8x8 pixel tiles
// in row-major order, so 64 consecutive positions are a tile of
// neighbouring pixels; otherwise q itself.
__device__ inline int queue_ray(int64_t q, int W) {
  if (W <= 0) return int(q);
  const int64_t tile = q >> 6, tiles_x = W >> 3;
  const int w = int(q & 63);
  const int64_t row = (tile / tiles_x) * 8 + (w >> 3), col = (tile % tiles_x) * 8 + (w & 7);
  return int(row * W + col);
}

#ifndef NGL_TRACE_COOP
#define NGL_TRACE_COOP 1
#endif

// serve_queue gathers features cooperatively, one 16-ray tile at a time,
// for FP32 features on the matrix cores (with 16-bit features one lane per
// ray measured faster); its staging rows per wavefront follow.
#ifndef NGL_TRACE_COOP_HALF
#define NGL_TRACE_COOP_HALF 1
#endif
template <typename FT, bool ANALYTIC, bool MFMA>
constexpr bool trace_coop() {
  return MFMA && !ANALYTIC && NGL_TRACE_COOP && (NGL_TRACE_COOP_HALF || std::is_same<FT, F32>::value);
}
template <typename FT, bool ANALYTIC, bool MFMA, class DEC>
constexpr int trace_stage_bytes() {
  return trace_coop<FT, ANALYTIC, MFMA>() ? DEC::TILE_BYTES : DEC::STAGE_BYTES;
}

// One wavefront serves a view's ray queue.  Each lane keeps one ray; a lane
// whose ray terminates takes the next ray from the queue, so every step is
// evaluated on a compacted set of active rays.  Every ray ends after at most
// max_steps evaluations and one pass over its pairs, and the queue is finite,
// so the loop ends.  All lanes of the wavefront reach the matrix-core decode
// together (idle lanes stage zeros).
template <int M, typename FT, bool XYZ, bool ANALYTIC, bool MFMA, class DEC>
__device__ __forceinline__ void serve_queue(const ngl_model& md, const TraceArgs& A, const DecLds<DEC>& S, float b2a,
                                            float b2b, const void* l1s = nullptr, bool l1 = false) {
  const int lane = threadIdx.x & 63;
  const bool blend = trace_blend(A);
  const int lod = A.lod;
  const int Lp = blend ? lod + 1 : lod;
  const int PD = A.pair_depth > 0 ? A.pair_depth : Lp + 1;  // depth of the pairs
  const int Lpair = PD - 1;                                 // their feature level
  const int Lc = Lp < Lpair ? Lp : Lpair;                   // deepest level of the held chain
  const int64_t nv_t = ANALYTIC ? 0 : md.nvox[PD];
  int64_t R = A.R;  // queue length
  const int32_t* ids = A.ray_ids;
  if (A.bucket_counts) {
    unsigned off = 0;
    for (int b = 0; b < A.bucket; ++b) off += A.bucket_sizes ? A.bucket_sizes[b] : A.bucket_counts[b];
    R = A.bucket_counts[A.bucket];
    ids += off;
  }
  float al = A.alpha;  // this lane's blend weight
  const int H = md.hidden;
  // matrix-core tracers over FP32 features gather rows cooperatively (see
  // coop_level); with 16-bit features one lane per ray measured faster
  constexpr bool COOP = trace_coop<FT, ANALYTIC, MFMA>();
  int ray = -1, p = 0, e = 0, k = 0, cp = -1;
  // the current pair's t_in, t_out and voxel, loaded together when p moves
  int pc = -1, v_c = -1;
  float tin_c = 0.0f, tout_c = 0.0f;
  bool ready = false;
  float t = 0.0f, prev = __builtin_inff();
  float oo[3] = {0.0f, 0.0f, 0.0f}, dd[3] = {0.0f, 0.0f, 0.0f};
  int vox[NGL_MAX_LODS];
  uint32_t cLc = 0;  // cell of the level-Lc voxel (the blend level lod + 1 when Lc = Lp)
#pragma unroll
  for (int l = 0; l < NGL_MAX_LODS; ++l) vox[l] = 0;
  bool exhausted = false;  // wave-uniform
  unsigned nfin = 0;       // rays this lane finished since the last report
#define NGL_FINISH(st_, hv_)            \
  do {                                  \
    const int64_t g_ = A.base + ray;    \
    A.t_hit[g_] = t;                    \
    A.status[g_] = (st_);               \
    A.steps[g_] = k;                    \
    A.hit_vox[g_] = (hv_);              \
    ray = -1;                           \
    ready = false;                      \
    ++nfin;                             \
  } while (0)
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
            ray = ids ? ids[my] : queue_ray(my, A.prm.image_width);
            if (A.alpha_pp) al = A.alpha_pp[ray];
            p = A.ray_off[ray];
            e = A.ray_off[ray + 1];
            k = 0;
            cp = -1;
            pc = -1;
            prev = __builtin_inff();
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              oo[a] = A.o[a * A.stride + ray];
              dd[a] = A.d[a * A.stride + ray];
            }
            t = p < e ? A.t_in[p] : 0.0f;
            if (A.resume) {
              t = A.st_t[ray];
              p = A.st_p[ray];
              k = A.st_k[ray];
              prev = A.st_prev[ray];
            }
            bool bad = false;
#pragma unroll
            for (int a = 0; a < 3; ++a) bad = bad || !__builtin_isfinite(oo[a]) || !__builtin_isfinite(dd[a]);
            if (bad) NGL_FINISH(NGL_RAY_INVALID, -1);
          }
        }
      }
      if (ray >= 0 && !ready) {
        while (p < e) {  // empty space: next voxel
          if (p != pc) {
            tin_c = A.t_in[p];
            tout_c = A.t_out[p];
            v_c = A.pair_vox[p];
            pc = p;
          }
          if (t > tout_c) ++p;
          else break;
        }
        if (p == e) {
          NGL_FINISH(NGL_RAY_MISS, -1);
        } else {
          const float ti = tin_c;
          if (t < ti) t = ti;  // outside the voxel: jump to its entry
          if (t > A.prm.t_far) NGL_FINISH(NGL_RAY_FAR, -1);
          else if (k == A.prm.max_steps) NGL_FINISH(NGL_RAY_MAX_STEPS, -1);
          else if (A.pause_at > 0 && k == A.pause_at) {
            // park: the state reproduces this point exactly on resumption
            A.st_t[ray] = t;
            A.st_p[ray] = p;
            A.st_k[ray] = k;
            A.st_prev[ray] = prev;
            A.parked[atomicAdd(A.parked_n, 1u)] = ray;
            ray = -1;
          } else {
            ready = true;
          }
        }
      }
      const bool waiting = (ray < 0 && !exhausted) || (ray >= 0 && !ready);
      if (__ballot(waiting) == 0) break;
    }
    const bool act = ray >= 0 && ready;
    const bool any_act = __ballot(act) != 0;
    const bool done = !any_act && exhausted && __ballot(ray >= 0) == 0;
    if (any_act) {
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
        v = v_c;
        if constexpr (ANALYTIC) {
          const float q0 = x[0] - A.prm.sphere[0], q1 = x[1] - A.prm.sphere[1], q2 = x[2] - A.prm.sphere[2];
          dist = sqrtf(q0 * q0 + q1 * q1 + q2 * q2) - A.prm.sphere[3];
        } else {
          if (v < 0 || int64_t(v) >= nv_t) {
            NGL_FINISH(NGL_RAY_INVALID, -1);  // hit list does not belong to this depth
          } else {
            if (p != cp) {
              ancestor_chain(md, v, Lpair, Lp, cp >= 0, vox, &cLc);
              cp = p;
            }
            if constexpr (!COOP) {
#pragma unroll
              for (int l = 1; l <= NGL_MAX_LODS; ++l)
                if (l <= lod)
                  interp_level<M, FT>(md, l, vox[l - 1], cell_x(cell_at(cLc, Lc, l)),
                                      cell_y(cell_at(cLc, Lc, l)), cell_z(cell_at(cLc, Lc, l)), x, z);
            }
            ok = true;
          }
        }
      }
      if constexpr (!ANALYTIC) {
        if constexpr (MFMA) {
          if constexpr (COOP) {
            // cooperative gather of the evaluating lanes' features, one
            // 16-ray tile at a time (tiles without one are skipped), the 4
            // lanes of group r serving ray 16 t + r
            constexpr int D = TileShape<M>::D;
            const int r = lane >> 2, g = lane & 3;
            const uint64_t okm = __ballot(ok);
            const bool mix = ok && al > 0.0f;  // Eq. 3 blend with the level lod+1 voxel
            const uint64_t mixing = blend ? __ballot(mix) : 0ull;
            typename DEC::Stage* rows = S.stage;
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) {
              if (((okm >> (16 * tt)) & 0xffffull) == 0) continue;
              const int q = 16 * tt + r;
              float xq[3];
#pragma unroll
              for (int a = 0; a < 3; ++a) xq[a] = __shfl(x[a], q, 64);
              float acc[D];
#pragma unroll
              for (int i = 0; i < D; ++i) acc[i] = 0.0f;
              const uint32_t cq_lc = uint32_t(__shfl(int(cLc), q, 64));
#pragma unroll
              for (int l = 1; l <= NGL_MAX_LODS; ++l)
                if (l <= lod) {
                  const uint32_t cq = cell_at(cq_lc, Lc, l);
                  tile_level<M, FT>(md, l, __shfl(ok ? vox[l - 1] : -1, q, 64), xq, cell_x(cq), cell_y(cq), cell_z(cq),
                                    g, acc, l1s, l1);
                }
              DEC::template tile_slice<D>(rows, r, g * D, acc);
              if (g == 0) DEC::tile_rest(rows, r, xq);
              wave_lds_sync();
              float d = b2a + DEC::tile(S.frag0, S.w2s0, rows, H);
              if (blend && ((mixing >> (16 * tt)) & 0xffffull)) {
                wave_lds_sync();
                const uint32_t cq = cq_lc;  // level lod + 1 = Lp
                tile_level<M, FT>(md, lod + 1, __shfl(mix ? vox[lod] : -1, q, 64), xq, cell_x(cq), cell_y(cq),
                                  cell_z(cq), g, acc);
                DEC::template tile_slice<D>(rows, r, g * D, acc);
                wave_lds_sync();
                const float d1 = b2b + DEC::tile(S.frag1, S.w2s1, rows, H);
                if (mix) d = (1.0f - al) * d + al * d1;
              }
              wave_lds_sync();
              if ((lane >> 4) == tt) dist = d;  // lane 16 tt + j owns ray slot 16 tt + j
            }
          } else {
          DEC::stage(S.stage, x, z);
          wave_lds_sync();
          // point tiles without an evaluating lane are skipped (the tail of
          // the queue runs waves with few live rays)
          dist = DEC::decode(S.frag0, S.w2s0, b2a, S.stage, H, __ballot(ok));
          const bool mix = ok && al > 0.0f;  // Eq. 3 blend with the level lod+1 voxel
          const uint64_t mixing = __ballot(mix);
          if (blend && mixing) {
            if (mix) interp_level<M, FT>(md, lod + 1, vox[lod], cell_x(cLc), cell_y(cLc), cell_z(cLc), x, z);
            wave_lds_sync();
            DEC::stage(S.stage, x, z);
            wave_lds_sync();
            const float d1 = DEC::decode(S.frag1, S.w2s1, b2b, S.stage, H, mixing);
            if (mix) dist = (1.0f - al) * dist + al * d1;
          }
          wave_lds_sync();
          }
        } else if (ok) {
          dist = decode_f32<M, XYZ>(md, lod, x, z);
          if (blend && al > 0.0f) {
            interp_level<M, FT>(md, lod + 1, vox[lod], cell_x(cLc), cell_y(cLc), cell_z(cLc), x, z);
            dist = (1.0f - al) * dist + al * decode_f32<M, XYZ>(md, lod + 1, x, z);
          }
        }
      }
      // 3. step
      if (act && ray >= 0) {
        ++k;
        if (dist < A.prm.delta) {
          NGL_FINISH(NGL_RAY_HIT, v);
        } else if (A.prm.osc_check && fabsf(dist - prev) < 6.0f * A.prm.delta) {
          NGL_FINISH(NGL_RAY_STALLED, -1);
        } else {
          prev = dist;
          t += dist;
          ready = false;
        }
      }
    }
    if (A.live) {
      // report finished rays once per iteration; the wavefront that takes
      // the count to zero stamps the view's end time
      unsigned tot = nfin;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) tot += __shfl_xor(tot, off, 64);
      nfin = 0;
      if (lane == 0 && tot > 0) {
        const unsigned old = atomicSub(A.live, tot);
        if (old == tot && A.done_clock) *A.done_clock = wall_clock64();
      }
    }
    if (done) break;
  }
}

#undef NGL_FINISH

// Register budget of the one-lane-per-ray tracers: at most 168 VGPRs, so
// three wavefronts fit on a SIMD (the dependent feature loads need them to
// overlap).
#ifndef NGL_TRACE_WAVES_PER_EU
#define NGL_TRACE_WAVES_PER_EU 3
#endif

template <int M, typename FT, bool XYZ, bool ANALYTIC, bool MFMA, int NW, class DEC>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NGL_TRACE_WAVES_PER_EU)))
void k_sphere_trace(ngl_model md, TraceArgs A) {
  extern __shared__ __align__(16) char smem[];
  const bool blend = trace_blend(A);
  const int H = md.hidden;
  DecLds<DEC> S(smem, H, blend && MFMA, trace_stage_bytes<FT, ANALYTIC, MFMA, DEC>() / 4);
  // level 1's table after the staging rows (when the launch reserved it)
  char* l1s = smem + DecLds<DEC>::fixed_bytes(H, blend && MFMA) + NW * size_t(trace_stage_bytes<FT, ANALYTIC, MFMA, DEC>());
  float b2a = 0.0f, b2b = 0.0f;
  if constexpr (MFMA) {
    DEC::load(md, A.lod, S.frag0, S.w2s0);
    if (blend) DEC::load(md, A.lod + 1, S.frag1, S.w2s1);
    if (A.l1) stage_l1<M, FT>(md, l1s);
    __syncthreads();
    b2a = md.b2[A.lod - 1];
    b2b = blend ? md.b2[A.lod] : 0.0f;
  }
  serve_queue<M, FT, XYZ, ANALYTIC, MFMA, DEC>(md, A, S, b2a, b2b, l1s, A.l1);
}

// Lanes per ray of the wide tracer (a divisor of the feature width M).
#ifndef NGL_TRACE_WIDE_LANES
#define NGL_TRACE_WIDE_LANES 8
#endif
template <int M>
constexpr int wide_lanes() {
  return NGL_TRACE_WIDE_LANES < M ? NGL_TRACE_WIDE_LANES : M;
}

// Wide form of serve_queue for the long rays left after the first phase:
// a group of G lanes serves one ray, lane g holding the feature slice
// [g*D, g*D + D) of every level.  A step's loads are then two short
// dependent rounds (corner ids, then row slices) spread over G lanes,
// where one lane per ray issues every row load itself; a few long rays
// finish in far less time.  Each feature element is accumulated over the
// same corners and levels in the same order, the staged decoder row and
// the step rule are those of serve_queue, so results are the same bits.
template <int M, typename FT, bool XYZ, class DEC, int G>
__device__ __forceinline__ void serve_queue_wide(const ngl_model& md, const TraceArgs& A, const DecLds<DEC>& S,
                                                 float* zbuf, float b2a, float b2b) {
  constexpr int D = M / G;    // feature elements per lane
  constexpr int NS = 64 / G;  // rays per wavefront
  constexpr int ZR = M + 1;   // zbuf row stride (odd: spreads LDS banks)
  static_assert(M % G == 0 && 64 % G == 0 && NS <= 16, "wide tracer shape");
  const int lane = threadIdx.x & 63;
  const int slot = lane / G, g = lane % G, lead = slot * G;
  const bool blend = trace_blend(A);
  const int lod = A.lod;
  const int Lp = blend ? lod + 1 : lod;
  const int PD = A.pair_depth > 0 ? A.pair_depth : Lp + 1;
  const int Lpair = PD - 1;
  const int Lc = Lp < Lpair ? Lp : Lpair;
  const int64_t nv_t = md.nvox[PD];
  int64_t R = A.R;
  const int32_t* ids = A.ray_ids;
  if (A.bucket_counts) {
    unsigned off = 0;
    for (int b = 0; b < A.bucket; ++b) off += A.bucket_sizes ? A.bucket_sizes[b] : A.bucket_counts[b];
    R = A.bucket_counts[A.bucket];
    ids += off;
  }
  float al = A.alpha;
  const int H = md.hidden;
  // ray state, the same in every lane of a group
  int ray = -1, p = 0, e = 0, k = 0, cp = -1;
  // the current pair's t_in, t_out and voxel, loaded together when p moves
  int pc = -1, v_c = -1;
  float tin_c = 0.0f, tout_c = 0.0f;
  bool ready = false;
  float t = 0.0f, prev = __builtin_inff();
  float oo[3] = {0.0f, 0.0f, 0.0f}, dd[3] = {0.0f, 0.0f, 0.0f};
  int vox[NGL_MAX_LODS];
  uint32_t cLc = 0;  // cell of the level-Lc voxel (the blend level lod + 1 when Lc = Lp)
#pragma unroll
  for (int l = 0; l < NGL_MAX_LODS; ++l) vox[l] = 0;
  bool exhausted = false;  // wave-uniform
  unsigned nfin = 0;
#define NGL_FINISH_W(st_, hv_)          \
  do {                                  \
    if (g == 0) {                       \
      const int64_t g_ = A.base + ray;  \
      A.t_hit[g_] = t;                  \
      A.status[g_] = (st_);             \
      A.steps[g_] = k;                  \
      A.hit_vox[g_] = (hv_);            \
      ++nfin;                           \
    }                                   \
    ray = -1;                           \
    ready = false;                      \
  } while (0)
  for (;;) {
    // 1. refill idle groups (requests made by each group's first lane)
    for (int round = 0; round < 8; ++round) {
      const uint64_t need = __ballot(ray < 0 && g == 0);
      if (need && !exhausted) {
        const int n = __popcll(need);
        const int first = __ffsll((unsigned long long)need) - 1;
        unsigned int base = 0;
        if (lane == first) base = atomicAdd(A.counter, unsigned(n));
        base = __shfl(base, first, 64);
        if (int64_t(base) + n >= R) exhausted = true;
        const int64_t my = int64_t(base) + __popcll(need & ((1ull << lead) - 1ull));
        if (ray < 0 && my < R) {
          ray = ids ? ids[my] : queue_ray(my, A.prm.image_width);
          if (A.alpha_pp) al = A.alpha_pp[ray];
          p = A.ray_off[ray];
          e = A.ray_off[ray + 1];
          k = 0;
          cp = -1;
          pc = -1;
          prev = __builtin_inff();
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            oo[a] = A.o[a * A.stride + ray];
            dd[a] = A.d[a * A.stride + ray];
          }
          t = p < e ? A.t_in[p] : 0.0f;
          if (A.resume) {
            t = A.st_t[ray];
            p = A.st_p[ray];
            k = A.st_k[ray];
            prev = A.st_prev[ray];
          }
          bool bad = false;
#pragma unroll
          for (int a = 0; a < 3; ++a) bad = bad || !__builtin_isfinite(oo[a]) || !__builtin_isfinite(dd[a]);
          if (bad) NGL_FINISH_W(NGL_RAY_INVALID, -1);
        }
      }
      if (ray >= 0 && !ready) {
        while (p < e) {  // empty space: next voxel
          if (p != pc) {
            tin_c = A.t_in[p];
            tout_c = A.t_out[p];
            v_c = A.pair_vox[p];
            pc = p;
          }
          if (t > tout_c) ++p;
          else break;
        }
        if (p == e) {
          NGL_FINISH_W(NGL_RAY_MISS, -1);
        } else {
          const float ti = tin_c;
          if (t < ti) t = ti;
          if (t > A.prm.t_far) NGL_FINISH_W(NGL_RAY_FAR, -1);
          else if (k == A.prm.max_steps) NGL_FINISH_W(NGL_RAY_MAX_STEPS, -1);
          else if (A.pause_at > 0 && k == A.pause_at) {
            if (g == 0) {
              A.st_t[ray] = t;
              A.st_p[ray] = p;
              A.st_k[ray] = k;
              A.st_prev[ray] = prev;
              A.parked[atomicAdd(A.parked_n, 1u)] = ray;
            }
            ray = -1;
          } else {
            ready = true;
          }
        }
      }
      const bool waiting = (ray < 0 && !exhausted) || (ray >= 0 && !ready);
      if (__ballot(waiting) == 0) break;
    }
    const bool act = ray >= 0 && ready;
    const bool any_act = __ballot(act) != 0;
    const bool done = !any_act && exhausted && __ballot(ray >= 0) == 0;
    if (any_act) {
      // 2. this lane's slice of the interpolated features
      float x[3] = {0.0f, 0.0f, 0.0f};
      float acc[D];
#pragma unroll
      for (int i = 0; i < D; ++i) acc[i] = 0.0f;
      int32_t v = -1;
      bool ok = false;
      if (act) {
        x[0] = fmaf(t, dd[0], oo[0]);
        x[1] = fmaf(t, dd[1], oo[1]);
        x[2] = fmaf(t, dd[2], oo[2]);
        v = v_c;
        if (v < 0 || int64_t(v) >= nv_t) {
          NGL_FINISH_W(NGL_RAY_INVALID, -1);
        } else {
          if (p != cp) {
            ancestor_chain(md, v, Lpair, Lp, cp >= 0, vox, &cLc);
            cp = p;
          }
#pragma unroll
          for (int l = 1; l <= NGL_MAX_LODS; ++l)
            if (l <= lod)
              interp_level_slice<M, FT, D>(md, l, vox[l - 1], cell_x(cell_at(cLc, Lc, l)),
                                           cell_y(cell_at(cLc, Lc, l)), cell_z(cell_at(cLc, Lc, l)), x, g * D, acc);
          ok = true;
        }
      }
      // 3. lane s < NS stages ray slot s's point as row s and decodes it
      const int srow = lane < NS ? lane : 0;
      const int src = srow * G;
      float xs[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) xs[a] = __shfl(x[a], src, 64);
      const bool oks = (__shfl(int(ok), src, 64) != 0) && lane < NS;
      const float als = __shfl(al, src, 64);
      float zs[M];
#pragma unroll
      for (int i = 0; i < D; ++i) zbuf[slot * ZR + g * D + i] = acc[i];
      wave_lds_sync();
#pragma unroll
      for (int i = 0; i < M; ++i) zs[i] = oks ? zbuf[srow * ZR + i] : 0.0f;
      DEC::stage(S.stage, xs, zs);
      wave_lds_sync();
      float dist = DEC::decode(S.frag0, S.w2s0, b2a, S.stage, H, __ballot(oks));
      const bool mixs = oks && als > 0.0f;  // Eq. 3 blend with the level lod+1 voxel
      const uint64_t mixing = __ballot(mixs);
      if (blend && mixing) {
        if (ok && al > 0.0f)
          interp_level_slice<M, FT, D>(md, lod + 1, vox[lod], cell_x(cLc), cell_y(cLc),
                                       cell_z(cLc), x, g * D, acc);
#pragma unroll
        for (int i = 0; i < D; ++i) zbuf[slot * ZR + g * D + i] = acc[i];
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < M; ++i) zs[i] = mixs ? zbuf[srow * ZR + i] : 0.0f;
        DEC::stage(S.stage, xs, zs);
        wave_lds_sync();
        const float d1 = DEC::decode(S.frag1, S.w2s1, b2b, S.stage, H, mixing);
        if (mixs) dist = (1.0f - als) * dist + als * d1;
      }
      wave_lds_sync();
      dist = __shfl(dist, slot, 64);
      // 4. step, in every lane of the group
      if (act && ray >= 0) {
        ++k;
        if (dist < A.prm.delta) {
          NGL_FINISH_W(NGL_RAY_HIT, v);
        } else if (A.prm.osc_check && fabsf(dist - prev) < 6.0f * A.prm.delta) {
          NGL_FINISH_W(NGL_RAY_STALLED, -1);
        } else {
          prev = dist;
          t += dist;
          ready = false;
        }
      }
    }
    if (A.live) {
      unsigned tot = nfin;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) tot += __shfl_xor(tot, off, 64);
      nfin = 0;
      if (lane == 0 && tot > 0) {
        const unsigned old = atomicSub(A.live, tot);
        if (old == tot && A.done_clock) *A.done_clock = wall_clock64();
      }
    }
    if (done) break;
  }
#undef NGL_FINISH_W
}

template <int M, typename FT, bool XYZ, int NW, class DEC>
__global__ __launch_bounds__(64 * NW) void k_sphere_trace_wide(ngl_model md, TraceArgs A) {
  constexpr int G = wide_lanes<M>();
  extern __shared__ __align__(16) char smem[];
  const bool blend = trace_blend(A);
  const int H = md.hidden;
  DecLds<DEC> S(smem, H, blend);
  float* zbuf = reinterpret_cast<float*>(smem + DecLds<DEC>::fixed_bytes(H, blend) + NW * DEC::STAGE_BYTES) +
                (threadIdx.x >> 6) * (64 / G) * (M + 1);
  DEC::load(md, A.lod, S.frag0, S.w2s0);
  if (blend) DEC::load(md, A.lod + 1, S.frag1, S.w2s1);
  __syncthreads();
  serve_queue_wide<M, FT, XYZ, DEC, G>(md, A, S, zbuf, md.b2[A.lod - 1], blend ? md.b2[A.lod] : 0.0f);
}

// Batched form: views in one launch.  Each block walks the views once, in
// rotation from its own start; at each view that still has queued rays it
// copies the model into LDS, stages its decoder and serves the view's queue
// with all its wavefronts, then moves on.  Every block visits each view at
// most once, so the grid drains.
struct BatchView {
  int64_t base;      // first ray of the view in the concatenated arrays
  int64_t R;
  int32_t lod;
  float alpha;
  int32_t tile_w;    // image width when the view is served in 8x8 tiles, else 0
};

struct BatchArgs {
  const ngl_model* table;  // device [n]
  int n;
  BatchView view[NGL_MAX_BATCH];
  const float* o;          // view i's rays: SoA block [3][R_i] at 3 * base_i
  const float* d;
  int64_t cap;             // pair capacity per view
  const int32_t* pair_vox;  // [n][cap]
  const float* t_in;
  const float* t_out;
  const int32_t* ray_off;   // view i at base_i + i, [R_i + 1]
  ngl_trace_params prm;
  float* t_hit;
  uint8_t* status;
  int32_t* steps;
  int32_t* hit_vox;
  unsigned int* counters;   // [n] queue heads
  unsigned int* live;       // [n] unfinished rays
  uint64_t* clock;          // nullable [n+1]
  // Phased (all zero/null otherwise): the first launch parks rays at
  // evaluation pause_at into view v's range [base_v, base_v + R_v) of pids
  // (count in pcount[v]); with `resume` the launch serves those instead,
  // from queue heads heads2[v].  State arrays are indexed by base_v + ray.
  int pause_at;
  bool resume;
  bool wide;  // host side: the wide (lanes-per-ray) kernel
  float* st_t;
  int32_t* st_p;
  int32_t* st_k;
  float* st_prev;
  int32_t* pids;
  unsigned int* pcount;     // [n]
  unsigned int* heads2;     // [n]
};

// View v's queue of a batched launch (phase fields included).
__device__ inline TraceArgs batch_view_args(const BatchArgs& B, int v) {
  TraceArgs A{};
  const int64_t base = B.view[v].base;
  A.o = B.o + 3 * base;  // each view's rays are one SoA block
  A.d = B.d + 3 * base;
  A.stride = B.view[v].R;
  A.base = base;
  A.R = B.view[v].R;
  A.lod = B.view[v].lod;
  A.alpha = B.view[v].alpha;
  A.pair_vox = B.pair_vox + int64_t(v) * B.cap;
  A.t_in = B.t_in + int64_t(v) * B.cap;
  A.t_out = B.t_out + int64_t(v) * B.cap;
  A.ray_off = B.ray_off + base + v;
  A.prm = B.prm;
  A.prm.image_width = B.view[v].tile_w;
  A.t_hit = B.t_hit;
  A.status = B.status;
  A.steps = B.steps;
  A.hit_vox = B.hit_vox;
  A.counter = (B.resume ? B.heads2 : B.counters) + v;
  A.live = B.live + v;
  A.done_clock = B.clock ? B.clock + 1 + v : nullptr;
  if (B.pause_at > 0 || B.resume) {
    A.st_t = B.st_t + base;
    A.st_p = B.st_p + base;
    A.st_k = B.st_k + base;
    A.st_prev = B.st_prev + base;
  }
  if (B.pause_at > 0) {
    A.pause_at = B.pause_at;
    A.parked = B.pids + base;
    A.parked_n = B.pcount + v;
  }
  if (B.resume) {
    A.resume = true;
    A.ray_ids = B.pids + base;
    A.bucket_counts = B.pcount + v;
    A.bucket = 0;
  }
  return A;
}

// Rays still queued for view v in this launch.
__device__ inline bool batch_view_has(const BatchArgs& B, int v) {
  if (B.resume) return __atomic_load_n(&B.heads2[v], __ATOMIC_RELAXED) < __atomic_load_n(&B.pcount[v], __ATOMIC_RELAXED);
  return int64_t(__atomic_load_n(&B.counters[v], __ATOMIC_RELAXED)) < B.view[v].R;
}

template <int M, typename FT, bool XYZ, int NW, class DEC>
__global__ __launch_bounds__(64 * NW) void k_trace_batch(BatchArgs B) {
  extern __shared__ __align__(16) char smem[];
  __shared__ ngl_model smd;
  __shared__ int s_has;
  const int H = B.table[0].hidden;
  for (int step = 0; step < B.n; ++step) {
    const int v = (int(blockIdx.x) + step) % B.n;
    if (threadIdx.x == 0) s_has = batch_view_has(B, v);
    __syncthreads();
    if (!s_has) {
      __syncthreads();
      continue;
    }
    {
      const uint32_t* src = reinterpret_cast<const uint32_t*>(B.table + v);
      uint32_t* dst = reinterpret_cast<uint32_t*>(&smd);
      for (int w = threadIdx.x; w < int(sizeof(ngl_model) / 4); w += blockDim.x) dst[w] = src[w];
    }
    __syncthreads();
    const TraceArgs A = batch_view_args(B, v);
    const bool blend = A.alpha > 0.0f;
    DecLds<DEC> S(smem, H, blend, trace_stage_bytes<FT, false, true, DEC>() / 4);
    DEC::load(smd, A.lod, S.frag0, S.w2s0);
    if (blend) DEC::load(smd, A.lod + 1, S.frag1, S.w2s1);
    __syncthreads();
    serve_queue<M, FT, XYZ, false, true, DEC>(smd, A, S, smd.b2[A.lod - 1], blend ? smd.b2[A.lod] : 0.0f);
    __syncthreads();  // every wavefront is done with this view's LDS
  }
}

// Parked rays of a phased batch, eight lanes per ray (serve_queue_wide).
template <int M, typename FT, bool XYZ, int NW, class DEC>
__global__ __launch_bounds__(64 * NW) void k_trace_batch_wide(BatchArgs B) {
  constexpr int G = wide_lanes<M>();
  extern __shared__ __align__(16) char smem[];
  __shared__ ngl_model smd;
  __shared__ int s_has;
  const int H = B.table[0].hidden;
  for (int step = 0; step < B.n; ++step) {
    const int v = (int(blockIdx.x) + step) % B.n;
    if (threadIdx.x == 0) s_has = batch_view_has(B, v);
    __syncthreads();
    if (!s_has) {
      __syncthreads();
      continue;
    }
    {
      const uint32_t* src = reinterpret_cast<const uint32_t*>(B.table + v);
      uint32_t* dst = reinterpret_cast<uint32_t*>(&smd);
      for (int w = threadIdx.x; w < int(sizeof(ngl_model) / 4); w += blockDim.x) dst[w] = src[w];
    }
    __syncthreads();
    const TraceArgs A = batch_view_args(B, v);
    const bool blend = A.alpha > 0.0f;
    DecLds<DEC> S(smem, H, blend, trace_stage_bytes<FT, false, true, DEC>() / 4);
    S.stage = reinterpret_cast<typename DEC::Stage*>(smem + DecLds<DEC>::fixed_bytes(H, true)) +
              (threadIdx.x >> 6) * DEC::STAGE_ELEMS;
    float* zbuf = reinterpret_cast<float*>(smem + DecLds<DEC>::fixed_bytes(H, true) + NW * DEC::STAGE_BYTES) +
                  (threadIdx.x >> 6) * (64 / G) * (M + 1);
    DEC::load(smd, A.lod, S.frag0, S.w2s0);
    if (blend) DEC::load(smd, A.lod + 1, S.frag1, S.w2s1);
    __syncthreads();
    serve_queue_wide<M, FT, XYZ, DEC, G>(smd, A, S, zbuf, smd.b2[A.lod - 1], blend ? smd.b2[A.lod] : 0.0f);
    __syncthreads();
  }
}

// Per-pixel LOD groups in one launch: group b holds the rays of integer
// LOD first + b (ids grouped on the device, sizes in counts[first - 1 + b]).
// Each block visits the groups once, in rotation from its own start,
// stages that LOD's two decoders and serves the group's queue, so the
// groups' tails overlap instead of running one launch after another.
struct BucketArgs {
  TraceArgs base;  // rays, hit lists, outputs, pair depth, ids, counts, alpha_pp
  int first;       // LOD of group 0
  int n;           // groups
  unsigned int* heads;  // [NGL_MAX_LODS] queue heads (zeroed)
};

template <int M, typename FT, bool XYZ, bool MFMA, int NW, class DEC>
__global__ __launch_bounds__(64 * NW) void k_trace_buckets(ngl_model md, BucketArgs B) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_has;
  const int H = md.hidden;
  for (int step = 0; step < B.n; ++step) {
    const int b = (int(blockIdx.x) + step) % B.n;
    const int lod = B.first + b;
    if (threadIdx.x == 0)
      s_has = __atomic_load_n(&B.heads[lod - 1], __ATOMIC_RELAXED) < B.base.bucket_counts[lod - 1];
    __syncthreads();
    if (!s_has) {
      __syncthreads();
      continue;
    }
    TraceArgs A = B.base;
    A.lod = lod;
    A.bucket = lod - 1;
    A.counter = B.heads + (lod - 1);
    if (lod >= md.num_lods) A.alpha_pp = nullptr;  // the finest LOD does not blend
    if (A.pause_at > 0) {
      // parked rays of group b go to the group's own range of the id list
      unsigned off = 0;
      for (int q = 0; q < lod - 1; ++q) off += A.bucket_counts[q];
      A.parked = B.base.parked + off;
      A.parked_n = B.base.parked_n + (lod - 1);
    }
    const bool blend = trace_blend(A);
    DecLds<DEC> S(smem, H, blend && MFMA, trace_stage_bytes<FT, false, MFMA, DEC>() / 4);
    float b2a = 0.0f, b2b = 0.0f;
    if constexpr (MFMA) {
      DEC::load(md, lod, S.frag0, S.w2s0);
      if (blend) DEC::load(md, lod + 1, S.frag1, S.w2s1);
      __syncthreads();
      b2a = md.b2[lod - 1];
      b2b = blend ? md.b2[lod] : 0.0f;
    }
    serve_queue<M, FT, XYZ, false, MFMA, DEC>(md, A, S, b2a, b2b);
    __syncthreads();  // every wavefront is done with this group's LDS
  }
}

// Parked rays of the LOD groups, eight lanes per ray (serve_queue_wide):
// group b's parked ids sit at its original offset, base.bucket_counts
// holds how many were parked, base.bucket_sizes the original sizes.
template <int M, typename FT, bool XYZ, int NW, class DEC>
__global__ __launch_bounds__(64 * NW) void k_trace_buckets_wide(ngl_model md, BucketArgs B) {
  constexpr int G = wide_lanes<M>();
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_has;
  const int H = md.hidden;
  for (int step = 0; step < B.n; ++step) {
    const int b = (int(blockIdx.x) + step) % B.n;
    const int lod = B.first + b;
    if (threadIdx.x == 0)
      s_has = __atomic_load_n(&B.heads[lod - 1], __ATOMIC_RELAXED) < B.base.bucket_counts[lod - 1];
    __syncthreads();
    if (!s_has) {
      __syncthreads();
      continue;
    }
    TraceArgs A = B.base;
    A.lod = lod;
    A.bucket = lod - 1;
    A.counter = B.heads + (lod - 1);
    if (lod >= md.num_lods) A.alpha_pp = nullptr;
    const bool blend = trace_blend(A);
    DecLds<DEC> S(smem, H, blend);
    // the slice buffers follow the staging areas of the blending layout (the largest)
    float* zbuf = reinterpret_cast<float*>(smem + DecLds<DEC>::fixed_bytes(H, true) + NW * DEC::STAGE_BYTES) +
                  (threadIdx.x >> 6) * (64 / G) * (M + 1);
    S.stage = reinterpret_cast<typename DEC::Stage*>(smem + DecLds<DEC>::fixed_bytes(H, true)) +
              (threadIdx.x >> 6) * DEC::STAGE_ELEMS;
    DEC::load(md, lod, S.frag0, S.w2s0);
    if (blend) DEC::load(md, lod + 1, S.frag1, S.w2s1);
    __syncthreads();
    serve_queue_wide<M, FT, XYZ, DEC, G>(md, A, S, zbuf, md.b2[lod - 1], blend ? md.b2[lod] : 0.0f);
    __syncthreads();
  }
}

static __global__ void k_zero_counter(unsigned int* c) {
  if (threadIdx.x == 0) *c = 0u;
}

template <int M, typename FT, bool XYZ, bool ANALYTIC, bool MFMA, int NW, class DEC>
static int launch_trace_nw(const ngl_model& md, const TraceArgs& A, hipStream_t s, size_t lds) {
  k_zero_counter<<<1, 64, 0, s>>>(A.counter);
  const void* kern = reinterpret_cast<const void*>(&k_sphere_trace<M, FT, XYZ, ANALYTIC, MFMA, NW, DEC>);
  int grid = resident_grid(kern, 64 * NW, lds, option(NGL_OPT_TRACE_BLOCKS_PER_CU));
  const int64_t need = (A.R + 64 * NW - 1) / (64 * NW);
  if (need < grid) grid = int(need);
  k_sphere_trace<M, FT, XYZ, ANALYTIC, MFMA, NW, DEC><<<grid, 64 * NW, lds, s>>>(md, A);
  NGL_LAUNCHED();
  return NGL_OK;
}

template <int M, typename FT, bool XYZ, int NW, class DEC>
static int launch_trace_wide_nw(const ngl_model& md, const TraceArgs& A, hipStream_t s, size_t lds) {
  k_zero_counter<<<1, 64, 0, s>>>(A.counter);
  constexpr int NS = 64 / wide_lanes<M>();
  const void* kern = reinterpret_cast<const void*>(&k_sphere_trace_wide<M, FT, XYZ, NW, DEC>);
  int grid = resident_grid(kern, 64 * NW, lds, option(NGL_OPT_TRACE_BLOCKS_PER_CU));
  const int64_t need = (A.R + NS * NW - 1) / (NS * NW);
  if (need < grid) grid = int(need);
  k_sphere_trace_wide<M, FT, XYZ, NW, DEC><<<grid, 64 * NW, lds, s>>>(md, A);
  NGL_LAUNCHED();
  return NGL_OK;
}

template <int M, typename FT, bool XYZ, class DEC>
static int launch_trace_wide(const ngl_model& md, const TraceArgs& A, hipStream_t s) {
  const size_t fixed = DecLds<DEC>::fixed_bytes(md.hidden, trace_blend(A));
  const size_t per_wave = DEC::STAGE_BYTES + size_t(64 / wide_lanes<M>()) * (M + 1) * 4;
  if (fixed + 4 * per_wave <= 65536) return launch_trace_wide_nw<M, FT, XYZ, 4, DEC>(md, A, s, fixed + 4 * per_wave);
  if (fixed + 2 * per_wave <= 65536) return launch_trace_wide_nw<M, FT, XYZ, 2, DEC>(md, A, s, fixed + 2 * per_wave);
  return launch_trace_wide_nw<M, FT, XYZ, 1, DEC>(md, A, s, fixed + per_wave);
}

template <int M, typename FT, bool XYZ, class DEC>
static int launch_trace_mfma(const ngl_model& md, const TraceArgs& A, hipStream_t s) {
  if (A.wide) return launch_trace_wide<M, FT, XYZ, DEC>(md, A, s);
  const size_t fixed = DecLds<DEC>::fixed_bytes(md.hidden, trace_blend(A));
  const int want = option(NGL_OPT_TRACE_WAVES);
  constexpr size_t SB = trace_stage_bytes<FT, false, true, DEC>();
  // level 1's rows in LDS (cooperative gather) when the table fits beside the decoder
  constexpr size_t L1B = trace_coop<FT, false, true>() ? l1_bytes<M, FT>() : 0;
  TraceArgs B = A;
  auto go = [&](int nw, auto launch) {
    size_t lds = fixed + nw * SB;
    B.l1 = L1B > 0 && l1_fits(md) && lds + L1B <= 65536;
    if (B.l1) lds += L1B;
    return launch(lds);
  };
  if ((want == 0 || want >= 4) && fixed + 4 * SB <= 65536)
    return go(4, [&](size_t lds) { return launch_trace_nw<M, FT, XYZ, false, true, 4, DEC>(md, B, s, lds); });
  if ((want == 0 || want >= 2) && fixed + 2 * SB <= 65536)
    return go(2, [&](size_t lds) { return launch_trace_nw<M, FT, XYZ, false, true, 2, DEC>(md, B, s, lds); });
  return go(1, [&](size_t lds) { return launch_trace_nw<M, FT, XYZ, false, true, 1, DEC>(md, B, s, lds); });
}

template <int M, typename FT, bool XYZ, bool ANALYTIC>
static int launch_trace(const ngl_model& md, const TraceArgs& A, hipStream_t s) {
  if (ANALYTIC) return launch_trace_nw<M, FT, XYZ, true, false, 4, DecF32<M, XYZ>>(md, A, s, 0);
  if (md.w_dtype == NGL_BF16) return launch_trace_mfma<M, FT, XYZ, DecBF16<M, XYZ>>(md, A, s);
  if (option(NGL_OPT_F32_DECODER) == 1) return launch_trace_mfma<M, FT, XYZ, DecF32<M, XYZ>>(md, A, s);
  return launch_trace_nw<M, FT, XYZ, false, false, 4, DecF32<M, XYZ>>(md, A, s, 0);
}

template <int M, typename FT, bool XYZ, int NW, class DEC>
static int launch_batch_nw(const BatchArgs& B, hipStream_t s, size_t lds) {
  const void* kern = reinterpret_cast<const void*>(&k_trace_batch<M, FT, XYZ, NW, DEC>);
  const int grid = resident_grid(kern, 64 * NW, lds, option(NGL_OPT_TRACE_BLOCKS_PER_CU));
  k_trace_batch<M, FT, XYZ, NW, DEC><<<grid, 64 * NW, lds, s>>>(B);
  NGL_LAUNCHED();
  return NGL_OK;
}

template <int M, typename FT, bool XYZ, class DEC>
static int launch_batch(const BatchArgs& B, bool any_blend, int H, hipStream_t s) {
  const size_t fixed = DecLds<DEC>::fixed_bytes(H, any_blend);
  const int want = option(NGL_OPT_TRACE_WAVES);
  constexpr size_t SB = trace_stage_bytes<FT, false, true, DEC>();
  if ((want == 0 || want >= 4) && fixed + 4 * SB <= 65536)
    return launch_batch_nw<M, FT, XYZ, 4, DEC>(B, s, fixed + 4 * SB);
  if ((want == 0 || want >= 2) && fixed + 2 * SB <= 65536)
    return launch_batch_nw<M, FT, XYZ, 2, DEC>(B, s, fixed + 2 * SB);
  return launch_batch_nw<M, FT, XYZ, 1, DEC>(B, s, fixed + SB);
}

template <int M, typename FT, bool XYZ, int NW, class DEC>
static int launch_batch_wide_nw(const BatchArgs& B, hipStream_t s, size_t lds) {
  const void* kern = reinterpret_cast<const void*>(&k_trace_batch_wide<M, FT, XYZ, NW, DEC>);
  const int grid = resident_grid(kern, 64 * NW, lds, option(NGL_OPT_TRACE_BLOCKS_PER_CU));
  k_trace_batch_wide<M, FT, XYZ, NW, DEC><<<grid, 64 * NW, lds, s>>>(B);
  NGL_LAUNCHED();
  return NGL_OK;
}

template <int M, typename FT, bool XYZ, class DEC>
static int launch_batch_wide(const BatchArgs& B, int H, hipStream_t s) {
  const size_t fixed = DecLds<DEC>::fixed_bytes(H, true);
  const size_t per_wave = DEC::STAGE_BYTES + size_t(64 / wide_lanes<M>()) * (M + 1) * 4;
  if (fixed + 4 * per_wave <= 65536) return launch_batch_wide_nw<M, FT, XYZ, 4, DEC>(B, s, fixed + 4 * per_wave);
  if (fixed + 2 * per_wave <= 65536) return launch_batch_wide_nw<M, FT, XYZ, 2, DEC>(B, s, fixed + 2 * per_wave);
  return launch_batch_wide_nw<M, FT, XYZ, 1, DEC>(B, s, fixed + per_wave);
}

template <int M, typename FT, bool XYZ>
struct BatchOp {
  static int run(const ngl_model& md, const BatchArgs& B, bool any_blend, hipStream_t s) {
    if (B.wide) {
      if (md.w_dtype == NGL_BF16) return launch_batch_wide<M, FT, XYZ, DecBF16<M, XYZ>>(B, md.hidden, s);
      return launch_batch_wide<M, FT, XYZ, DecF32<M, XYZ>>(B, md.hidden, s);
    }
    if (md.w_dtype == NGL_BF16) return launch_batch<M, FT, XYZ, DecBF16<M, XYZ>>(B, any_blend, md.hidden, s);
    return launch_batch<M, FT, XYZ, DecF32<M, XYZ>>(B, any_blend, md.hidden, s);
  }
};

struct BatchInit {
  int n;
  int64_t R[NGL_MAX_BATCH];
};

static __global__ void k_batch_init(unsigned int* counters, unsigned int* live, BatchInit I, uint64_t* clock,
                                    unsigned int* pcount, unsigned int* heads2) {
  const int i = threadIdx.x;
  if (i < I.n) {
    counters[i] = 0u;
    live[i] = unsigned(I.R[i]);
    pcount[i] = 0u;
    heads2[i] = 0u;
  }
  if (i == 0 && clock) clock[0] = wall_clock64();
}

template <int M, typename FT, bool XYZ, bool MFMA, int NW, class DEC>
static int launch_buckets_nw(const ngl_model& md, const BucketArgs& B, hipStream_t s, size_t lds) {
  const void* kern = reinterpret_cast<const void*>(&k_trace_buckets<M, FT, XYZ, MFMA, NW, DEC>);
  const int grid = resident_grid(kern, 64 * NW, lds, option(NGL_OPT_TRACE_BLOCKS_PER_CU));
  k_trace_buckets<M, FT, XYZ, MFMA, NW, DEC><<<grid, 64 * NW, lds, s>>>(md, B);
  NGL_LAUNCHED();
  return NGL_OK;
}

// Wavefronts per block from the LDS the two staged decoders leave.
template <int M, typename FT, bool XYZ, bool MFMA, class DEC>
static int launch_buckets(const ngl_model& md, const BucketArgs& B, hipStream_t s) {
  if constexpr (!MFMA) return launch_buckets_nw<M, FT, XYZ, false, 4, DEC>(md, B, s, 0);
  const size_t fixed = DecLds<DEC>::fixed_bytes(md.hidden, true);
  constexpr size_t SB = trace_stage_bytes<FT, false, MFMA, DEC>();
  if (fixed + 4 * SB <= 65536) return launch_buckets_nw<M, FT, XYZ, MFMA, 4, DEC>(md, B, s, fixed + 4 * SB);
  if (fixed + 2 * SB <= 65536) return launch_buckets_nw<M, FT, XYZ, MFMA, 2, DEC>(md, B, s, fixed + 2 * SB);
  return launch_buckets_nw<M, FT, XYZ, MFMA, 1, DEC>(md, B, s, fixed + SB);
}

template <int M, typename FT, bool XYZ, int NW, class DEC>
static int launch_buckets_wide_nw(const ngl_model& md, const BucketArgs& B, hipStream_t s, size_t lds) {
  const void* kern = reinterpret_cast<const void*>(&k_trace_buckets_wide<M, FT, XYZ, NW, DEC>);
  const int grid = resident_grid(kern, 64 * NW, lds, option(NGL_OPT_TRACE_BLOCKS_PER_CU));
  k_trace_buckets_wide<M, FT, XYZ, NW, DEC><<<grid, 64 * NW, lds, s>>>(md, B);
  NGL_LAUNCHED();
  return NGL_OK;
}

template <int M, typename FT, bool XYZ, class DEC>
static int launch_buckets_wide(const ngl_model& md, const BucketArgs& B, hipStream_t s) {
  const size_t fixed = DecLds<DEC>::fixed_bytes(md.hidden, true);
  const size_t per_wave = DEC::STAGE_BYTES + size_t(64 / wide_lanes<M>()) * (M + 1) * 4;
  if (fixed + 4 * per_wave <= 65536) return launch_buckets_wide_nw<M, FT, XYZ, 4, DEC>(md, B, s, fixed + 4 * per_wave);
  if (fixed + 2 * per_wave <= 65536) return launch_buckets_wide_nw<M, FT, XYZ, 2, DEC>(md, B, s, fixed + 2 * per_wave);
  return launch_buckets_wide_nw<M, FT, XYZ, 1, DEC>(md, B, s, fixed + per_wave);
}

template <int M, typename FT, bool XYZ>
struct BucketOp {
  static int run(const ngl_model& md, const BucketArgs& B, hipStream_t s) {
    if (B.base.wide) {
      if (md.w_dtype == NGL_BF16) return launch_buckets_wide<M, FT, XYZ, DecBF16<M, XYZ>>(md, B, s);
      return launch_buckets_wide<M, FT, XYZ, DecF32<M, XYZ>>(md, B, s);
    }
    if (md.w_dtype == NGL_BF16) return launch_buckets<M, FT, XYZ, true, DecBF16<M, XYZ>>(md, B, s);
    if (option(NGL_OPT_F32_DECODER) == 1) return launch_buckets<M, FT, XYZ, true, DecF32<M, XYZ>>(md, B, s);
    return launch_buckets<M, FT, XYZ, false, DecF32<M, XYZ>>(md, B, s);
  }
};

template <int M, typename FT, bool XYZ>
struct TraceOp {
  static int run(const ngl_model& md, const TraceArgs& A, hipStream_t s) { return launch_trace<M, FT, XYZ, false>(md, A, s); }
};

// Per-width and per-feature-type runners, defined in
// ngl_trace_m<width>_<type>.hip (one translation unit each, so the heavy
// kernel instantiations compile in parallel).
#define NGL_TRACE_DECLARE_FT(M_, T_)                                                                      \
  int trace_run_m##M_##_##T_(const ngl_model& md, const TraceArgs& A, hipStream_t s);                     \
  int batch_run_m##M_##_##T_(const ngl_model& md, const BatchArgs& B, bool any_blend, hipStream_t s);     \
  int bucket_run_m##M_##_##T_(const ngl_model& md, const BucketArgs& B, hipStream_t s);
#define NGL_TRACE_DECLARE(M_) NGL_TRACE_DECLARE_FT(M_, f32) NGL_TRACE_DECLARE_FT(M_, f16) NGL_TRACE_DECLARE_FT(M_, bf16)
NGL_TRACE_DECLARE(8)
NGL_TRACE_DECLARE(16)
NGL_TRACE_DECLARE(32)
NGL_TRACE_DECLARE(64)
#undef NGL_TRACE_DECLARE
#undef NGL_TRACE_DECLARE_FT
int trace_run_analytic(const ngl_model& md, const TraceArgs& A, hipStream_t s);

#define NGL_TRACE_DEFINE_FT(M_, T_, FT_)                                                                   \
  int trace_run_m##M_##_##T_(const ngl_model& md, const TraceArgs& A, hipStream_t s) {                     \
    return md.with_xyz ? TraceOp<M_, FT_, true>::run(md, A, s) : TraceOp<M_, FT_, false>::run(md, A, s);    \
  }                                                                                                        \
  int batch_run_m##M_##_##T_(const ngl_model& md, const BatchArgs& B, bool any_blend, hipStream_t s) {     \
    return md.with_xyz ? BatchOp<M_, FT_, true>::run(md, B, any_blend, s)                                  \
                       : BatchOp<M_, FT_, false>::run(md, B, any_blend, s);                                \
  }                                                                                                        \
  int bucket_run_m##M_##_##T_(const ngl_model& md, const BucketArgs& B, hipStream_t s) {                   \
    return md.with_xyz ? BucketOp<M_, FT_, true>::run(md, B, s) : BucketOp<M_, FT_, false>::run(md, B, s);  \
  }

}  // namespace ngl
