// Adaptive-stepping sphere tracing (Sec. 3.4, Fig. 3; stopping rules of
// App. A.4) on gfx950.  Each ray walks its front-to-back voxel list from the
// ray-octree intersection: outside the current voxel it jumps to the voxel's
// entry, inside it evaluates the SDF from that voxel and its ancestors and
// takes a sphere-tracing step.
#include "ngl_trace_impl.h"

#include <algorithm>
#include <cmath>
#include <mutex>

namespace ngl {

// Runners per feature width: the translation unit of the model's feature
// type (FP32, FP16 or BF16).
#define NGL_FT_SWITCH(fn, M_, ...)                          \
  switch (md.feat_dtype) {                                  \
    case NGL_F32: return fn##_m##M_##_f32(__VA_ARGS__);     \
    case NGL_F16: return fn##_m##M_##_f16(__VA_ARGS__);     \
    default: return fn##_m##M_##_bf16(__VA_ARGS__);         \
  }
#define NGL_TRACE_WIDTH_RUNNERS(M_)                                                                        \
  static int trace_run_m##M_(const ngl_model& md, const TraceArgs& A, hipStream_t s) {                     \
    NGL_FT_SWITCH(trace_run, M_, md, A, s)                                                                 \
  }                                                                                                        \
  static int batch_run_m##M_(const ngl_model& md, const BatchArgs& B, bool any_blend, hipStream_t s) {     \
    NGL_FT_SWITCH(batch_run, M_, md, B, any_blend, s)                                                      \
  }                                                                                                        \
  static int bucket_run_m##M_(const ngl_model& md, const BucketArgs& B, hipStream_t s) {                   \
    NGL_FT_SWITCH(bucket_run, M_, md, B, s)                                                                \
  }
NGL_TRACE_WIDTH_RUNNERS(8)
NGL_TRACE_WIDTH_RUNNERS(16)
NGL_TRACE_WIDTH_RUNNERS(32)
NGL_TRACE_WIDTH_RUNNERS(64)
#undef NGL_TRACE_WIDTH_RUNNERS
#undef NGL_FT_SWITCH

static int trace_by_width(const ngl_model& m, const TraceArgs& A, hipStream_t s) {
  NGL_BY_WIDTH(m.feat_dim, trace_run, m, A, s)
}

// Workspace of the phased trace: counters ([0..1] parked per phase, [4..6]
// queue heads), parked state per ray and two ping-pong id lists.
struct PhaseWS {
  unsigned* counts;
  float* st_t;
  int32_t* st_p;
  int32_t* st_k;
  float* st_prev;
  int32_t* ids[2];
  static constexpr size_t align(size_t b) { return (b + 255) & ~size_t(255); }
  static constexpr size_t bytes(int64_t R) { return 256 + 6 * align(4 * size_t(R)); }
  PhaseWS(void* ws, int64_t R) {
    char* p = static_cast<char*>(ws);
    const size_t a = align(4 * size_t(R));
    counts = reinterpret_cast<unsigned*>(p);
    st_t = reinterpret_cast<float*>(p + 256);
    st_p = reinterpret_cast<int32_t*>(p + 256 + a);
    st_k = reinterpret_cast<int32_t*>(p + 256 + 2 * a);
    st_prev = reinterpret_cast<float*>(p + 256 + 3 * a);
    ids[0] = reinterpret_cast<int32_t*>(p + 256 + 4 * a);
    ids[1] = reinterpret_cast<int32_t*>(p + 256 + 5 * a);
  }
};

__global__ void k_phase_init(unsigned* c) {
  if (threadIdx.x < 8) c[threadIdx.x] = 0u;
}

// Workspace of ngl_sphere_trace_static: the phased layout for
// NGL_STATIC_TRACE_MAX_RAYS rays (4 * R is a multiple of 256, so PhaseWS's
// aligned arrays fill it exactly).  Host code never passes this name to a
// kernel: its device address, per GPU, comes from static_trace_ws().
static_assert(PhaseWS::bytes(NGL_STATIC_TRACE_MAX_RAYS) == NGL_STATIC_TRACE_BYTES, "static trace workspace size");
static __device__ __align__(256) char scratch[NGL_STATIC_TRACE_BYTES];

// Device address of `scratch` on the current GPU, looked up once per GPU
// (each GPU holds its own copy of the array).
static int static_trace_ws(void** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  NGL_HIP(hipGetDevice(&dev));
  NGL_REQUIRE(dev >= 0 && dev < kMaxDevices, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    NGL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    NGL_REQUIRE(p != nullptr, "no device address for the static trace workspace");
    addr[dev] = p;
  }
  *out = addr[dev];
  return NGL_OK;
}

static int batch_by_width(const ngl_model& m, const BatchArgs& B, bool any_blend, hipStream_t s) {
  NGL_BY_WIDTH(m.feat_dim, batch_run, m, B, any_blend, s)
}

static int buckets_by_width(const ngl_model& m, const BucketArgs& B, hipStream_t s) {
  NGL_BY_WIDTH(m.feat_dim, bucket_run, m, B, s)
}

// Workspace of the per-ray LOD trace: [3][NGL_MAX_LODS] counters (group
// sizes, scatter cursors, queue heads), ray ids grouped by L*, blend weight
// and L* per ray.
struct LodWS {
  unsigned* counts;
  int32_t* ids;
  float* alpha;
  uint8_t* lint;
  static size_t align(size_t b) { return (b + 255) & ~size_t(255); }
  // phased form: parked state and ids per ray
  float* st_t = nullptr;
  int32_t* st_p = nullptr;
  int32_t* st_k = nullptr;
  float* st_prev = nullptr;
  int32_t* pids = nullptr;
  static size_t bytes(int64_t R) { return 256 + align(4 * size_t(R)) + align(4 * size_t(R)) + align(size_t(R)); }
  static size_t bytes_phased(int64_t R) { return bytes(R) + 5 * align(4 * size_t(R)); }
  LodWS(void* ws, int64_t R, bool phased) {
    char* p = static_cast<char*>(ws);
    counts = reinterpret_cast<unsigned*>(p);
    p += 256;
    ids = reinterpret_cast<int32_t*>(p);
    p += align(4 * size_t(R));
    alpha = reinterpret_cast<float*>(p);
    p += align(4 * size_t(R));
    lint = reinterpret_cast<uint8_t*>(p);
    p += align(size_t(R));
    if (phased) {
      st_t = reinterpret_cast<float*>(p);
      st_p = reinterpret_cast<int32_t*>(p + align(4 * size_t(R)));
      st_k = reinterpret_cast<int32_t*>(p + 2 * align(4 * size_t(R)));
      st_prev = reinterpret_cast<float*>(p + 3 * align(4 * size_t(R)));
      pids = reinterpret_cast<int32_t*>(p + 4 * align(4 * size_t(R)));
    }
  }
};

// counts: [0, MAX) group sizes, [MAX, 2 MAX) scatter offsets, [2 MAX, 3 MAX)
// queue heads, [3 MAX, 4 MAX) parked per group, [4 MAX, 5 MAX) heads of the
// parked queues.
__global__ void k_lod_init(unsigned* c) {
  if (threadIdx.x < 5 * NGL_MAX_LODS) c[threadIdx.x] = 0u;
}

// L* and alpha per ray; group sizes counted per block in LDS, then one
// global add per group and block.
__global__ __launch_bounds__(256) void k_lod_select(ngl_lod_select sel, int num_lods, int64_t R,
                                                    const int32_t* __restrict__ ray_off,
                                                    const float* __restrict__ t_in, float t_far, float* lod_out,
                                                    float* alpha, uint8_t* lint, unsigned* counts) {
  __shared__ unsigned cnt[NGL_MAX_LODS];
  if (threadIdx.x < NGL_MAX_LODS) cnt[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r < R) {
    const int b = ray_off[r], e = ray_off[r + 1];
    const float dist = b < e ? t_in[b] : t_far;
    float Lc, a;
    int li;
    lod_of_distance(sel, num_lods, dist, &Lc, &li, &a);
    if (lod_out) lod_out[r] = Lc;
    alpha[r] = a;
    lint[r] = uint8_t(li);
    atomicAdd(&cnt[li - 1], 1u);
  }
  __syncthreads();
  if (threadIdx.x < NGL_MAX_LODS && cnt[threadIdx.x]) atomicAdd(&counts[threadIdx.x], cnt[threadIdx.x]);
}

// Ray ids grouped by L*: ranks within the block from LDS counters, one
// global range reservation per group and block.
__global__ __launch_bounds__(256) void k_lod_scatter(int64_t R, const uint8_t* __restrict__ lint,
                                                     const unsigned* __restrict__ counts, unsigned* cursor,
                                                     int32_t* ids) {
  __shared__ unsigned cnt[NGL_MAX_LODS], base[NGL_MAX_LODS];
  if (threadIdx.x < NGL_MAX_LODS) cnt[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool in = r < R;
  const int li = in ? int(lint[r]) : 1;
  unsigned rank = 0;
  if (in) rank = atomicAdd(&cnt[li - 1], 1u);
  __syncthreads();
  if (threadIdx.x < NGL_MAX_LODS && cnt[threadIdx.x]) {
    unsigned off = 0;
    for (unsigned b = 0; b < threadIdx.x; ++b) off += counts[b];
    base[threadIdx.x] = off + atomicAdd(&cursor[threadIdx.x], cnt[threadIdx.x]);
  }
  __syncthreads();
  if (in) ids[base[li - 1] + rank] = int32_t(r);
}

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
  NGL_REQUIRE(params->image_width == 0 || (params->image_width > 0 && params->image_width % 8 == 0 &&
                                           R % (8 * int64_t(params->image_width)) == 0),
              "image_width %d: needs a multiple of 8 and R a multiple of 8 widths", params->image_width);
  if (!analytic) {
    NGL_REQUIRE(lod >= 1 && lod <= m->num_lods, "lod %d outside 1..%d", lod, m->num_lods);
    NGL_REQUIRE(!(alpha > 0.0f) || lod < m->num_lods, "blending needs lod < num_lods");
  }
  if (R == 0) return NGL_OK;
  NGL_REQUIRE(o && d && ray_off && t_hit && status && steps && hit_vox, "null buffer");
  NGL_REQUIRE(ws != nullptr && ws_bytes >= 256, "workspace too small: %zu < 256 bytes", ws_bytes);
  hipStream_t s = (hipStream_t)stream;
  TraceArgs A{o, d, R, 0, R, int(lod), alpha, pair_vox, t_in, t_out, ray_off, *params, t_hit, status, steps,
              hit_vox, static_cast<unsigned int*>(ws), nullptr, nullptr};
  if (analytic) return trace_run_analytic(*m, A, s);
  if (ws_bytes < PhaseWS::bytes(R)) return trace_by_width(*m, A, s);
  // Phased: rays still running at the first pause count (then the second)
  // are parked and served again from a dense queue, so the long grazing
  // rays finish in full wavefronts instead of a tail of near-empty ones.
  int pause[2], np = 0;
  const int p1 = option(NGL_OPT_TRACE_PAUSE1), p2 = option(NGL_OPT_TRACE_PAUSE2);
  if (p1 > 0 && p1 < params->max_steps) pause[np++] = p1;
  if (p2 > (np ? p1 : 0) && p2 < params->max_steps) pause[np++] = p2;
  if (np == 0) return trace_by_width(*m, A, s);
  const int phases = np + 1;
  PhaseWS W(ws, R);
  k_phase_init<<<1, 64, 0, s>>>(W.counts);
  NGL_LAUNCHED();
  for (int ph = 0; ph < phases; ++ph) {
    TraceArgs B = A;
    B.counter = W.counts + 4 + ph;
    B.pause_at = ph + 1 < phases ? pause[ph] : 0;
    B.st_t = W.st_t;
    B.st_p = W.st_p;
    B.st_k = W.st_k;
    B.st_prev = W.st_prev;
    if (ph + 1 < phases) {
      B.parked = W.ids[ph & 1];
      B.parked_n = W.counts + ph;
    }
    B.wide = ph > 0 && ph + 1 == phases && option(NGL_OPT_TRACE_WIDE) == 1;
    if (ph > 0) {
      B.resume = true;
      B.ray_ids = W.ids[(ph - 1) & 1];
      B.bucket_counts = W.counts + (ph - 1);
      B.bucket = 0;
    }
    rc = trace_by_width(*m, B, s);
    if (rc) return rc;
  }
  return NGL_OK;
}

int ngl_sphere_trace_static(const ngl_model* m, const float* o, const float* d, int64_t R, int32_t lod,
                            float alpha, const int32_t* pair_vox, const float* t_in, const float* t_out,
                            const int32_t* ray_off, const ngl_trace_params* params, float* t_hit,
                            uint8_t* status, int32_t* steps, int32_t* hit_vox, void* stream) {
  if (R > NGL_STATIC_TRACE_MAX_RAYS)
    NGL_FAIL(NGL_E_CAPACITY, "ngl_sphere_trace_static: %lld rays exceed NGL_STATIC_TRACE_MAX_RAYS (%d)",
             (long long)R, NGL_STATIC_TRACE_MAX_RAYS);
  void* ws = nullptr;
  int rc = ngl::static_trace_ws(&ws);
  if (rc) return rc;
  return ngl_sphere_trace(m, o, d, R, lod, alpha, pair_vox, t_in, t_out, ray_off, params, t_hit, status, steps,
                          hit_vox, ws, NGL_STATIC_TRACE_BYTES, stream);
}

int ngl_sphere_trace_workspace_rays(int64_t R, size_t* bytes) {
  NGL_REQUIRE(bytes != nullptr && R >= 0, "bad arguments");
  *bytes = ngl::PhaseWS::bytes(R);
  return NGL_OK;
}

int ngl_sphere_trace_lod_workspace(int64_t R, size_t* bytes) {
  NGL_REQUIRE(bytes != nullptr && R >= 0, "bad arguments");
  *bytes = ngl::LodWS::bytes_phased(R);
  return NGL_OK;
}

int ngl_sphere_trace_lod(const ngl_model* m, const float* o, const float* d, int64_t R, int32_t pair_depth,
                         const ngl_lod_select* sel, const int32_t* pair_vox, const float* t_in, const float* t_out,
                         const int32_t* ray_off, const ngl_trace_params* params, float* t_hit, uint8_t* status,
                         int32_t* steps, int32_t* hit_vox, float* lod_out, void* ws, size_t ws_bytes, void* stream) {
  using namespace ngl;
  NGL_REQUIRE(params != nullptr && sel != nullptr, "params or sel is null");
  NGL_REQUIRE(params->analytic == 0, "analytic mode has no LOD");
  int rc = check_model(m, true);
  if (rc) return rc;
  NGL_REQUIRE(R >= 0 && R < (int64_t(1) << 31), "ray count out of range");
  NGL_REQUIRE(params->max_steps >= 0, "max_steps must be >= 0");
  const int L = m->num_lods;
  NGL_REQUIRE(std::isfinite(sel->d_near) && std::isfinite(sel->d_far) && sel->d_far > sel->d_near,
              "need finite d_near < d_far");
  NGL_REQUIRE(sel->lod_near >= 1.0f && sel->lod_near <= float(L) && sel->lod_far >= 1.0f && sel->lod_far <= float(L),
              "lod_near and lod_far must be in [1, %d]", L);
  const float lmax = std::max(sel->lod_near, sel->lod_far), lmin = std::min(sel->lod_near, sel->lod_far);
  NGL_REQUIRE(pair_depth >= 2 && pair_depth <= L + 1 && float(pair_depth - 1) >= std::ceil(lmax),
              "pair_depth %d does not reach LOD %g (need depth >= %d, <= %d)", pair_depth, double(lmax),
              int(std::ceil(lmax)) + 1, L + 1);
  if (R == 0) return NGL_OK;
  NGL_REQUIRE(o && d && ray_off && t_hit && status && steps && hit_vox, "null buffer");
  NGL_REQUIRE(ws != nullptr && ws_bytes >= LodWS::bytes(R), "workspace too small: %zu < %zu bytes", ws_bytes,
              LodWS::bytes(R));
  hipStream_t s = (hipStream_t)stream;
  // Phased (matrix-core decoders, workspace large enough, a pause count
  // below max_steps and the wide phase enabled): rays still running at
  // the pause are parked per group and finished eight lanes per ray.
  const int pause = option(NGL_OPT_TRACE_PAUSE1);
  const bool phased = ws_bytes >= LodWS::bytes_phased(R) && pause > 0 && pause < params->max_steps &&
                      option(NGL_OPT_TRACE_WIDE) == 1 &&
                      (m->w_dtype == NGL_BF16 || option(NGL_OPT_F32_DECODER) == 1);
  LodWS W(ws, R, phased);
  k_lod_init<<<1, 64, 0, s>>>(W.counts);
  NGL_LAUNCHED();
  const unsigned g = unsigned((R + 255) / 256);
  k_lod_select<<<g, 256, 0, s>>>(*sel, L, R, ray_off, t_in, params->t_far, lod_out, W.alpha, W.lint, W.counts);
  NGL_LAUNCHED();
  k_lod_scatter<<<g, 256, 0, s>>>(R, W.lint, W.counts, W.counts + NGL_MAX_LODS, W.ids);
  NGL_LAUNCHED();
  const int first = std::max(1, int(std::floor(lmin)));
  const int last = std::min(L, int(std::floor(lmax)));
  BucketArgs B{};
  B.base = TraceArgs{o, d, R, 0, R, first, 0.0f, pair_vox, t_in, t_out, ray_off, *params, t_hit, status, steps,
                     hit_vox, nullptr, nullptr, nullptr};
  B.base.pair_depth = pair_depth;
  B.base.ray_ids = W.ids;
  B.base.bucket_counts = W.counts;
  B.base.alpha_pp = W.alpha;
  B.first = first;
  B.n = last - first + 1;
  B.heads = W.counts + 2 * NGL_MAX_LODS;  // zeroed by k_lod_init
  if (!phased) return buckets_by_width(*m, B, s);
  B.base.pause_at = pause;
  B.base.st_t = W.st_t;
  B.base.st_p = W.st_p;
  B.base.st_k = W.st_k;
  B.base.st_prev = W.st_prev;
  B.base.parked = W.pids;
  B.base.parked_n = W.counts + 3 * NGL_MAX_LODS;
  rc = buckets_by_width(*m, B, s);
  if (rc) return rc;
  BucketArgs C = B;
  C.base.pause_at = 0;
  C.base.parked = nullptr;
  C.base.parked_n = nullptr;
  C.base.resume = true;
  C.base.wide = true;
  C.base.ray_ids = W.pids;
  C.base.bucket_counts = W.counts + 3 * NGL_MAX_LODS;
  C.base.bucket_sizes = W.counts;
  C.heads = W.counts + 4 * NGL_MAX_LODS;
  return buckets_by_width(*m, C, s);
}

int ngl_model_table_bytes(int32_t n, size_t* bytes) {
  NGL_REQUIRE(bytes && n >= 1 && n <= NGL_MAX_BATCH, "n must be in 1..%d", NGL_MAX_BATCH);
  *bytes = sizeof(ngl_model) * size_t(n);
  return NGL_OK;
}

int ngl_model_table_upload(const ngl_model* models, int32_t n, void* table, void* stream) {
  NGL_REQUIRE(models && table && n >= 1 && n <= NGL_MAX_BATCH, "invalid model table upload");
  hipStream_t s = (hipStream_t)stream;
  NGL_HIP(hipMemcpyAsync(table, models, sizeof(ngl_model) * size_t(n), hipMemcpyHostToDevice, s));
  NGL_HIP(hipStreamSynchronize(s));
  return NGL_OK;
}

namespace {
struct BatchLayout {
  int64_t base[NGL_MAX_BATCH];
  int64_t R_total = 0, R_max = 0;
  float* o = nullptr;
  float* d = nullptr;
  int32_t* pair_ray = nullptr;
  int32_t* pair_vox = nullptr;
  float* t_in = nullptr;
  float* t_out = nullptr;
  int32_t* ray_off = nullptr;
  unsigned int* counters = nullptr;
  unsigned int* live = nullptr;
  unsigned int* pcount = nullptr;
  unsigned int* heads2 = nullptr;
  float* st_t = nullptr;
  int32_t* st_p = nullptr;
  int32_t* st_k = nullptr;
  float* st_prev = nullptr;
  int32_t* pids = nullptr;
  char* trav_ws = nullptr;
  size_t trav_bytes = 0;
  size_t bytes = 0;
};

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

BatchLayout batch_layout(const ngl_view* views, int n, int64_t cap, void* ws) {
  BatchLayout L;
  for (int i = 0; i < n; ++i) {
    const int64_t R = int64_t(views[i].width) * views[i].height;
    L.base[i] = L.R_total;
    L.R_total += R;
    if (R > L.R_max) L.R_max = R;
  }
  char* b = static_cast<char*>(ws);
  size_t off = 0;
  auto take = [&](size_t nb) {
    char* q = b ? b + off : nullptr;
    off += al256(nb);
    return q;
  };
  L.o = reinterpret_cast<float*>(take(sizeof(float) * 3 * size_t(L.R_total)));
  L.d = reinterpret_cast<float*>(take(sizeof(float) * 3 * size_t(L.R_total)));
  L.pair_ray = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * size_t(n) * size_t(cap)));
  L.pair_vox = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * size_t(n) * size_t(cap)));
  L.t_in = reinterpret_cast<float*>(take(sizeof(float) * size_t(n) * size_t(cap)));
  L.t_out = reinterpret_cast<float*>(take(sizeof(float) * size_t(n) * size_t(cap)));
  L.ray_off = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * size_t(L.R_total + n)));
  L.counters = reinterpret_cast<unsigned int*>(take(sizeof(unsigned int) * NGL_MAX_BATCH));
  L.live = reinterpret_cast<unsigned int*>(take(sizeof(unsigned int) * NGL_MAX_BATCH));
  L.pcount = reinterpret_cast<unsigned int*>(take(sizeof(unsigned int) * NGL_MAX_BATCH));
  L.heads2 = reinterpret_cast<unsigned int*>(take(sizeof(unsigned int) * NGL_MAX_BATCH));
  L.st_t = reinterpret_cast<float*>(take(sizeof(float) * size_t(L.R_total)));
  L.st_p = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * size_t(L.R_total)));
  L.st_k = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * size_t(L.R_total)));
  L.st_prev = reinterpret_cast<float*>(take(sizeof(float) * size_t(L.R_total)));
  L.pids = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * size_t(L.R_total)));
  size_t tb = 0;
  ngl_trace_octree_workspace(L.R_max, cap, &tb);
  L.trav_bytes = tb;
  L.trav_ws = take(tb);
  L.bytes = off;
  return L;
}
}  // namespace

int ngl_render_batch_workspace(const ngl_view* views, int32_t n, int64_t pair_capacity, size_t* bytes) {
  NGL_REQUIRE(views && bytes && n >= 1 && n <= NGL_MAX_BATCH, "n must be in 1..%d", NGL_MAX_BATCH);
  NGL_REQUIRE(pair_capacity >= 0 && pair_capacity < (int64_t(1) << 31), "pair_capacity out of range");
  *bytes = batch_layout(views, n, pair_capacity, nullptr).bytes;
  return NGL_OK;
}

int ngl_render_batch(const ngl_model* models, const void* table, const ngl_view* views, int32_t n,
                     const ngl_trace_params* params, int64_t pair_capacity, void* ws, size_t ws_bytes, float* t_hit,
                     uint8_t* status, int32_t* steps, int32_t* hit_vox, int64_t* counts, uint64_t* frame_clock,
                     void* stream) {
  using namespace ngl;
  NGL_REQUIRE(models && table && views && params, "null argument");
  NGL_REQUIRE(n >= 1 && n <= NGL_MAX_BATCH, "n must be in 1..%d", NGL_MAX_BATCH);
  NGL_REQUIRE(params->analytic == 0, "batched rendering traces the models (analytic mode is per call)");
  NGL_REQUIRE(params->max_steps >= 0, "max_steps must be >= 0");
  NGL_REQUIRE(t_hit && status && steps && hit_vox && counts, "null output buffer");
  const ngl_model& m0 = models[0];
  bool any_blend = false;
  for (int i = 0; i < n; ++i) {
    const ngl_model* m = models + i;
    int rc = check_model(m, true);
    if (rc) return rc;
    NGL_REQUIRE(m->feat_dim == m0.feat_dim && m->hidden == m0.hidden && m->with_xyz == m0.with_xyz &&
                    m->feat_dtype == m0.feat_dtype && m->w_dtype == m0.w_dtype,
                "model %d differs in feat_dim, hidden, with_xyz or dtypes from model 0", i);
    const ngl_view& v = views[i];
    NGL_REQUIRE(v.width > 0 && v.height > 0, "view %d has an empty image", i);
    NGL_REQUIRE(v.lod >= 1 && v.lod <= m->num_lods, "view %d: lod %d outside 1..%d", i, v.lod, m->num_lods);
    NGL_REQUIRE(v.alpha >= 0.0f && v.alpha < 1.0f, "view %d: alpha must be in [0,1)", i);
    NGL_REQUIRE(!(v.alpha > 0.0f) || v.lod < m->num_lods, "view %d: blending needs lod < num_lods", i);
    NGL_REQUIRE(m->nvox[0] > 0, "model %d is empty", i);
    any_blend = any_blend || v.alpha > 0.0f;
  }
  BatchLayout L = batch_layout(views, n, pair_capacity, ws);
  NGL_REQUIRE(L.R_total < (int64_t(1) << 31), "too many rays in the batch");
  NGL_REQUIRE(ws != nullptr && ws_bytes >= L.bytes, "workspace too small: %zu < %zu bytes", ws_bytes, L.bytes);
  hipStream_t s = (hipStream_t)stream;
  BatchInit I{};
  I.n = n;
  for (int i = 0; i < n; ++i) I.R[i] = int64_t(views[i].width) * views[i].height;
  k_batch_init<<<1, 64, 0, s>>>(L.counters, L.live, I, frame_clock, L.pcount, L.heads2);
  NGL_LAUNCHED();
  // rays and hit lists, view by view (the traversal workspace is reused)
  for (int i = 0; i < n; ++i) {
    const ngl_view& v = views[i];
    const int64_t R = I.R[i];
    float* o = L.o + 3 * L.base[i];
    float* d = L.d + 3 * L.base[i];
    int rc = ngl_camera_rays(v.eye, v.target, v.up, v.fov_y_deg, v.width, v.height, o, d, stream);
    if (rc) return rc;
    const int depth = (v.alpha > 0.0f ? v.lod + 1 : v.lod) + 1;
    const int64_t pb = int64_t(i) * pair_capacity;
    rc = ngl_trace_octree(models + i, o, d, R, depth, pair_capacity, L.trav_ws, L.trav_bytes, L.pair_ray + pb,
                          L.pair_vox + pb, L.t_in + pb, L.t_out + pb, L.ray_off + L.base[i] + i, counts + 2 * i,
                          stream);
    if (rc) return rc;
  }
  BatchArgs B{};
  B.table = static_cast<const ngl_model*>(table);
  B.n = n;
  for (int i = 0; i < n; ++i) {
    const bool tiles = views[i].width % 8 == 0 && views[i].height % 8 == 0;
    B.view[i] = BatchView{L.base[i], I.R[i], views[i].lod, views[i].alpha, tiles ? views[i].width : 0};
  }
  B.o = L.o;
  B.d = L.d;
  B.cap = pair_capacity;
  B.pair_vox = L.pair_vox;
  B.t_in = L.t_in;
  B.t_out = L.t_out;
  B.ray_off = L.ray_off;
  B.prm = *params;
  B.t_hit = t_hit;
  B.status = status;
  B.steps = steps;
  B.hit_vox = hit_vox;
  B.counters = L.counters;
  B.live = L.live;
  B.clock = frame_clock;
  // Phased as ngl_sphere_trace: rays still running at the pause count are
  // parked per view and finished by the lanes-per-ray kernel.
  const int pause = option(NGL_OPT_TRACE_PAUSE1);
  if (!(pause > 0 && pause < params->max_steps && option(NGL_OPT_TRACE_WIDE) == 1))
    return batch_by_width(m0, B, any_blend, s);
  B.pause_at = pause;
  B.st_t = L.st_t;
  B.st_p = L.st_p;
  B.st_k = L.st_k;
  B.st_prev = L.st_prev;
  B.pids = L.pids;
  B.pcount = L.pcount;
  B.heads2 = L.heads2;
  const int rc1 = batch_by_width(m0, B, any_blend, s);
  if (rc1) return rc1;
  BatchArgs C = B;
  C.pause_at = 0;
  C.resume = true;
  C.wide = true;
  return batch_by_width(m0, C, any_blend, s);
}

}  // extern "C"
