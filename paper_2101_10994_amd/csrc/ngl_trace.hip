// Adaptive-stepping sphere tracing (Sec. 3.4, Fig. 3; stopping rules of
// App. A.4) on gfx950.  Each ray walks its front-to-back voxel list from the
// ray-octree intersection: outside the current voxel it jumps to the voxel's
// entry, inside it evaluates the SDF from that voxel and its ancestors and
// takes a sphere-tracing step.
#include "ngl_trace_impl.h"

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
  TraceArgs A{o, d, R, 0, R, int(lod), alpha, pair_vox, t_in, t_out, ray_off, *params, t_hit, status, steps,
              hit_vox, static_cast<unsigned int*>(ws), nullptr, nullptr};
  if (analytic) return trace_run_analytic(*m, A, s);
  NGL_BY_WIDTH(m->feat_dim, trace_run, *m, A, s)
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
  k_batch_init<<<1, 64, 0, s>>>(L.counters, L.live, I, frame_clock);
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
  for (int i = 0; i < n; ++i) B.view[i] = BatchView{L.base[i], I.R[i], views[i].lod, views[i].alpha};
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
  NGL_BY_WIDTH(m0.feat_dim, batch_run, m0, B, any_blend, s)
}

}  // extern "C"
