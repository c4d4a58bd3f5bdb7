// Status strings, thread-local error text and model validation for the C ABI.
#include "ngl_common.h"

#include <atomic>
#include <map>
#include <mutex>
#include <tuple>

namespace ngl {

static thread_local std::string g_last_error;

// Library options; defaults are the fastest measured choices.
static std::atomic<int> g_options[NGL_OPT_COUNT] = {{1}, {0}, {0}, {24}, {0}, {1}, {1}, {0}};

int option(int key) { return (key >= 0 && key < NGL_OPT_COUNT) ? g_options[key].load() : 0; }

int resident_grid(const void* kern, int threads, size_t lds, int cap) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, int, size_t>, std::pair<int, int>> cache;  // -> (CUs, per CU)
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  const auto key = std::make_tuple(dev, kern, threads, lds);
  std::pair<int, int> v;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
      v = it->second;
    } else {
      int cus = 0, per = 0;
      if (dev < 0 || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, threads, lds) != hipSuccess || per < 1) per = 1;
      v = std::make_pair(cus, per);
      cache.emplace(key, v);
    }
  }
  const int per = (cap > 0 && cap < v.second) ? cap : v.second;
  return v.first * per;
}

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

int check_model(const ngl_model* m, bool need_features) {
  NGL_REQUIRE(m != nullptr, "model is null");
  NGL_REQUIRE(m->num_lods >= 1 && m->num_lods <= NGL_MAX_LODS, "num_lods %d outside 1..%d", m->num_lods,
              NGL_MAX_LODS);
  const int D = m->num_lods + 1;
  for (int d = 0; d <= D; ++d) {
    NGL_REQUIRE(m->nvox[d] >= 0 && m->nvox[d] < (int64_t(1) << 31), "nvox[%d] out of range", d);
    if (m->nvox[d] > 0) {
      NGL_REQUIRE(m->cell[d] != nullptr, "cell[%d] is null", d);
      if (d < D) NGL_REQUIRE(m->child_mask[d] && m->first_child[d], "child arrays of depth %d are null", d);
      if (d > 0) NGL_REQUIRE(m->parent[d] != nullptr, "parent[%d] is null", d);
    }
  }
  if (!need_features) return NGL_OK;
  NGL_REQUIRE(m->feat_dim >= 8 && m->feat_dim <= NGL_MAX_FEAT_DIM && m->feat_dim % 8 == 0,
              "feat_dim %d must be a multiple of 8 in 8..%d", m->feat_dim, NGL_MAX_FEAT_DIM);
  NGL_REQUIRE(m->hidden >= 16 && m->hidden <= NGL_MAX_HIDDEN && m->hidden % 16 == 0,
              "hidden %d must be a multiple of 16 in 16..%d", m->hidden, NGL_MAX_HIDDEN);
  NGL_REQUIRE(m->feat_dtype == NGL_F32 || m->feat_dtype == NGL_F16 || m->feat_dtype == NGL_BF16,
              "unknown feat_dtype %d", m->feat_dtype);
  NGL_REQUIRE(m->w_dtype == NGL_F32 || m->w_dtype == NGL_BF16, "w_dtype %d must be F32 or BF16", m->w_dtype);
  NGL_REQUIRE(m->with_xyz == 0 || m->with_xyz == 1, "with_xyz must be 0 or 1");
  NGL_REQUIRE(m->b2 != nullptr, "b2 is null");
  for (int l = 1; l <= m->num_lods; ++l) {
    NGL_REQUIRE(m->ncorner[l - 1] >= 0 && m->ncorner[l - 1] < (int64_t(1) << 31), "ncorner[%d] out of range",
                l - 1);
    if (m->nvox[l + 1] > 0)
      NGL_REQUIRE(m->corners[l - 1] && m->feat[l - 1], "corner table or features of level %d are null", l);
    const uint64_t row = uint64_t(m->feat_dim) * (m->feat_dtype == NGL_F32 ? 4u : 2u);
    NGL_REQUIRE(uint64_t(m->ncorner[l - 1]) * row < (uint64_t(1) << 32), "features of level %d exceed 4 GiB", l);
    NGL_REQUIRE((reinterpret_cast<uintptr_t>(m->feat[l - 1]) & 15u) == 0 &&
                    (reinterpret_cast<uintptr_t>(m->corners[l - 1]) & 15u) == 0,
                "features and corner table of level %d must be 16-byte aligned", l);
    NGL_REQUIRE(m->W1[l - 1] && m->b1[l - 1] && m->w2[l - 1], "decoder %d is null", l);
  }
  return NGL_OK;
}

}  // namespace ngl

extern "C" {

const char* ngl_status_str(int s) {
  switch (s) {
    case NGL_OK: return "ok";
    case NGL_E_INVALID: return "invalid argument";
    case NGL_E_CAPACITY: return "capacity exceeded";
    case NGL_E_HIP: return "HIP runtime error";
    case NGL_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* ngl_last_error(void) { return ngl::g_last_error.c_str(); }

int ngl_version(void) { return 1; }

int ngl_set_option(int key, int value) {
  NGL_REQUIRE(key >= 0 && key < NGL_OPT_COUNT, "unknown option %d", key);
  if (key == NGL_OPT_F32_DECODER) NGL_REQUIRE(value == 0 || value == 1, "NGL_OPT_F32_DECODER takes 0 or 1");
  if (key == NGL_OPT_TRACE_WAVES)
    NGL_REQUIRE(value == 0 || value == 1 || value == 2 || value == 4, "NGL_OPT_TRACE_WAVES takes 0, 1, 2 or 4");
  if (key == NGL_OPT_TRACE_BLOCKS_PER_CU) NGL_REQUIRE(value >= 0 && value <= 64, "NGL_OPT_TRACE_BLOCKS_PER_CU takes 0..64");
  if (key == NGL_OPT_TRACE_PAUSE1 || key == NGL_OPT_TRACE_PAUSE2)
    NGL_REQUIRE(value >= 0 && value <= 4096, "NGL_OPT_TRACE_PAUSE1/2 take 0..4096");
  if (key == NGL_OPT_TRACE_WIDE) NGL_REQUIRE(value == 0 || value == 1, "NGL_OPT_TRACE_WIDE takes 0 or 1");
  if (key == NGL_OPT_COOP_GATHER) NGL_REQUIRE(value == 0 || value == 1, "NGL_OPT_COOP_GATHER takes 0 or 1");
  if (key == NGL_OPT_QUERY_BLOCKS_PER_CU)
    NGL_REQUIRE(value >= 0 && value <= 64, "NGL_OPT_QUERY_BLOCKS_PER_CU takes 0..64");
  ngl::g_options[key].store(value);
  return NGL_OK;
}

int ngl_workspace_bytes(int op, const ngl_model* m, int64_t n, int64_t aux, size_t* bytes) {
  NGL_REQUIRE(bytes != nullptr, "bytes is null");
  NGL_REQUIRE(n >= 0 && aux >= 0, "negative size");
  switch (op) {
    case NGL_OP_TRACE_OCTREE: return ngl_trace_octree_workspace(n, aux, bytes);
    case NGL_OP_SPHERE_TRACE: return ngl_sphere_trace_workspace_rays(n, bytes);
    case NGL_OP_SPHERE_TRACE_LOD: return ngl_sphere_trace_lod_workspace(n, bytes);
    case NGL_OP_TRAIN:
      NGL_REQUIRE(m != nullptr, "NGL_OP_TRAIN needs the model");
      return ngl_train_workspace(m, n, bytes);
    case NGL_OP_SAMPLE_SURFACE: return ngl_sample_surface_workspace(n, bytes);
    case NGL_OP_OCTREE_BUILD_DEVICE:
      NGL_REQUIRE(aux >= 1 && aux <= NGL_MAX_LODS, "aux (num_lods) %lld outside 1..%d", (long long)aux, NGL_MAX_LODS);
      return ngl_octree_build_device_workspace(n, int32_t(aux), bytes);
    case NGL_OP_PACK_DECODERS:
      NGL_REQUIRE(m != nullptr, "NGL_OP_PACK_DECODERS needs the model");
      return ngl_packed_decoder_bytes(m, bytes);
    default: NGL_FAIL(NGL_E_INVALID, "unknown op %d", op);
  }
}

int ngl_get_option(int key, int* value) {
  NGL_REQUIRE(key >= 0 && key < NGL_OPT_COUNT && value != nullptr, "unknown option %d or null value", key);
  *value = ngl::g_options[key].load();
  return NGL_OK;
}

}  // extern "C"
