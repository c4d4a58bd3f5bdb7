// SDF queries (Sec. 3.2, Eq. 2; continuous LOD, Eq. 3) on gfx950.
//
// One lane per point: exact location of the finest needed cell, one descent
// of the octree that yields the voxel of every level, the trilinear corner
// gather summed across levels in registers, then the per-LOD decoder.
#include "ngl_query_impl.h"


extern "C" {

int ngl_query_sdf(const ngl_model* m, const float* x, int64_t P, int32_t lod, float alpha, const float* alpha_pp,
                  float* sdf, uint8_t* valid, int32_t* vox_out, void* stream) {
  int rc = ngl::check_model(m, true);
  if (rc) return rc;
  NGL_REQUIRE(P >= 0, "negative point count");
  NGL_REQUIRE(lod >= 1 && lod <= m->num_lods, "lod %d outside 1..%d", lod, m->num_lods);
  NGL_REQUIRE(alpha >= 0.0f && alpha < 1.0f, "alpha must be in [0,1)");
  NGL_REQUIRE(!(alpha > 0.0f || alpha_pp) || lod < m->num_lods, "blending needs lod < num_lods");
  if (P == 0) return NGL_OK;
  NGL_REQUIRE(x && sdf, "x or sdf is null");
  using namespace ngl;
  NGL_BY_WIDTH(m->feat_dim, query_run, *m, x, P, int(lod), alpha, alpha_pp, sdf, valid, vox_out, (hipStream_t)stream)
}

int ngl_query_sdf_all_lods(const ngl_model* m, const float* x, int64_t P, float* sdf_all, void* stream) {
  int rc = ngl::check_model(m, true);
  if (rc) return rc;
  NGL_REQUIRE(P >= 0, "negative point count");
  if (P == 0) return NGL_OK;
  NGL_REQUIRE(x && sdf_all, "x or sdf_all is null");
  if (m->w_dtype != NGL_F32) NGL_FAIL(NGL_E_UNSUPPORTED, "all-LOD queries need FP32 decoder weights");
  using namespace ngl;
  NGL_BY_WIDTH(m->feat_dim, query_all_run, *m, x, P, sdf_all, (hipStream_t)stream)
}

int ngl_sdf_normals(const ngl_model* m, const float* x, const float* o, const float* d, const float* t_hit,
                    const uint8_t* status, int64_t P, int32_t lod, float alpha, float h, float* normals,
                    void* stream) {
  int rc = ngl::check_model(m, true);
  if (rc) return rc;
  NGL_REQUIRE(P >= 0, "negative point count");
  NGL_REQUIRE(lod >= 1 && lod <= m->num_lods, "lod %d outside 1..%d", lod, m->num_lods);
  NGL_REQUIRE(alpha >= 0.0f && alpha < 1.0f, "alpha must be in [0,1)");
  NGL_REQUIRE(!(alpha > 0.0f) || lod < m->num_lods, "blending needs lod < num_lods");
  NGL_REQUIRE(h > 0.0f, "h must be positive");
  if (P == 0) return NGL_OK;
  NGL_REQUIRE(normals != nullptr, "normals is null");
  NGL_REQUIRE(status ? (o && d && t_hit) : (x != nullptr), "points, or rays with t_hit and status, are required");
  ngl::NormalArgs A{status ? nullptr : x, o, d, t_hit, status, P, int(lod), alpha, h, normals};
  using namespace ngl;
  NGL_BY_WIDTH(m->feat_dim, normals_run, *m, A, (hipStream_t)stream)
}

}  // extern "C"
