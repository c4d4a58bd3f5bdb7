// Training forward+backward of Eq. 4 (Sec. 3.3) on gfx950.
#include "ngl_common.h"
#include "ngl_device.h"

extern "C" {

int ngl_train_workspace(const ngl_model* m, int64_t P, size_t* bytes) {
  NGL_REQUIRE(m && bytes && P >= 0, "invalid workspace query");
  *bytes = 0;
  NGL_FAIL(NGL_E_UNSUPPORTED, "training step not available in this build");
}

int ngl_backward_all_lods(const ngl_model*, const float*, int64_t, const float*, float* const*, float* const*,
                          float* const*, float* const*, float*, void*, size_t, void*) {
  NGL_FAIL(NGL_E_UNSUPPORTED, "training step not available in this build");
}

int ngl_train_fwd_bwd(const ngl_model*, const float*, const float*, int64_t, float*, float*, float* const*,
                      float* const*, float* const*, float* const*, float*, void*, size_t, void*) {
  NGL_FAIL(NGL_E_UNSUPPORTED, "training step not available in this build");
}

}  // extern "C"
