// Sphere-tracing kernel instantiations for feature width 8, FP32 features.
#include "ngl_trace_impl.h"

namespace ngl {

NGL_TRACE_DEFINE_FT(8, f32, F32)
int trace_run_analytic(const ngl_model& md, const TraceArgs& A, hipStream_t s) {
  return launch_trace<8, F32, true, true>(md, A, s);
}

}  // namespace ngl
