// Sphere-tracing kernel instantiations for feature width 16, FP32 features.
#include "ngl_trace_impl.h"

namespace ngl {

NGL_TRACE_DEFINE_FT(16, f32, F32)

}  // namespace ngl
