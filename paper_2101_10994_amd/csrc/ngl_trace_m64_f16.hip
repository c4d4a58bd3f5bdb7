// Sphere-tracing kernel instantiations for feature width 64, FP16 features.
#include "ngl_trace_impl.h"

namespace ngl {

NGL_TRACE_DEFINE_FT(64, f16, F16)

}  // namespace ngl
