// Sphere-tracing kernel instantiations for feature width 64, BF16 features.
#include "ngl_trace_impl.h"

namespace ngl {

NGL_TRACE_DEFINE_FT(64, bf16, BF16)

}  // namespace ngl
