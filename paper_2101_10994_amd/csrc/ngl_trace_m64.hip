// Sphere-tracing kernel instantiations for feature width 64.
#include "ngl_trace_impl.h"

namespace ngl {

NGL_TRACE_DEFINE(64)

}  // namespace ngl
