// Sphere-tracing kernel instantiations for feature width 32.
#include "ngl_trace_impl.h"

namespace ngl {

NGL_TRACE_DEFINE(32)

}  // namespace ngl
