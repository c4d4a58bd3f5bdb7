// Sphere-tracing kernel instantiations for feature width 16.
#include "ngl_trace_impl.h"

namespace ngl {

NGL_TRACE_DEFINE(16)

}  // namespace ngl
