// Query and normal kernel instantiations for feature width 64.
#include "ngl_query_impl.h"

namespace ngl {

NGL_QUERY_DEFINE(64)

}  // namespace ngl
