// Query and normal kernel instantiations for feature width 32.
#include "ngl_query_impl.h"

namespace ngl {

NGL_QUERY_DEFINE(32)

}  // namespace ngl
