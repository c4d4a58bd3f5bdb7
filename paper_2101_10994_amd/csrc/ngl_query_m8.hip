// Query and normal kernel instantiations for feature width 8.
#include "ngl_query_impl.h"

namespace ngl {

NGL_QUERY_DEFINE(8)

}  // namespace ngl
