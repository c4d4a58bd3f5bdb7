// Query and normal kernel instantiations for feature width 16.
#include "ngl_query_impl.h"

namespace ngl {

NGL_QUERY_DEFINE(16)

}  // namespace ngl
