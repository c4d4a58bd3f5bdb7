// Host-side helpers shared by the library's translation units: error
// reporting through the C ABI and model validation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "ngl.h"

namespace ngl {

void set_error(const char* fmt, ...);

#define NGL_FAIL(code, ...)        \
  do {                             \
    ::ngl::set_error(__VA_ARGS__); \
    return (code);                 \
  } while (0)

#define NGL_REQUIRE(cond, ...) \
  do {                         \
    if (!(cond)) NGL_FAIL(NGL_E_INVALID, __VA_ARGS__); \
  } while (0)

#define NGL_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      NGL_FAIL(NGL_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));      \
  } while (0)

// Reports the launch status of the preceding kernel(s).
#define NGL_LAUNCHED()                                                         \
  do {                                                                         \
    hipError_t e_ = hipGetLastError();                                         \
    if (e_ != hipSuccess)                                                      \
      NGL_FAIL(NGL_E_HIP, "kernel launch failed: %s", hipGetErrorString(e_));  \
  } while (0)

// Current value of a library option (ngl_set_option).
int option(int key);

// Checks the structural fields of a model view used by every device call.
int check_model(const ngl_model* m, bool need_features);

inline int din_of(const ngl_model& m) { return m.feat_dim + (m.with_xyz ? 3 : 0); }

}  // namespace ngl
