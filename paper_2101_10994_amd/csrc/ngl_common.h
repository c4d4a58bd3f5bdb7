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

// Grid of a persistent launch: the blocks of `kern` that can be resident at
// once with `threads` threads and `lds` bytes of dynamic LDS per block, on
// every CU of the current device; with cap > 0 at most `cap` blocks per CU.
// Cached per (device, kernel, threads, lds), so launches with different
// LDS sizes (one or two staged decoders) each get their own occupancy.
int resident_grid(const void* kern, int threads, size_t lds, int cap);

// Checks the structural fields of a model view used by every device call.
int check_model(const ngl_model* m, bool need_features);

inline int din_of(const ngl_model& m) { return m.feat_dim + (m.with_xyz ? 3 : 0); }

// Calls fn_m8 / fn_m16 / fn_m32 / fn_m64 (one translation unit per feature
// width keeps the kernel instantiations of each width apart).
#define NGL_BY_WIDTH(width, fn, ...)                                                   \
  switch (width) {                                                                     \
    case 8: return fn##_m8(__VA_ARGS__);                                               \
    case 16: return fn##_m16(__VA_ARGS__);                                             \
    case 32: return fn##_m32(__VA_ARGS__);                                             \
    case 64: return fn##_m64(__VA_ARGS__);                                             \
    default: NGL_FAIL(NGL_E_UNSUPPORTED, "feat_dim %d not compiled (8, 16, 32, 64)", int(width)); \
  }

}  // namespace ngl
