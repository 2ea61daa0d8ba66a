// Error reporting shared by the host sources of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "peval.h"

namespace peval {

// Records a message for peval_last_error() and returns code.
int fail(int code, const char *fmt, ...);
std::string &last_error_slot();

}  // namespace peval

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return ::peval::fail(e_ == hipErrorOutOfMemory ? PEVAL_ENOMEM : PEVAL_EDEVICE, "%s: %s (%s:%d)", \
                           #expr, hipGetErrorString(e_), __FILE__, __LINE__);                  \
  } while (0)

#define PEVAL_TRY(expr)              \
  do {                               \
    int rc_ = (expr);                \
    if (rc_ != PEVAL_OK) return rc_; \
  } while (0)
