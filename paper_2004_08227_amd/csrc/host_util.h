// Host-side helpers shared by the solver and batch runtimes.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "common.h"

namespace mplpxx {

// text of the last failure on the calling thread (mplpxx_last_error)
inline thread_local std::string g_last_error;

inline int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_TRY(expr)                                                                                       \
  do {                                                                                                      \
    hipError_t e_ = (expr);                                                                                 \
    if (e_ != hipSuccess) {                                                                                 \
      if (e_ == hipErrorOutOfMemory) return ::mplpxx::fail(MPLPXX_ENOMEM, "%s: %s", #expr, hipGetErrorString(e_)); \
      return ::mplpxx::fail(MPLPXX_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));                       \
    }                                                                                                       \
  } while (0)

// smallest register tile (16, 32, 64, 128) holding L labels
inline int next_tile(int L) {
  int lt = 16;
  while (lt < L) lt *= 2;
  return lt;
}

}  // namespace mplpxx
