// Host-side helpers shared by the solver and batch runtimes.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "common.h"

namespace mplpxx {

// text of the last failure on the calling thread (mplpxx_last_error)
inline thread_local std::string g_last_error;

// Records the failure's text.  It also takes the HIP runtime's last error,
// which a failed runtime call leaves set: left there, the next launch check
// of a later call (hipGetLastError after a launch) would report it again.
inline int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  (void)hipGetLastError();
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

// Truncated linear parameters (w, tau) per edge: finite, w >= 0, tau >= 0,
// and the costs fl(w * tau), fl(w * d) within the FP32 cost bound.
inline int check_trunc_linear_params(const float* prm, int64_t m) {
  for (int64_t e = 0; e < m; ++e) {
    const float w = prm[2 * e], tau = prm[2 * e + 1];
    if (!(w >= 0.0f && tau >= 0.0f && std::isfinite(w) && std::isfinite(tau)))
      return fail(MPLPXX_EINVAL, "edge %lld: truncated linear costs need finite w >= 0 and tau >= 0", (long long)e);
    if (!(w * tau <= (float)MPLPXX_F32_MAX_COST) || !(w * (float)MPLPXX_MAX_LABELS <= (float)MPLPXX_F32_MAX_COST))
      return fail(MPLPXX_EINVAL, "edge %lld: truncated linear cost above %g", (long long)e, MPLPXX_F32_MAX_COST);
  }
  return MPLPXX_OK;
}

// Truncated quadratic parameters (w, tau) per edge: finite, w >= 0, tau >= 0,
// and every entry fl(w * min(d^2, tau)) within the FP32 cost bound.
inline int check_trunc_quad_params(const float* prm, int64_t m) {
  const float dmax = (float)((MPLPXX_MAX_LABELS - 1) * (MPLPXX_MAX_LABELS - 1));
  for (int64_t e = 0; e < m; ++e) {
    const float w = prm[2 * e], tau = prm[2 * e + 1];
    if (!(w >= 0.0f && tau >= 0.0f && std::isfinite(w) && std::isfinite(tau)))
      return fail(MPLPXX_EINVAL, "edge %lld: truncated quadratic costs need finite w >= 0 and tau >= 0", (long long)e);
    if (!(w * (tau < dmax ? tau : dmax) <= (float)MPLPXX_F32_MAX_COST))
      return fail(MPLPXX_EINVAL, "edge %lld: truncated quadratic cost above %g", (long long)e, MPLPXX_F32_MAX_COST);
  }
  return MPLPXX_OK;
}

// parameter check of a structured cost kind (Potts weights are checked as
// costs by the caller)
inline int check_structured_params(int kind, const float* prm, int64_t m) {
  if (kind == MPLPXX_COST_TRUNC_LINEAR) return check_trunc_linear_params(prm, m);
  if (kind == MPLPXX_COST_TRUNC_QUAD) return check_trunc_quad_params(prm, m);
  return MPLPXX_OK;
}
inline bool known_cost_kind(int kind) {
  return kind == MPLPXX_COST_POTTS || kind == MPLPXX_COST_TRUNC_LINEAR || kind == MPLPXX_COST_TRUNC_QUAD;
}

// smallest register tile (16, 32, 64, 128) holding L labels
inline int next_tile(int L) {
  int lt = 16;
  while (lt < L) lt *= 2;
  return lt;
}

}  // namespace mplpxx
