// Streaming-read probe: the HBM read rate that a plain read kernel reaches
// on the current device.  It is the measured ceiling reported beside the
// published 8 TB/s for the bandwidth fractions of the message-passing
// kernels, whose tables are read-only streams (Sec. 4: each pass reads every
// entry of the edge's table once).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "host_util.h"

using namespace mplpxx;

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// Every thread reads 16-byte vectors at a grid stride with nontemporal
// loads (streamed, not kept in the caches), eight loads in flight per
// thread, and folds them into one sum; the sum is stored only if it equals a
// value the (zero-filled) buffer cannot produce, so the loads stay live and
// the probe writes nothing.  (Measured on the MI355X over 4 GiB: 16
// workgroups per compute unit with 8 nontemporal loads in flight read at
// 6.4 TB/s, plain loads at 5.2-5.8 TB/s.)
constexpr int kInFlight = 8;
__global__ void __launch_bounds__(256) k_stream_read(const f4* __restrict__ p, size_t n4, float* __restrict__ out) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  for (; i + (kInFlight - 1) * stride < n4; i += kInFlight * stride) {
    f4 v[kInFlight];
#pragma unroll
    for (int k = 0; k < kInFlight; ++k) v[k] = __builtin_nontemporal_load(p + i + k * stride);
#pragma unroll
    for (int k = 0; k < kInFlight; ++k) acc += v[k];
  }
  for (; i < n4; i += stride) acc += __builtin_nontemporal_load(p + i);
  const float s = (acc.x + acc.y) + (acc.z + acc.w);
  if (s == 1234567.0f) out[0] = s;
}

struct ProbeRes {
  void* buf = nullptr;
  float* out = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~ProbeRes() {
    if (st) (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (buf) (void)hipFree(buf);
    if (out) (void)hipFree(out);
  }
};

}  // namespace

extern "C" int mplpxx_stream_read_probe(int64_t bytes, int32_t reps, double* gbs_median, double* gbs_best) {
  if (!gbs_median) return fail(MPLPXX_EINVAL, "gbs_median must not be NULL");
  if (bytes < ((int64_t)1 << 20) || bytes % 16 != 0)
    return fail(MPLPXX_EINVAL, "bytes must be a multiple of 16 and at least 1 MiB (got %lld)", (long long)bytes);
  if (reps < 1 || reps > 1000) return fail(MPLPXX_EINVAL, "reps must be 1..1000 (got %d)", reps);
  int dev = 0, cus = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  ProbeRes r;
  HIP_TRY(hipStreamCreateWithFlags(&r.st, hipStreamNonBlocking));
  HIP_TRY(hipEventCreate(&r.e0));
  HIP_TRY(hipEventCreate(&r.e1));
  HIP_TRY(hipMalloc(&r.buf, (size_t)bytes));
  HIP_TRY(hipMalloc(reinterpret_cast<void**>(&r.out), sizeof(float)));
  HIP_TRY(hipMemsetAsync(r.buf, 0, (size_t)bytes, r.st));
  const size_t n4 = (size_t)bytes / 16;
  // sixteen 256-thread workgroups per compute unit
  const int grid = std::max(1, cus) * 16;
  std::vector<double> gbs;
  for (int k = 0; k <= reps; ++k) {  // (the first run warms up)
    HIP_TRY(hipEventRecord(r.e0, r.st));
    hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, r.st, static_cast<const f4*>(r.buf), n4, r.out);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(r.e1, r.st));
    HIP_TRY(hipEventSynchronize(r.e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.e0, r.e1));
    if (k > 0 && ms > 0.f) gbs.push_back((double)bytes / (ms * 1e-3) / 1e9);
  }
  if (gbs.empty()) return fail(MPLPXX_EDEVICE, "stream probe: no timed run");
  std::sort(gbs.begin(), gbs.end());
  *gbs_median = gbs.size() % 2 ? gbs[gbs.size() / 2] : 0.5 * (gbs[gbs.size() / 2 - 1] + gbs[gbs.size() / 2]);
  if (gbs_best) *gbs_best = gbs.back();
  return MPLPXX_OK;
}
