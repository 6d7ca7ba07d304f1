// mplpxx_solve_noalloc: the whole solve of mplpxx_create_device +
// mplpxx_iterate + mplpxx_dual_bound + state read-out, for callers that
// cannot allocate device memory.  Its working memory (packed tables,
// messages, mailboxes, slot metadata, reduction buffers) lives in one static
// device array per GPU; the caller passes the inputs and the outputs.  The
// kernels are the ones of the FP32 persistent mailbox engine, so the results
// are bitwise those of the allocating entry points.
// (Paper: Tourani et al., MPLP++, ECCV 2018, Sec. 4 (H), Sec. 6 Alg. 1,
// Eq. (3).)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.h"
#include "host_util.h"
#include "schedule.h"

using namespace mplpxx;

// Working memory of every call on one GPU (each GPU holds its own copy until
// the process ends).  In host code `scratch` names a host-side stand-in, not
// the device array: its device address comes from hipGetSymbolAddress, once
// per device (scratch_base below), and only that address is ever passed on.
static constexpr size_t kScratchBytes = (size_t)MPLPXX_NOALLOC_SCRATCH_MB << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_base[kMaxDevices] = {};

// Device address of this GPU's array (looked up on the first call on the
// device, with that device current).
int scratch_base(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(MPLPXX_EINVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_base[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MPLPXX_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_base[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_base[dev];
  return MPLPXX_OK;
}

// Carves 256-byte aligned regions out of the array.
struct Carver {
  size_t used = 0;
  size_t take(size_t bytes) {
    const size_t at = used;
    used += (bytes + 255) / 256 * 256;
    return at;
  }
};

bool device_memory_of(const void* p, int dev) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) && a.device == dev;
}

// phi in the caller's edge order from phi in slot order
__global__ void __launch_bounds__(256) k_phi_by_edge(const float* __restrict__ phi_slot,
                                                     const int* __restrict__ slot_of_edge, int row,
                                                     float* __restrict__ out) {
  const int e = blockIdx.x;
  const float* src = phi_slot + (size_t)slot_of_edge[e] * row;
  for (int i = threadIdx.x; i < row; i += 256) out[(size_t)e * row + i] = src[i];
}

}  // namespace

extern "C" int mplpxx_solve_noalloc(int32_t n, int32_t L, int64_t m, const int32_t* edges, const float* unaries_dev,
                                    const float* pairwise_dev, int32_t iters, float* U_dev, float* phi_dev,
                                    double* dual, void* hip_stream) {
  if (n < 1) return fail(MPLPXX_EINVAL, "n must be >= 1 (got %d)", n);
  if (L < 1 || L > MPLPXX_MAX_LABELS) return fail(MPLPXX_EINVAL, "L must be in [1, %d] (got %d)", MPLPXX_MAX_LABELS, L);
  if (m < 0 || m > (int64_t)n * (n - 1) / 2) return fail(MPLPXX_EINVAL, "m must be in [0, n(n-1)/2]");
  if (iters < 0) return fail(MPLPXX_EINVAL, "iters must be >= 0");
  if (!unaries_dev || !U_dev) return fail(MPLPXX_EINVAL, "unaries/U is NULL");
  if (m > 0 && (!edges || !pairwise_dev || !phi_dev)) return fail(MPLPXX_EINVAL, "edges/pairwise/phi is NULL");
  const hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (!device_memory_of(unaries_dev, dev) || !device_memory_of(U_dev, dev) ||
      (m > 0 && (!device_memory_of(pairwise_dev, dev) || !device_memory_of(phi_dev, dev))))
    return fail(MPLPXX_EINVAL, "unaries, pairwise, U and phi must be device memory of the current device %d", dev);

  // schedule and slot metadata (host memory only)
  GraphPrep g;
  int rc = prepare_graph(n, (int)m, edges, g, MPLPXX_SCHED_AUTO);
  if (rc != MPLPXX_OK) return rc;
  int max_deg = 0, max_step = 1;
  for (int d : g.deg) max_deg = std::max(max_deg, d);
  for (int s = 0; s < g.S; ++s) max_step = std::max(max_step, g.step_ptr[s + 1] - g.step_ptr[s]);
  if (max_deg >= 65536) return fail(MPLPXX_EINVAL, "node degrees must stay below 65536 (got %d)", max_deg);

  // launch shape of mplpxx_iterate's FP32 persistent engine
  int cus = 0;
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int LT = next_tile(L), NT = 256;
  int G = cus;
  if (max_step > cus) G = std::max(cus, std::min(max_step, max_blocks_per_cu_mb(LT, NT) * cus));
  G = std::max(1, std::min<int>(G, (int)std::max<int64_t>(m, 1)));
  const size_t nL = (size_t)n * L, mLL = (size_t)m * L * L;
  const size_t owned = ((size_t)m + G - 1) / G;
  const size_t phi_lds = owned * 2 * L * sizeof(float);
  const int in_lds = phi_lds <= 96 * 1024 && G <= cus ? 1 : 0;

  Carver c;
  const size_t o_tab = c.take((mLL + kTailPad) * sizeof(float));
  const size_t o_phi = c.take(((size_t)m * 2 * L + kTailPad) * sizeof(float));
  const size_t o_ulo = c.take(nL * sizeof(float));
  const size_t o_mb = c.take(nL * sizeof(unsigned long long));
  const size_t o_slots = c.take((size_t)std::max<int64_t>(m, 1) * sizeof(SlotInfo));
  const size_t o_deg = c.take((size_t)n * sizeof(int));
  const size_t o_err = c.take(8 * sizeof(int));
  const size_t o_sink = c.take((size_t)G * (NT + 128) * sizeof(unsigned long long));
  const size_t o_nptr = c.take(((size_t)n + 1) * sizeof(int));
  const size_t o_inc = c.take((size_t)std::max<int64_t>(2 * m, 1) * sizeof(int));
  const size_t o_nmin = c.take((size_t)n * sizeof(double));
  const size_t o_emin = c.take((size_t)std::max<int64_t>(m, 1) * sizeof(double));
  const size_t o_dual = c.take(sizeof(double));
  const size_t o_se = c.take((size_t)std::max<int64_t>(m, 1) * sizeof(int));
  const size_t o_sf = c.take((size_t)std::max<int64_t>(m, 1) * sizeof(int));
  const size_t o_soe = c.take((size_t)std::max<int64_t>(m, 1) * sizeof(int));
  if (c.used > kScratchBytes)
    return fail(MPLPXX_EINVAL, "the model needs %zu bytes of working memory; mplpxx_solve_noalloc holds at most %zu",
                c.used, kScratchBytes);
  unsigned char* base = nullptr;
  rc = scratch_base(dev, &base);
  if (rc != MPLPXX_OK) return rc;
  float* d_tab = reinterpret_cast<float*>(base + o_tab);
  float* d_phi = reinterpret_cast<float*>(base + o_phi);
  float* d_ulo = reinterpret_cast<float*>(base + o_ulo);
  auto* d_mb = reinterpret_cast<unsigned long long*>(base + o_mb);
  auto* d_slots = reinterpret_cast<SlotInfo*>(base + o_slots);
  int* d_deg = reinterpret_cast<int*>(base + o_deg);
  int* d_err = reinterpret_cast<int*>(base + o_err);
  auto* d_sink = reinterpret_cast<unsigned long long*>(base + o_sink);
  int* d_nptr = reinterpret_cast<int*>(base + o_nptr);
  int* d_inc = reinterpret_cast<int*>(base + o_inc);
  double* d_nmin = reinterpret_cast<double*>(base + o_nmin);
  double* d_emin = reinterpret_cast<double*>(base + o_emin);
  double* d_dual = reinterpret_cast<double*>(base + o_dual);
  int* d_se = reinterpret_cast<int*>(base + o_se);
  int* d_sf = reinterpret_cast<int*>(base + o_sf);
  int* d_soe = reinterpret_cast<int*>(base + o_soe);

  // host metadata: incidence lists (for Eq. 3), table order and orientation
  std::vector<int> node_ptr(n + 1, 0), inc(2 * (size_t)m), se(m), sf(m);
  for (int i = 0; i < (int)m; ++i) {
    node_ptr[g.slots[i].u + 1]++;
    node_ptr[g.slots[i].v + 1]++;
    se[i] = g.order[i];
    sf[i] = g.flip[g.order[i]];
  }
  for (int u = 0; u < n; ++u) node_ptr[u + 1] += node_ptr[u];
  {
    std::vector<int> fillp(node_ptr.begin(), node_ptr.end() - 1);
    for (int i = 0; i < (int)m; ++i) {
      inc[fillp[g.slots[i].u]++] = 2 * i + 0;
      inc[fillp[g.slots[i].v]++] = 2 * i + 1;
    }
  }
  // Everything that must start at zero is cleared by fill kernels: the last
  // call's contents are still in the array.
  HIP_TRY(launch_fill_int(d_err, 0, 8, st));
  HIP_TRY(launch_fill_int(reinterpret_cast<int*>(d_phi), 0, (size_t)m * 2 * L + kTailPad, st));
  HIP_TRY(launch_fill_int(reinterpret_cast<int*>(d_tab + mLL), 0, kTailPad, st));
  HIP_TRY(launch_fill_int(reinterpret_cast<int*>(d_ulo), 0, nL, st));
  HIP_TRY(hipMemcpyAsync(d_nptr, node_ptr.data(), node_ptr.size() * sizeof(int), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_deg, g.deg.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice, st));
  if (m > 0) {
    HIP_TRY(hipMemcpyAsync(d_inc, inc.data(), inc.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_slots, g.slots.data(), (size_t)m * sizeof(SlotInfo), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_se, se.data(), (size_t)m * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_sf, sf.data(), (size_t)m * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_soe, g.slot_of_edge.data(), (size_t)m * sizeof(int), hipMemcpyHostToDevice, st));
  }
  // finiteness of the inputs (the error word doubles as the flag), U = theta_u
  HIP_TRY(launch_check_finite<float>(unaries_dev, nL, d_err + 7, st));
  if (m > 0) HIP_TRY(launch_check_finite<float>(pairwise_dev, mLL, d_err + 7, st));
  HIP_TRY(hipMemcpyAsync(U_dev, unaries_dev, nL * sizeof(float), hipMemcpyDeviceToDevice, st));
  if (m > 0) HIP_TRY(launch_pack_tables<float>(pairwise_dev, d_tab, d_se, d_sf, (int)m, L, st));
  HIP_TRY(hipStreamSynchronize(st));  // (the host vectors above go out of scope)
  int flag = 0;
  HIP_TRY(hipMemcpy(&flag, d_err + 7, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) return fail(MPLPXX_EINVAL, "non-finite (or, in FP32, above 1e18) cost");

  if (m > 0 && iters > 0) {
    HsArgs<float> a{};
    a.tables = d_tab;
    a.phi = d_phi;
    a.U = U_dev;
    a.Ulo = d_ulo;
    a.slots = d_slots;
    a.deg = d_deg;
    a.err = d_err;
    a.sink = d_sink;
    a.L = L;
    a.m = (int)m;
    a.n = n;
    a.spin_limit = 1ll << 22;
    HIP_TRY(launch_mb_init(U_dev, d_ulo, d_mb, nL, st));
    HIP_TRY(launch_persistent_mb(a, d_mb, LT, NT, G, iters, in_lds, in_lds ? phi_lds : 0, st));
    HIP_TRY(launch_mb_fini(U_dev, d_ulo, d_mb, n, L, nullptr, st));
  }
  HIP_TRY(launch_dual<float>(unaries_dev, d_tab, d_phi, d_nptr, d_inc, n, L, (int)m, d_nmin, d_emin, d_dual, st));
  if (m > 0) hipLaunchKernelGGL(k_phi_by_edge, dim3((unsigned)m), dim3(256), 0, st, d_phi, d_soe, 2 * L, phi_dev);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  int err[8] = {0};
  HIP_TRY(hipMemcpy(err, d_err, sizeof(err), hipMemcpyDeviceToHost));
  if (err[0] != 0)
    return fail(err[0], "device wait exceeded its bound (workgroup %d, slot %d, node %d, expected version %d, seen %d)",
                err[1], err[2], err[3], err[4], err[5]);
  if (dual) HIP_TRY(hipMemcpy(dual, d_dual, sizeof(double), hipMemcpyDeviceToHost));
  return MPLPXX_OK;
}
