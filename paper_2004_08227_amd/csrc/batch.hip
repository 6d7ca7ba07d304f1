// Batched MPLP++: many independent FP32 models solved by one persistent
// launch.  Each workgroup runs a list of tasks; a task is "the slots first,
// first+stride, ... of model b for all iterations", executed by the mailbox
// engine (device_common.h).  A large model is split over a team of
// workgroups (stride = team size, each member's first task, so the whole team
// runs at once); small models are packed, one after another, into single
// workgroups.  A model that runs on one workgroup and whose unaries fit in
// LDS keeps them there for the launch (no mailbox traffic, no waiting: the
// workgroup orders its own updates with barriers).  The host plans the tasks
// (batch.cpp).
//
// Two kernels run such task lists: k_batch, whose workgroups run the mailbox
// engine (one update at a time, any L), and k_wbatch, whose waves each run
// whole updates on the wave engine (L <= 64, many updates in flight per
// compute unit).
#include "device_common.h"
#include "wave_engine.h"
#include "wave_batch.h"

namespace mplpxx {

template <int NT, int MAXLT> union BatchSmem {
  SmemMB<16, NT> s16;
  SmemMB<32, NT> s32;
  SmemMB<64, NT> s64;
  SmemMB<(MAXLT > 64 ? 128 : 64), NT> s128;
};

template <int LT, int NT>
__device__ __forceinline__ bool run_task(const BatchArgs& b, const BatchModel& md, const BatchTask& task,
                                         SmemMB<LT, NT>& sm, int iters, unsigned char* dyn) {
  if (threadIdx.x == 0) sm.abort_flag = 0;
  MbView v{b.tables + uni(md.table_off), b.phi + uni(md.phi_off), b.mb + uni(md.u_off), b.slots + uni(md.slot_off),
           b.deg + uni(md.node_off), nullptr, nullptr, nullptr, uni(md.L), uni(md.m), uni(md.n), nullptr, nullptr,
           b.sink + (size_t)blockIdx.x * (NT + 128)};
  // messages prefetched with the tables when the task owns at least
  // DEPTH + 2 slots
  constexpr int kDepth = LT <= 64 ? 2 : 1;
  const int owned = (md.m - task.first + task.stride - 1) / task.stride;
  const bool far = owned >= kDepth + 2;
  if (!task.lds) {
    __syncthreads();
    return far ? mb_run<LT, NT, false, false, false, false, true, kDepth>(v, task.first, task.stride, iters, sm, nullptr,
                                                                  b.spin_limit, b.err)
               : mb_run<LT, NT, false, false, false, false, false, kDepth>(v, task.first, task.stride, iters, sm, nullptr,
                                                                   b.spin_limit, b.err);
  }
  // the model's unaries into LDS (hi, and lo as bf16 bits), run, and back
  const int nl = md.n * md.L;
  v.lds_hi = reinterpret_cast<float*>(dyn);
  v.lds_lo = reinterpret_cast<unsigned short*>(dyn + lds_lo_offset(md.n, md.L));
  for (int i = threadIdx.x; i < nl; i += blockDim.x) {
    const unsigned long long w = v.mb[i];
    v.lds_hi[i] = mb_hi(w);
    v.lds_lo[i] = (unsigned short)(__float_as_uint(mb_lo(w)) >> 16);
  }
  __syncthreads();
  const bool ok = far ? mb_run<LT, NT, false, false, false, true, true, kDepth>(v, 0, 1, iters, sm, nullptr, b.spin_limit, b.err)
                     : mb_run<LT, NT, false, false, false, true, false, kDepth>(v, 0, 1, iters, sm, nullptr, b.spin_limit,
                                                                       b.err);
  __syncthreads();
  for (int i = threadIdx.x; i < nl; i += blockDim.x)
    v.mb[i] = mb_pack(v.lds_hi[i], __uint_as_float((unsigned)v.lds_lo[i] << 16), 0u);
  return ok;
}

// A workgroup runs its own tasks (the planner gives each team member its
// share of a team model), then takes single-workgroup tasks from the shared
// queue, one at a time in queue order (longest first), until it is empty:
// whichever workgroup is free next runs the next one, so the load balances
// itself whatever the planner's time estimates.  Sets [t, end) to the next
// task; false when the queue is empty.
__device__ __forceinline__ bool next_queued(const BatchArgs& b, int& s_q, int& t, int& end) {
  if (threadIdx.x == 0) s_q = atomicAdd(b.ticket + 1, 1);
  __syncthreads();
  const int q = s_q;
  __syncthreads();  // every thread has read s_q before it is written again
  if (q >= b.qlen) return false;
  t = b.qbegin + q;
  end = t + 1;
  return true;
}

// at least two waves per SIMD: one 6-wave workgroup per compute unit, with
// registers for every tile size without spills
template <int NT, int MAXLT>
__global__ void __launch_bounds__(NT + 128, 2) k_batch(BatchArgs b, int iters) {
  __shared__ BatchSmem<NT, MAXLT> sm;
  __shared__ int s_wg, s_q;
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  // logical workgroup = order of arrival: workgroups that hold a ticket have
  // started, so the first tickets (where the planner puts every team) run
  // together whatever order the hardware dispatches in
  if (threadIdx.x == 0) {
    s_wg = atomicAdd(b.ticket, 1);
    b.wg_time[2 * s_wg] = wall_clock64();
  }
  __syncthreads();
  const int wg = s_wg;
  int t = b.task_ptr[wg], end = b.task_ptr[wg + 1];
  for (;;) {
    if (t == end && !next_queued(b, s_q, t, end)) break;
    const BatchTask task = b.tasks[t];
    const BatchModel md = b.models[task.model];
    bool ok = true;
    if (md.lt == 16) ok = run_task<16, NT>(b, md, task, sm.s16, iters, dyn_lds);
    else if (md.lt == 32) ok = run_task<32, NT>(b, md, task, sm.s32, iters, dyn_lds);
    else if (md.lt == 64 || MAXLT == 64) ok = run_task<64, NT>(b, md, task, sm.s64, iters, dyn_lds);
    else ok = run_task<(MAXLT > 64 ? 128 : 64), NT>(b, md, task, sm.s128, iters, dyn_lds);
    if (!ok) break;
    __syncthreads();  // shared memory is reused by the next task
    ++t;
  }
  if (threadIdx.x == 0) b.wg_time[2 * wg + 1] = wall_clock64();
}

static const void* batch_kernel(int max_lt) {
  return max_lt <= 64 ? (const void*)k_batch<256, 64> : (const void*)k_batch<256, 128>;
}

hipError_t launch_batch(const BatchArgs& b, int max_lt, int grid, int iters, size_t dyn_lds, hipStream_t st) {
  if (max_lt <= 64)
    hipLaunchKernelGGL((k_batch<256, 64>), dim3(grid), dim3(256 + 128), dyn_lds, st, b, iters);
  else
    hipLaunchKernelGGL((k_batch<256, 128>), dim3(grid), dim3(256 + 128), dyn_lds, st, b, iters);
  return hipGetLastError();
}

int batch_blocks_per_cu(int max_lt, size_t dyn_lds) {
  int nb = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel(max_lt), 256 + 128, dyn_lds);
  return e == hipSuccess ? nb : 0;
}

// largest dynamic LDS a workgroup of the batched kernel can have (raises the
// kernel's limit to it)
size_t batch_lds_limit(int max_lt) {
  int dev = 0, per_block = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
  hipFuncAttributes fa{};
  if (hipFuncGetAttributes(&fa, batch_kernel(max_lt)) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  if ((size_t)per_block <= fa.sharedSizeBytes) return 0;
  const size_t limit = (size_t)per_block - fa.sharedSizeBytes;
  if (hipFuncSetAttribute(batch_kernel(max_lt), hipFuncAttributeMaxDynamicSharedMemorySize, (int)limit) != hipSuccess) {
    (void)hipGetLastError();  // (not left for a later launch check)
    return 0;
  }
  return limit;
}

// ---------------------------------------------------------------------------
// The batched launch on the wave engine (wave_engine.h): every wave of a
// workgroup is a worker.  Task (first, stride) of a team of `stride`
// workgroups gives wave w of the member the slots first + w stride,
// first + (w + NW) stride, ...; a whole model on one workgroup (stride 1)
// deals its slots to the NW waves round-robin.
// ---------------------------------------------------------------------------
// twelve workers per compute unit: one 12-wave workgroup at three waves per
// SIMD (168 registers hold the 64-label tile and its working vectors).
// Measured on the batched pose mix, this beats 8 waves at two per SIMD and
// two workgroups per compute unit (6 waves each, or 8 at four per SIMD,
// which spills the 64-label path).
#ifndef MPLPXX_WV_WAVES
#define MPLPXX_WV_WAVES 12
#endif
#ifndef MPLPXX_WV_WPE
#define MPLPXX_WV_WPE 3
#endif
constexpr int kWvWaves = MPLPXX_WV_WAVES;
constexpr int kWvSink = 192;  // scratch words per wave

template <int LT, int KIND = kCostDense>
__device__ __forceinline__ void wv_task(const BatchArgs& b, const BatchModel& md, const BatchTask& task,
                                        WvScratch& scr, int iters, unsigned char* dyn, int* abort) {
  const int wave = threadIdx.x >> 6;
  WvView v{b.tables + uni(md.table_off), b.phi + uni(md.phi_off), b.mb + uni(md.u_off), b.slots + uni(md.slot_off),
           uni(md.L), uni(md.m), uni(md.n), nullptr, nullptr, nullptr,
           b.sink + ((size_t)blockIdx.x * kWvWaves + wave) * kWvSink};
  const int first = uni(task.first + wave * task.stride);
  const int stride = uni(task.stride * kWvWaves);
  const int owned = first < md.m ? (md.m - first + stride - 1) / stride : 0;
  const bool far = owned >= 2;
  if (!task.lds) {
    if (far) (void)wv_run<LT, false, true, KIND>(v, first, stride, iters, scr, b.spin_limit, b.err, abort);
    else (void)wv_run<LT, false, false, KIND>(v, first, stride, iters, scr, b.spin_limit, b.err, abort);
    return;
  }
  // the model's unaries and update counters into LDS, run, and back
  const int nl = md.n * md.L;
  v.lds_hi = reinterpret_cast<float*>(dyn);
  v.lds_lo = reinterpret_cast<unsigned short*>(dyn + lds_lo_offset(md.n, md.L));
  v.lds_ver = reinterpret_cast<int*>(dyn + wv_ver_offset(md.n, md.L));
  for (int i = threadIdx.x; i < nl; i += blockDim.x) {
    const unsigned long long w = v.mb[i];
    v.lds_hi[i] = mb_hi(w);
    v.lds_lo[i] = (unsigned short)(__float_as_uint(mb_lo(w)) >> 16);
  }
  for (int i = threadIdx.x; i < md.n; i += blockDim.x) v.lds_ver[i] = 0;
  __syncthreads();
  if (far) (void)wv_run<LT, true, true, KIND>(v, first, stride, iters, scr, b.spin_limit, b.err, abort);
  else (void)wv_run<LT, true, false, KIND>(v, first, stride, iters, scr, b.spin_limit, b.err, abort);
  __syncthreads();
  for (int i = threadIdx.x; i < nl; i += blockDim.x)
    v.mb[i] = mb_pack(v.lds_hi[i], __uint_as_float((unsigned)v.lds_lo[i] << 16), 0u);
}

// KIND: a batch of models with structured costs (mplpxx_batch_create_potts,
// mplpxx_batch_create_structured); separate instances, so that the dense
// kernel keeps its own register allocation
template <int KIND>
__global__ void __launch_bounds__(kWvWaves * 64, MPLPXX_WV_WPE) k_wbatch(BatchArgs b, int iters) {
  __shared__ WvScratch scr[kWvWaves];
  __shared__ int s_wg, s_abort, s_q;
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  if (threadIdx.x == 0) {
    s_wg = atomicAdd(b.ticket, 1);
    s_abort = 0;
    b.wg_time[2 * s_wg] = wall_clock64();
  }
  __syncthreads();
  const int wg = s_wg;
  WvScratch& my = scr[threadIdx.x >> 6];
  int t = b.task_ptr[wg], end = b.task_ptr[wg + 1];
  for (;;) {
    if (t == end && !next_queued(b, s_q, t, end)) break;
    const BatchTask task = b.tasks[t];
    const BatchModel& md = b.models[task.model];
    if constexpr (KIND != kCostDense) {
      wv_task<64, KIND>(b, md, task, my, iters, dyn_lds, &s_abort);
    } else {
      if (md.lt == 16) wv_task<16>(b, md, task, my, iters, dyn_lds, &s_abort);
      else if (md.lt == 32) wv_task<32>(b, md, task, my, iters, dyn_lds, &s_abort);
      else wv_task<64>(b, md, task, my, iters, dyn_lds, &s_abort);
    }
    __syncthreads();  // LDS is reused by the next task; every wave has stopped
    if (*(volatile int*)&s_abort) break;
    ++t;
  }
  if (threadIdx.x == 0) b.wg_time[2 * wg + 1] = wall_clock64();
}

int wbatch_waves() { return kWvWaves; }
size_t wbatch_sink_words() { return (size_t)kWvWaves * kWvSink; }

static const void* wbatch_kernel(int kind) {
  return kind == MPLPXX_COST_TRUNC_QUAD     ? (const void*)k_wbatch<MPLPXX_COST_TRUNC_QUAD>
         : kind == MPLPXX_COST_TRUNC_LINEAR ? (const void*)k_wbatch<MPLPXX_COST_TRUNC_LINEAR>
         : kind == MPLPXX_COST_POTTS      ? (const void*)k_wbatch<MPLPXX_COST_POTTS>
                                          : (const void*)k_wbatch<kCostDense>;
}

hipError_t launch_wbatch(const BatchArgs& b, int grid, int iters, size_t dyn_lds, int kind, hipStream_t st) {
  if (kind == MPLPXX_COST_TRUNC_QUAD)
    hipLaunchKernelGGL(k_wbatch<MPLPXX_COST_TRUNC_QUAD>, dim3(grid), dim3(kWvWaves * 64), dyn_lds, st, b, iters);
  else if (kind == MPLPXX_COST_TRUNC_LINEAR)
    hipLaunchKernelGGL(k_wbatch<MPLPXX_COST_TRUNC_LINEAR>, dim3(grid), dim3(kWvWaves * 64), dyn_lds, st, b, iters);
  else if (kind == MPLPXX_COST_POTTS)
    hipLaunchKernelGGL(k_wbatch<MPLPXX_COST_POTTS>, dim3(grid), dim3(kWvWaves * 64), dyn_lds, st, b, iters);
  else hipLaunchKernelGGL(k_wbatch<kCostDense>, dim3(grid), dim3(kWvWaves * 64), dyn_lds, st, b, iters);
  return hipGetLastError();
}

int wbatch_blocks_per_cu(size_t dyn_lds, int kind) {
  int nb = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, wbatch_kernel(kind), kWvWaves * 64, dyn_lds);
  return e == hipSuccess ? nb : 0;
}

// static LDS of the wave kernel, and the largest dynamic LDS it can have
// (raises the kernel's limit to it)
size_t wbatch_lds_limit(size_t* static_bytes, int kind) {
  int dev = 0, per_block = 0;
  if (static_bytes) *static_bytes = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
  hipFuncAttributes fa{};
  if (hipFuncGetAttributes(&fa, wbatch_kernel(kind)) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  if (static_bytes) *static_bytes = fa.sharedSizeBytes;
  if ((size_t)per_block <= fa.sharedSizeBytes) return 0;
  const size_t limit = (size_t)per_block - fa.sharedSizeBytes;
  if (hipFuncSetAttribute(wbatch_kernel(kind), hipFuncAttributeMaxDynamicSharedMemorySize, (int)limit) != hipSuccess) {
    (void)hipGetLastError();  // (not left for a later launch check)
    return 0;
  }
  return limit;
}

// mailbox <- (U, Ulo, version 0) and back
__global__ void k_u_to_mb(const float* __restrict__ U, const float* __restrict__ Ulo,
                          unsigned long long* __restrict__ mb, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    mb[i] = mb_pack(U[i], Ulo[i], 0u);
}
__global__ void k_mb_to_u(float* __restrict__ U, float* __restrict__ Ulo, const unsigned long long* __restrict__ mb,
                          size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const unsigned long long w = mb[i];
    U[i] = mb_hi(w);
    Ulo[i] = mb_lo(w);
  }
}
static unsigned blocks_for(size_t count) {
  size_t b = (count + 255) / 256;
  return (unsigned)(b > 2048 ? 2048 : (b == 0 ? 1 : b));
}
hipError_t launch_u_to_mb(const float* U, const float* Ulo, unsigned long long* mb, size_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_u_to_mb, dim3(blocks_for(count)), dim3(256), 0, st, U, Ulo, mb, count);
  return hipGetLastError();
}
hipError_t launch_mb_to_u(float* U, float* Ulo, const unsigned long long* mb, size_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_mb_to_u, dim3(blocks_for(count)), dim3(256), 0, st, U, Ulo, mb, count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-model dual bounds (Eq. 3) of a batch, FP64, fixed-order reductions.
// ---------------------------------------------------------------------------
template <int NT, bool kMin>
__device__ __forceinline__ double breduce(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s >= 1; s >>= 1) {
    if (tid < s) sh[tid] = kMin ? __builtin_fmin(sh[tid], sh[tid + s]) : sh[tid] + sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(128) k_batch_node_terms(const float* __restrict__ unaries, const float* __restrict__ phi,
                                                          const BatchModel* __restrict__ models,
                                                          const int* __restrict__ node_model,
                                                          const int* __restrict__ node_ptr, const int* __restrict__ inc,
                                                          double* __restrict__ node_min) {
  __shared__ double sh[128];
  const int g = blockIdx.x;
  const BatchModel md = models[node_model[g]];
  const int u = g - md.node_off;
  const int L = md.L;
  const int s = threadIdx.x;
  double acc = __builtin_inf();
  if (s < L) {
    acc = (double)unaries[md.u_off + (size_t)u * L + s];
    const int* np = node_ptr + md.csr_off;
    for (int k = np[u]; k < np[u + 1]; ++k) {
      const int code = inc[md.inc_off + k];
      acc += (double)phi[md.phi_off + (size_t)(code >> 1) * 2 * L + (size_t)(code & 1) * L + s];
    }
  }
  const double mn = breduce<128, true>(acc, sh);
  if (s == 0) node_min[g] = mn;
}

__global__ void __launch_bounds__(256) k_batch_edge_terms(const float* __restrict__ tables, const float* __restrict__ phi,
                                                          const BatchModel* __restrict__ models,
                                                          const int* __restrict__ slot_model,
                                                          double* __restrict__ edge_min) {
  __shared__ double sh[256];
  const int g = blockIdx.x;
  const BatchModel md = models[slot_model[g]];
  const int slot = g - md.slot_off;
  const int L = md.L;
  // (structured costs: the expanded table from the slot's parameters)
  const float* tab = tables + md.table_off + (md.potts ? (size_t)slot * cost_params(md.potts) : (size_t)slot * L * L);
  const float* p0 = phi + md.phi_off + (size_t)slot * 2 * L;
  const float* p1 = p0 + L;
  double mn = __builtin_inf();
  for (int i = threadIdx.x; i < L * L; i += 256) {
    const int s = i / L, t = i - s * L;
    const float th = md.potts ? structured_cost(md.potts, tab, s, t) : tab[i];
    mn = __builtin_fmin(mn, (double)th - (double)p0[s] - (double)p1[t]);
  }
  mn = breduce<256, true>(mn, sh);
  if (threadIdx.x == 0) edge_min[g] = mn;
}

__global__ void __launch_bounds__(256) k_batch_sum(const BatchModel* __restrict__ models,
                                                  const double* __restrict__ node_min,
                                                  const double* __restrict__ edge_min, double* __restrict__ out) {
  __shared__ double sh[256];
  const BatchModel md = models[blockIdx.x];
  double acc = 0.0;
  for (int i = threadIdx.x; i < md.n; i += 256) acc += node_min[md.node_off + i];
  for (int i = threadIdx.x; i < md.m; i += 256) acc += edge_min[md.slot_off + i];
  acc = breduce<256, false>(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

hipError_t launch_batch_dual(const float* unaries, const float* tables, const float* phi, const BatchModel* models,
                             const int* node_model, const int* slot_model, const int* node_ptr, const int* inc,
                             int total_nodes, int total_slots, int count, double* node_min, double* edge_min,
                             double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_node_terms, dim3(total_nodes), dim3(128), 0, st, unaries, phi, models, node_model,
                     node_ptr, inc, node_min);
  if (total_slots > 0)
    hipLaunchKernelGGL(k_batch_edge_terms, dim3(total_slots), dim3(256), 0, st, tables, phi, models, slot_model,
                       edge_min);
  hipLaunchKernelGGL(k_batch_sum, dim3(count), dim3(256), 0, st, models, node_min, edge_min, out);
  return hipGetLastError();
}

}  // namespace mplpxx
