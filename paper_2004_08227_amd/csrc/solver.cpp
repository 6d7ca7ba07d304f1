// Host runtime of the MPLP++ solver library: the C ABI of include/mplpxx.h.
//
// create  -> validate, orient edges u < v (Sec. 3 "Notation"), build the
//            schedule (Alg. 1, Sec. 6), pack the tables in schedule order,
//            copy everything to device memory, start from phi = 0;
// iterate -> BCA-iterations (Sec. 5) with the handshake update (H) of Sec. 4
//            on the device, one of two engines:
//              step        one kernel per matching (kernel boundaries are the
//                          paper's barrier between matchings);
//              persistent  one cooperative kernel per call; a workgroup waits
//                          only for the two nodes of its next edge;
// dual    -> Eq. (3) recomputed from costs and messages in FP64;
// decode  -> Eq. (5) and the energy of Eq. (1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "schedule.h"

using namespace mplpxx;

#include "host_util.h"

namespace {

// (64: one compute wave, FP32 mailbox engine at up to 32 labels; the other
// engines then run 256)
bool valid_threads(int LT, int NT) {
  if (NT == 64) return LT <= 32;
  if (NT != 256 && NT != 512 && NT != 1024) return false;
  return NT <= 16 * LT;
}

template <typename T> T* dalloc(size_t count, hipError_t* err) {
  void* p = nullptr;
  *err = hipMalloc(&p, count * sizeof(T) > 0 ? count * sizeof(T) : 16);
  return static_cast<T*>(p);
}

}  // namespace

struct mplpxx_solver {
  int n = 0, L = 0, m = 0, dtype = 0, S = 0;
  size_t esz = 4;
  std::vector<int> step_ptr, order;      // schedule (edge ids of the input list)
  std::vector<int> slot_of_edge;         // inverse of order
  std::vector<SlotInfo> slots;
  std::vector<int> flip;                 // per input edge: 1 if given as (v, u)
  std::vector<int> deg;
  // device
  void* d_tables = nullptr;
  void* d_phi = nullptr;
  void* d_U = nullptr;
  float* d_Ulo = nullptr;                // FP32: bf16 corrections of U (compensated sums)
  void* d_unaries = nullptr;
  SlotInfo* d_slots = nullptr;
  int* d_deg = nullptr;
  int* d_ver = nullptr;
  int* d_err = nullptr;
  int* d_node_ptr = nullptr;
  int* d_inc = nullptr;
  double* d_node_min = nullptr;
  double* d_edge_min = nullptr;
  double* d_scalar = nullptr;
  int* d_labels = nullptr;
  double* d_trace_nodes = nullptr;
  double* d_trace_out = nullptr;
  float* d_trace_e = nullptr;            // FP32: [cap][m][8] edge terms of the trace
  int trace_cap = 0;
  unsigned long long* d_mb = nullptr;    // FP32 mailboxes of the persistent engine
  unsigned long long* d_sink = nullptr;  // scratch words of its workgroups
  size_t sink_words = 0;
  long long* d_stamps = nullptr;         // per-slot timestamps (profiling option)
  bool profile = false;
  int wallclock_khz = 0;
  // adjoint of K unrolled iterations
  int adj_K = 0, adj_every = 0, adj_nck = 0;
  bool adj_ready = false;
  long long adj_iter_mark = -1;           // `iterations` right after the forward
  void* d_ck_U = nullptr;                 // [nck + 1][n][L] (last = final state)
  float* d_ck_Ulo = nullptr;              // FP32: [nck + 1][n][L] corrections
  void* d_ck_phi = nullptr;               // [nck + 1][m][2][L]
  unsigned char* d_rec = nullptr;         // [every][m][3][L]
  void* d_Ub = nullptr;                   // [n][L]
  void* d_pb = nullptr;                   // [m][2][L]
  void* d_thb = nullptr;                  // [m][L][L]
  // persistent FP64 adjoint (L <= 64): mailboxes [2][n][L][2] (unaries of
  // the forward, then their adjoints), and the reverse steps' scatter
  // vectors [every][m][3][L]; d_rec then holds two segments of records
  unsigned long long* d_mb64 = nullptr;
  double* d_contrib = nullptr;
  size_t adj_bytes = 0;                   // device bytes of the adjoint buffers above
  int* d_slot_of_edge = nullptr;          // [m]
  int* d_edge_flip = nullptr;             // [m]
  int adjoint_f64 = 1;                    // FP32 handles: differentiate an FP64 run
  mplpxx_solver* shadow = nullptr;        // the FP64 twin for that (same graph, widened costs)
  // execution
  hipStream_t user_stream = nullptr;
  hipStream_t own_stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int engine_opt = ENGINE_AUTO;
  int rule = MPLPXX_RULE_H;  // BCA-update (Sec. 4)
  int sched = MPLPXX_SCHED_AUTO;  // schedule kind of Alg. 1
  int threads_opt = 0;
  int potts = 0;             // structured cost kind (MPLPXX_COST_*): d_tables holds its parameters per slot
  int grid_opt = 0;
  int phi_opt = 0;       // FP32 persistent engine: 0 auto, 1 messages in LDS when they fit, 2 in global memory
  int prefetch_opt = 0;  // FP32 persistent engine: tables loaded 1 or 2 steps ahead (0 auto)
  long long spin_limit = 1ll << 22;
  int num_cus = 0;
  long long iterations = 0;
  double last_ms = 0.0;
  bool timed = false;

  hipStream_t stream() const { return user_stream ? user_stream : own_stream; }
  int LT() const { return next_tile(L); }
  // Structured costs run either one compute wave in label order (potts_mb.h;
  // threads 64) or the dense engine's four compute waves with each tile
  // formed from the slot's parameters (threads 256).  Default: the formed
  // tiles for the truncated kinds and for Potts costs up to 32 labels.
  bool gen_tiles() const {
    if (!potts) return false;
    if (threads_opt) return threads_opt == 256;
    return potts != MPLPXX_COST_POTTS || L <= 32;
  }
  int NT() const {
    if (potts) {
      if (!gen_tiles()) return 64;  // label order: one compute wave
      if (threads_opt) return 256;
      // formed tiles: one compute wave at 16 labels when a matching has
      // more edges than there are compute units, as for tables below
      return LT() == 16 && max_step > num_cus ? 64 : 256;
    }
    // default: one compute wave at 16 labels when a matching has more edges
    // than there are compute units (several workgroups then share a compute
    // unit: sparse graphs of 1,000 nodes run 3-5 % faster per iteration, a
    // complete graph of 200 nodes within 0.4 %); four waves otherwise
    const bool one_wave = dtype == MPLPXX_F32 && engine() == ENGINE_PERSISTENT;
    int nt = threads_opt ? threads_opt : (one_wave && LT() == 16 && max_step > num_cus ? 64 : 256);
    if (!valid_threads(LT(), nt)) nt = 256;
    if (nt == 64 && !one_wave) nt = 256;
    // the FP32 persistent engine adds two sync waves: at most 512 + 128 threads
    if (dtype == MPLPXX_F32 && engine() == ENGINE_PERSISTENT && nt > 512) nt = 512;
    return nt;
  }
  int max_deg = 0;
  int max_step = 1;  // edges of the largest matching
  int engine() const {
    // FP32 mailboxes carry 16-bit versions: degrees must stay below 2^16
    if (dtype == MPLPXX_F32 && max_deg >= 65536) return ENGINE_STEP;
    if (rule != MPLPXX_RULE_H) return ENGINE_STEP;  // (M), (U): per-matching engine (but see below)
    if (engine_opt == ENGINE_STEP || engine_opt == ENGINE_PERSISTENT) return engine_opt;
    return ENGINE_PERSISTENT;
  }
  // (M) and (U) on FP32 dense handles also run on the mailbox engine (four
  // compute waves) when no trace is asked for; traces use the per-matching
  // engine, with the same bits
  bool rule_mailbox() const {
    return rule != MPLPXX_RULE_H && dtype == MPLPXX_F32 && !potts && max_deg < 65536 && engine_opt != ENGINE_STEP &&
           (threads_opt == 0 || threads_opt == 256);
  }
  // FP32 mailbox engine: one workgroup per compute unit, or, when a matching
  // has more edges than there are compute units, one workgroup per edge of
  // the largest matching as far as they fit (each workgroup then runs about
  // one update per matching instead of several one after another)
  bool mb_engine() const { return dtype == MPLPXX_F32 && engine() == ENGINE_PERSISTENT; }
  int grid() const {
    int g = grid_opt > 0 ? grid_opt : num_cus;
    if (grid_opt == 0 && (mb_engine() || rule_mailbox()) && max_step > num_cus)
      g = std::max(num_cus, std::min(max_step, (potts && !gen_tiles() ? max_blocks_per_cu_mb_potts()
                                                                       : max_blocks_per_cu_mb(LT(), NT())) *
                                                     num_cus));
    if (g > m) g = m;
    if (g < 1) g = 1;
    return g;
  }
};

namespace {

void free_all(mplpxx_solver* h) {
  void* ptrs[] = {h->d_tables, h->d_phi, h->d_U, h->d_Ulo, h->d_ck_Ulo, h->d_unaries, h->d_slots, h->d_deg, h->d_ver, h->d_err,
                  h->d_node_ptr, h->d_inc, h->d_node_min, h->d_edge_min, h->d_scalar, h->d_labels,
                  h->d_trace_nodes, h->d_trace_out, h->d_trace_e, h->d_mb, h->d_sink, h->d_stamps, h->d_ck_U, h->d_ck_phi,
                  h->d_rec, h->d_Ub, h->d_pb, h->d_thb, h->d_slot_of_edge, h->d_edge_flip, h->d_mb64, h->d_contrib};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
}

// FP32 values must be finite with |x| <= MPLPXX_F32_MAX_COST (the FP32 engines
// pad tables with 2^126 and rely on every real value staying far below it)
bool finite_host(const void* p, size_t count, int dtype) {
  if (dtype == MPLPXX_F32) {
    const float* f = static_cast<const float*>(p);
    for (size_t i = 0; i < count; ++i)
      if (!(std::fabs(f[i]) <= (float)MPLPXX_F32_MAX_COST)) return false;
  } else {
    const double* f = static_cast<const double*>(p);
    for (size_t i = 0; i < count; ++i)
      if (!std::isfinite(f[i])) return false;
  }
  return true;
}

// Validates the graph and fills orientation, schedule, slot metadata.
int prepare_solver_graph(mplpxx_solver* h, const int32_t* edges) {
  GraphPrep g;
  const int rc = prepare_graph(h->n, h->m, edges, g, h->sched);
  if (rc != MPLPXX_OK) return rc;
  h->S = g.S;
  h->step_ptr.swap(g.step_ptr);
  h->order.swap(g.order);
  h->slot_of_edge.swap(g.slot_of_edge);
  h->slots.swap(g.slots);
  h->flip.swap(g.flip);
  h->deg.swap(g.deg);
  h->max_deg = 0;
  for (int d : h->deg) h->max_deg = std::max(h->max_deg, d);
  h->max_step = 1;
  for (int s = 0; s < h->S; ++s) h->max_step = std::max(h->max_step, h->step_ptr[s + 1] - h->step_ptr[s]);
  return MPLPXX_OK;
}

// True when p is device memory of device dev (a host or foreign pointer
// handed to a kernel would fault the GPU instead of failing the call).
bool is_device_memory(const void* p, int dev) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) && a.device == dev;
}

int create_impl(int32_t n, int32_t L, int64_t m, const int32_t* edges, const void* unaries, const void* pairwise,
                int32_t dtype, bool device_costs, hipStream_t copy_stream, mplpxx_solver** out,
                int32_t sched = MPLPXX_SCHED_AUTO, int potts = 0) {
  if (!out) return fail(MPLPXX_EINVAL, "out is NULL");
  *out = nullptr;
  if (dtype != MPLPXX_F32 && dtype != MPLPXX_F64) return fail(MPLPXX_EINVAL, "unknown dtype %d", dtype);
  if (n < 1) return fail(MPLPXX_EINVAL, "n must be >= 1 (got %d)", n);
  if (L < 1 || L > MPLPXX_MAX_LABELS) return fail(MPLPXX_EINVAL, "L must be in [1, %d] (got %d)", MPLPXX_MAX_LABELS, L);
  if (m < 0 || m > (int64_t)n * (n - 1) / 2) return fail(MPLPXX_EINVAL, "m must be in [0, n(n-1)/2] (got %lld)", (long long)m);
  if (m > 0x3fffffff) return fail(MPLPXX_EINVAL, "too many edges");
  if (!unaries) return fail(MPLPXX_EINVAL, "unaries is NULL");
  if (sched != MPLPXX_SCHED_AUTO && sched != MPLPXX_SCHED_GREEDY && sched != MPLPXX_SCHED_COLOR)
    return fail(MPLPXX_EINVAL, "unknown schedule kind %d", sched);
  if (m > 0 && (!edges || !pairwise)) return fail(MPLPXX_EINVAL, "edges/pairwise is NULL");
  if (potts && !known_cost_kind(potts)) return fail(MPLPXX_EINVAL, "unknown cost kind %d", potts);
  if (potts && (dtype != MPLPXX_F32 || device_costs)) return fail(MPLPXX_EINVAL, "structured costs take FP32 host costs");
  if (potts && L > 64) return fail(MPLPXX_EINVAL, "structured costs take L <= 64 (got %d)", L);
  const size_t esz = dtype == MPLPXX_F32 ? 4 : 8;
  // (Potts models: one weight per edge instead of an L x L table)
  const size_t nL = (size_t)n * L, mLL = potts ? (size_t)m * cost_params(potts) : (size_t)m * L * L;
  if (!device_costs) {
    if (!finite_host(unaries, nL, dtype)) return fail(MPLPXX_EINVAL, "non-finite (or, in FP32, above 1e18) unary cost");
    if (m > 0 && !finite_host(pairwise, mLL, dtype)) return fail(MPLPXX_EINVAL, "non-finite (or, in FP32, above 1e18) pairwise cost");
  }
  mplpxx_solver* h = new (std::nothrow) mplpxx_solver();
  if (!h) return fail(MPLPXX_ENOMEM, "host allocation failed");
  h->n = n;
  h->L = L;
  h->m = (int)m;
  h->dtype = dtype;
  h->esz = esz;
  h->sched = sched;
  h->potts = potts;
  int rc = prepare_solver_graph(h, edges);
  if (rc != MPLPXX_OK) {
    delete h;
    return rc;
  }
  if (potts && h->max_deg >= 65536) {
    delete h;
    return fail(MPLPXX_EINVAL, "Potts models need degrees below 65536 (the mailbox engine's versions)");
  }
  auto bail = [&](int code) {
    free_all(h);
    delete h;
    return code;
  };
#define TRY(expr)                                  \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) {                        \
      int c_ = e_ == hipErrorOutOfMemory ? MPLPXX_ENOMEM : MPLPXX_EDEVICE; \
      fail(c_, "%s: %s", #expr, hipGetErrorString(e_)); \
      return bail(c_);                             \
    }                                              \
  } while (0)
  int dev = 0;
  TRY(hipGetDevice(&dev));
  if (device_costs && (!is_device_memory(unaries, dev) || (m > 0 && !is_device_memory(pairwise, dev)))) {
    fail(MPLPXX_EINVAL, "unaries/pairwise must be device memory of the current device %d", dev);
    return bail(MPLPXX_EINVAL);
  }
  TRY(hipDeviceGetAttribute(&h->num_cus, hipDeviceAttributeMultiprocessorCount, dev));
  TRY(hipDeviceGetAttribute(&h->wallclock_khz, hipDeviceAttributeWallClockRate, dev));
  TRY(hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking));
  TRY(hipEventCreate(&h->ev0));
  TRY(hipEventCreate(&h->ev1));
  hipError_t ae = hipSuccess;
  h->d_tables = dalloc<char>(mLL * esz + kTailPad * esz, &ae); TRY(ae);
  h->d_phi = dalloc<char>((size_t)m * 2 * L * esz + kTailPad * esz, &ae); TRY(ae);
  h->d_U = dalloc<char>(nL * esz, &ae); TRY(ae);
  h->d_unaries = dalloc<char>(nL * esz, &ae); TRY(ae);
  h->d_slots = dalloc<SlotInfo>(m, &ae); TRY(ae);
  h->d_deg = dalloc<int>(n, &ae); TRY(ae);
  h->d_ver = dalloc<int>(n, &ae); TRY(ae);
  h->d_err = dalloc<int>(8, &ae); TRY(ae);
  h->d_node_ptr = dalloc<int>(n + 1, &ae); TRY(ae);
  h->d_inc = dalloc<int>(2 * (size_t)m, &ae); TRY(ae);
  h->d_node_min = dalloc<double>(n, &ae); TRY(ae);
  h->d_edge_min = dalloc<double>(m, &ae); TRY(ae);
  h->d_scalar = dalloc<double>(4, &ae); TRY(ae);
  h->d_labels = dalloc<int>(n, &ae); TRY(ae);
  if (dtype == MPLPXX_F32) {
    h->d_mb = dalloc<unsigned long long>(nL, &ae);
    TRY(ae);
    h->d_Ulo = dalloc<float>(nL, &ae);
    TRY(ae);
  }

  hipStream_t st = h->own_stream;
  // incidence lists (CSR by node, slots ascending) for dual and decode
  std::vector<int> node_ptr(n + 1, 0), inc(2 * (size_t)m);
  for (int i = 0; i < h->m; ++i) {
    node_ptr[h->slots[i].u + 1]++;
    node_ptr[h->slots[i].v + 1]++;
  }
  for (int u = 0; u < n; ++u) node_ptr[u + 1] += node_ptr[u];
  {
    std::vector<int> fillp(node_ptr.begin(), node_ptr.end() - 1);
    for (int i = 0; i < h->m; ++i) {
      inc[fillp[h->slots[i].u]++] = 2 * i + 0;
      inc[fillp[h->slots[i].v]++] = 2 * i + 1;
    }
  }
  TRY(hipMemcpyAsync(h->d_node_ptr, node_ptr.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice, st));
  if (m) TRY(hipMemcpyAsync(h->d_inc, inc.data(), inc.size() * sizeof(int), hipMemcpyHostToDevice, st));
  if (m) TRY(hipMemcpyAsync(h->d_slots, h->slots.data(), m * sizeof(SlotInfo), hipMemcpyHostToDevice, st));
  TRY(hipMemcpyAsync(h->d_deg, h->deg.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
  TRY(hipMemsetAsync(h->d_phi, 0, (size_t)m * 2 * L * esz + kTailPad * esz, st));
  TRY(hipMemsetAsync(static_cast<char*>(h->d_tables) + mLL * esz, 0, kTailPad * esz, st));
  TRY(hipMemsetAsync(h->d_err, 0, 8 * sizeof(int), st));

  if (!device_costs) {
    TRY(hipMemcpyAsync(h->d_unaries, unaries, nL * esz, hipMemcpyHostToDevice, st));
    if (m) {
      // pack tables in slot order, transposing edges given as (v, u)
      // (structured costs: the parameters in slot order, symmetric in s, t;
      // a Potts weight of -0 is stored as +0, which stands for the same
      // table)
      std::vector<char> packed(mLL * esz);
      const size_t tb = (potts ? (size_t)cost_params(potts) : (size_t)L * L) * esz;
      const char* src = static_cast<const char*>(pairwise);
      for (int i = 0; i < h->m; ++i) {
        const int e = h->order[i];
        char* dst = packed.data() + (size_t)i * tb;
        const char* s = src + (size_t)e * tb;
        if (potts == MPLPXX_COST_POTTS) {
          const float wv = *reinterpret_cast<const float*>(s) + 0.0f;
          std::memcpy(dst, &wv, sizeof(float));
        } else if (potts == MPLPXX_COST_TRUNC_QUAD || potts == MPLPXX_COST_TRUNC_LINEAR) {
          // (w and tau of -0 as +0: every cost is then +0 or positive)
          const float wt[2] = {reinterpret_cast<const float*>(s)[0] + 0.0f, reinterpret_cast<const float*>(s)[1] + 0.0f};
          std::memcpy(dst, wt, sizeof wt);
        } else if (potts || !h->flip[e]) {
          std::memcpy(dst, s, tb);
        } else {
          for (int r = 0; r < L; ++r)
            for (int c = 0; c < L; ++c)
              std::memcpy(dst + ((size_t)r * L + c) * esz, s + ((size_t)c * L + r) * esz, esz);
        }
      }
      TRY(hipMemcpyAsync(h->d_tables, packed.data(), packed.size(), hipMemcpyHostToDevice, st));
      TRY(hipStreamSynchronize(st));  // `packed` goes out of scope
    }
  } else {
    int* d_flag = nullptr;
    int* d_se = nullptr;
    int* d_sf = nullptr;
    TRY(hipStreamSynchronize(st));
    hipStream_t cs = copy_stream ? copy_stream : st;
    if (copy_stream) TRY(hipStreamSynchronize(copy_stream));
    TRY(hipMalloc(&d_flag, sizeof(int)));
    TRY(hipMemsetAsync(d_flag, 0, sizeof(int), cs));
    TRY(hipMemcpyAsync(h->d_unaries, unaries, nL * esz, hipMemcpyDeviceToDevice, cs));
    if (dtype == MPLPXX_F32) {
      TRY(launch_check_finite<float>((const float*)unaries, nL, d_flag, cs));
      if (m) TRY(launch_check_finite<float>((const float*)pairwise, mLL, d_flag, cs));
    } else {
      TRY(launch_check_finite<double>((const double*)unaries, nL, d_flag, cs));
      if (m) TRY(launch_check_finite<double>((const double*)pairwise, mLL, d_flag, cs));
    }
    if (m) {
      std::vector<int> se(m), sf(m);
      for (int i = 0; i < h->m; ++i) {
        se[i] = h->order[i];
        sf[i] = h->flip[h->order[i]];
      }
      TRY(hipMalloc(&d_se, m * sizeof(int)));
      TRY(hipMalloc(&d_sf, m * sizeof(int)));
      TRY(hipMemcpyAsync(d_se, se.data(), m * sizeof(int), hipMemcpyHostToDevice, cs));
      TRY(hipMemcpyAsync(d_sf, sf.data(), m * sizeof(int), hipMemcpyHostToDevice, cs));
      if (dtype == MPLPXX_F32)
        TRY(launch_pack_tables<float>((const float*)pairwise, (float*)h->d_tables, d_se, d_sf, h->m, L, cs));
      else
        TRY(launch_pack_tables<double>((const double*)pairwise, (double*)h->d_tables, d_se, d_sf, h->m, L, cs));
    }
    int flag = 0;
    TRY(hipMemcpyAsync(&flag, d_flag, sizeof(int), hipMemcpyDeviceToHost, cs));
    TRY(hipStreamSynchronize(cs));
    (void)hipFree(d_flag);
    if (d_se) (void)hipFree(d_se);
    if (d_sf) (void)hipFree(d_sf);
    if (flag) {
      fail(MPLPXX_EINVAL, "non-finite cost");
      return bail(MPLPXX_EINVAL);
    }
  }
  TRY(hipMemcpyAsync(h->d_U, h->d_unaries, nL * esz, hipMemcpyDeviceToDevice, st));
  if (h->d_Ulo) TRY(hipMemsetAsync(h->d_Ulo, 0, nL * sizeof(float), st));
  TRY(hipStreamSynchronize(st));
#undef TRY
  *out = h;
  return MPLPXX_OK;
}

int sync_and_check(mplpxx_solver* h) {
  HIP_TRY(hipStreamSynchronize(h->stream()));
  int err[8] = {0};
  HIP_TRY(hipMemcpy(err, h->d_err, 8 * sizeof(int), hipMemcpyDeviceToHost));
  if (err[0] != 0) {
    (void)hipMemsetAsync(h->d_err, 0, 8 * sizeof(int), h->stream());
    (void)hipStreamSynchronize(h->stream());
    return fail(err[0], "device wait exceeded its bound (workgroup %d, slot %d, node %d, expected version %d, seen %d)",
                err[1], err[2], err[3], err[4], err[5]);
  }
  return MPLPXX_OK;
}

template <typename T> HsArgs<T> hs_args(mplpxx_solver* h, double* trace) {
  HsArgs<T> a{};
  a.tables = static_cast<const T*>(h->d_tables);
  a.phi = static_cast<T*>(h->d_phi);
  a.U = static_cast<T*>(h->d_U);
  a.Ulo = sizeof(T) == 4 ? reinterpret_cast<T*>(h->d_Ulo) : nullptr;
  a.slots = h->d_slots;
  a.deg = h->d_deg;
  a.ver = h->d_ver;
  a.err = h->d_err;
  a.trace = trace;
  a.stamps = h->profile ? h->d_stamps : nullptr;
  a.L = h->L;
  a.m = h->m;
  a.n = h->n;
  a.spin_limit = h->spin_limit;
  return a;
}

// messages of a workgroup's slots kept in LDS up to this size
constexpr size_t kPhiLdsBudget = 96 * 1024;

template <typename T> int iterate_t(mplpxx_solver* h, int k, double* trace_host) {
  hipStream_t st = h->stream();
  if (h->profile && !h->d_stamps && h->m > 0) {
    HIP_TRY(hipMalloc(&h->d_stamps, (size_t)h->m * kStampStride * sizeof(long long)));
    HIP_TRY(hipMemsetAsync(h->d_stamps, 0, (size_t)h->m * kStampStride * sizeof(long long), st));
  }
  // FP32 traces add the edge terms of Eq. (3): rounding-level numbers, but
  // with a bias, so over many edges they matter at the 1e-5 level
  constexpr int kTraceW = 8;  // partial minima per slot (waves of the mailbox engine, at most 8)
  const bool edge_terms = sizeof(T) == 4 && h->m > 0;
  if (trace_host && k > h->trace_cap) {
    for (void** p : {(void**)&h->d_trace_nodes, (void**)&h->d_trace_out, (void**)&h->d_trace_e})
      if (*p) { (void)hipFree(*p); *p = nullptr; }
    h->trace_cap = 0;
    HIP_TRY(hipMalloc(&h->d_trace_nodes, (size_t)k * h->n * sizeof(double)));
    HIP_TRY(hipMalloc(&h->d_trace_out, (size_t)k * sizeof(double)));
    if (edge_terms) HIP_TRY(hipMalloc(&h->d_trace_e, (size_t)k * h->m * kTraceW * sizeof(float)));
    h->trace_cap = k;
  }
  int trace_w = 1;
  const bool rule_mb = !trace_host && h->rule_mailbox();
  const int engine = rule_mb ? ENGINE_PERSISTENT : h->engine();
  const int LT = h->LT(), NT = rule_mb ? 256 : h->NT();
  HIP_TRY(hipEventRecord(h->ev0, st));
  if (h->m > 0 && k > 0) {
    if (engine == ENGINE_STEP) {
      HsArgs<T> a = hs_args<T>(h, nullptr);
      for (int it = 0; it < k; ++it) {
        for (int s = 0; s < h->S; ++s) {
          const int b = h->step_ptr[s], c = h->step_ptr[s + 1] - b;
          if (h->rule == MPLPXX_RULE_H) HIP_TRY(launch_handshake<T>(a, ENGINE_STEP, LT, NT, b, c, 0, 1, st));
          else HIP_TRY(launch_step_rule<T>(a, h->rule, LT, NT, b, c, st));
        }
        if (trace_host) {
          HIP_TRY(launch_trace_nodes<T>(static_cast<const T*>(h->d_U), a.Ulo, h->n, h->L,
                                        h->d_trace_nodes + (size_t)it * h->n, st));
          if (edge_terms)
            HIP_TRY(launch_trace_edges<T>(static_cast<const T*>(h->d_tables), static_cast<const T*>(h->d_phi), h->m,
                                          h->L, h->d_trace_e + (size_t)it * h->m, st));
        }
      }
    } else if (sizeof(T) == 4) {
      // FP32: tagged mailboxes; messages stay in LDS when they fit
      HsArgs<float> a = hs_args<float>(h, trace_host ? h->d_trace_nodes : nullptr);
      if (trace_host) {
        a.trace_e = h->d_trace_e;
        trace_w = NT / 64;
      }
      const int G = h->grid();
      const size_t words = (size_t)G * (NT + 128);
      if (h->sink_words < words) {
        if (h->d_sink) (void)hipFree(h->d_sink);
        h->d_sink = nullptr;
        h->sink_words = 0;
        HIP_TRY(hipMalloc(&h->d_sink, words * sizeof(unsigned long long)));
        h->sink_words = words;
      }
      a.sink = h->d_sink;
      const size_t owned = ((size_t)h->m + G - 1) / G;
      const size_t phi_bytes = owned * 2 * h->L * sizeof(float);
      // (more than one workgroup per compute unit: messages in HBM, so that
      // the workgroups' LDS never limits how many fit)
      const int in_lds = phi_bytes <= kPhiLdsBudget && G <= h->num_cus && h->phi_opt != 2 ? 1 : 0;
      HIP_TRY(launch_mb_init(static_cast<const float*>(h->d_U), h->d_Ulo, h->d_mb, (size_t)h->n * h->L, st));
      if (h->potts && !h->gen_tiles())
        HIP_TRY(launch_persistent_mb_potts(a, h->d_mb, G, k, in_lds, in_lds ? phi_bytes : 0, st, h->potts));
      else
        HIP_TRY(launch_persistent_mb(a, h->d_mb, LT, NT, G, k, in_lds, in_lds ? phi_bytes : 0, st, h->prefetch_opt,
                                     h->gen_tiles() ? h->potts : 0, rule_mb ? h->rule : MPLPXX_RULE_H));
      HIP_TRY(launch_mb_fini(static_cast<float*>(h->d_U), h->d_Ulo, h->d_mb, h->n, h->L,
                             trace_host ? h->d_trace_nodes + (size_t)(k - 1) * h->n : nullptr, st));
    } else if (!trace_host && h->L <= 64) {
      // FP64 without a trace: the mailbox forward (two tagged words per
      // label, no fences; bitwise the version-counter engine below)
      const size_t nL = (size_t)h->n * h->L;
      if (!h->d_mb64) HIP_TRY(hipMalloc(&h->d_mb64, 2 * nL * 2 * sizeof(unsigned long long)));
      HIP_TRY(launch_mb64_init(static_cast<const double*>(h->d_U), h->d_mb64, nL, st));
      HIP_TRY(launch_adj64(static_cast<const double*>(h->d_tables), static_cast<double*>(h->d_phi), h->d_mb64, k,
                           nullptr, std::max(1, std::min(h->m, h->num_cus)), nullptr, nullptr, nullptr, nullptr, nullptr,
                           0, 0, h->d_slots, h->L, h->m, h->d_err, h->spin_limit, st));
      HIP_TRY(launch_mb64_fini(static_cast<double*>(h->d_U), h->d_mb64, nL, st));
    } else {
      HsArgs<T> a = hs_args<T>(h, trace_host ? h->d_trace_nodes : nullptr);
      HIP_TRY(launch_fill_int(h->d_ver, 0, h->n, st));
      HIP_TRY(launch_handshake<T>(a, ENGINE_PERSISTENT, LT, NT, 0, 0, h->grid(), k, st));
    }
  }
  HIP_TRY(hipEventRecord(h->ev1, st));
  h->timed = true;
  if (trace_host && k > 0) {
    // nodes without edges (all of them when m == 0) read U directly
    HIP_TRY(launch_trace_sum<T>(h->d_trace_nodes, edge_terms ? h->d_trace_e : nullptr, h->m, trace_w,
                                static_cast<const T*>(h->d_U), h->d_deg, h->n, h->L, k, h->d_trace_out, st));
  }
  h->iterations += k;
  if (!h->user_stream || trace_host) {
    int rc = sync_and_check(h);
    if (rc != MPLPXX_OK) return rc;
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    h->last_ms = ms;
    if (trace_host && k > 0)
      HIP_TRY(hipMemcpy(trace_host, h->d_trace_out, (size_t)k * sizeof(double), hipMemcpyDeviceToHost));
  }
  return MPLPXX_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Adjoint of K unrolled iterations (checkpoint every `every` iterations).
// ---------------------------------------------------------------------------
namespace {

// FP64 handles with tiles up to 64 labels differentiate on the persistent
// mailbox kernels (one launch per segment and direction); the per-matching
// engine option keeps one launch per matching.  Both give the same bits.
template <typename T> bool adjoint_persistent(const mplpxx_solver* h) {
  return sizeof(T) == 8 && h->L <= 64 && h->m > 0 && h->engine() != ENGINE_STEP;
}
// workgroups of one role of the persistent adjoint launch: one per compute
// unit for a launch with one role, half of them each when the reverse of
// one segment runs beside the recomputation of the previous one (a
// workgroup of either role fits beside one of the other on a unit); at most
// one per slot
int adjoint_grid(const mplpxx_solver* h, bool two_roles) {
  return std::max(1, std::min(h->m, two_roles ? h->num_cus / 2 : h->num_cus));
}

// `seg` iterations of an FP64 handle on the persistent forward, the
// unaries through the mailboxes
int fwd64_segment(mplpxx_solver* h, int seg) {
  hipStream_t st = h->stream();
  const size_t nL = (size_t)h->n * h->L;
  HIP_TRY(launch_mb64_init(static_cast<const double*>(h->d_U), h->d_mb64, nL, st));
  HIP_TRY(launch_adj64(static_cast<const double*>(h->d_tables), static_cast<double*>(h->d_phi), h->d_mb64, seg, nullptr,
                       adjoint_grid(h, false), nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0, h->d_slots, h->L,
                       h->m, h->d_err, h->spin_limit, st));
  HIP_TRY(launch_mb64_fini(static_cast<double*>(h->d_U), h->d_mb64, nL, st));
  const int rc = sync_and_check(h);
  if (rc == MPLPXX_OK) h->iterations += seg;
  return rc;
}

template <typename T> int adjoint_forward_t(mplpxx_solver* h, int K, int every, double* loss) {
  hipStream_t st = h->stream();
  const size_t nL = (size_t)h->n * h->L, mp = (size_t)h->m * 2 * h->L, esz = sizeof(T);
  const int nck = (int)(((long long)K + every - 1) / every);  // (64-bit: K + every can pass 2^31)
  const bool pers = adjoint_persistent<T>(h);
  // (re)allocate checkpoint and record storage
  for (void** p : {&h->d_ck_U, &h->d_ck_phi, (void**)&h->d_rec, (void**)&h->d_ck_Ulo, (void**)&h->d_contrib})
    if (*p) { (void)hipFree(*p); *p = nullptr; }
  if (pers) {
    if (!h->d_mb64) HIP_TRY(hipMalloc(&h->d_mb64, 2 * nL * 2 * sizeof(unsigned long long)));
    HIP_TRY(hipMalloc(&h->d_contrib, (size_t)every * h->m * 3 * h->L * sizeof(double)));
  }
  const size_t rec_bytes = (pers ? 2 : 1) * (size_t)every * h->m * 3 * h->L;
  HIP_TRY(hipMalloc(&h->d_ck_U, (nck + 1) * nL * esz));
  if (h->d_Ulo) HIP_TRY(hipMalloc((void**)&h->d_ck_Ulo, (nck + 1) * nL * sizeof(float)));
  HIP_TRY(hipMalloc(&h->d_ck_phi, std::max<size_t>(1, (nck + 1) * mp * esz)));
  HIP_TRY(hipMalloc(&h->d_rec, std::max<size_t>(1, rec_bytes)));
  if (!h->d_Ub) HIP_TRY(hipMalloc(&h->d_Ub, nL * esz));
  if (!h->d_pb) HIP_TRY(hipMalloc(&h->d_pb, std::max<size_t>(1, mp * esz)));
  if (!h->d_thb) HIP_TRY(hipMalloc(&h->d_thb, std::max<size_t>(1, (size_t)h->m * h->L * h->L * esz)));
  h->adj_bytes = (nck + 1) * nL * esz + (h->d_Ulo ? (nck + 1) * nL * sizeof(float) : 0) + (nck + 1) * mp * esz +
                 rec_bytes + nL * esz + mp * esz + (size_t)h->m * h->L * h->L * esz + (size_t)h->m * 2 * sizeof(int) +
                 (pers ? 2 * nL * 2 * sizeof(unsigned long long) + (size_t)every * h->m * 3 * h->L * sizeof(double) : 0);
  if (!h->d_slot_of_edge && h->m) {
    HIP_TRY(hipMalloc(&h->d_slot_of_edge, h->m * sizeof(int)));
    HIP_TRY(hipMalloc(&h->d_edge_flip, h->m * sizeof(int)));
    HIP_TRY(hipMemcpyAsync(h->d_slot_of_edge, h->slot_of_edge.data(), h->m * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(h->d_edge_flip, h->flip.data(), h->m * sizeof(int), hipMemcpyHostToDevice, st));
  }
  // start from phi = 0, U = theta_u
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipMemsetAsync(h->d_phi, 0, mp * esz, st));
  HIP_TRY(hipMemcpyAsync(h->d_U, h->d_unaries, nL * esz, hipMemcpyDeviceToDevice, st));
  if (h->d_Ulo) HIP_TRY(hipMemsetAsync(h->d_Ulo, 0, nL * sizeof(float), st));
  h->iterations = 0;
  for (int c = 0; c < nck; ++c) {
    HIP_TRY(hipMemcpyAsync((char*)h->d_ck_U + c * nL * esz, h->d_U, nL * esz, hipMemcpyDeviceToDevice, st));
    if (h->d_Ulo)
      HIP_TRY(hipMemcpyAsync(h->d_ck_Ulo + c * nL, h->d_Ulo, nL * sizeof(float), hipMemcpyDeviceToDevice, st));
    if (h->m) HIP_TRY(hipMemcpyAsync((char*)h->d_ck_phi + c * mp * esz, h->d_phi, mp * esz, hipMemcpyDeviceToDevice, st));
    const int seg = std::min(every, K - c * every);
    const int rc = pers ? fwd64_segment(h, seg) : iterate_t<T>(h, seg, nullptr);
    if (rc != MPLPXX_OK) return rc;
  }
  HIP_TRY(hipMemcpyAsync((char*)h->d_ck_U + nck * nL * esz, h->d_U, nL * esz, hipMemcpyDeviceToDevice, st));
  if (h->d_Ulo)
    HIP_TRY(hipMemcpyAsync(h->d_ck_Ulo + nck * nL, h->d_Ulo, nL * sizeof(float), hipMemcpyDeviceToDevice, st));
  if (h->m) HIP_TRY(hipMemcpyAsync((char*)h->d_ck_phi + nck * mp * esz, h->d_phi, mp * esz, hipMemcpyDeviceToDevice, st));
  // loss = sum_u min_s U_u in FP64 (node minima, then a fixed-order sum)
  const T* lo = sizeof(T) == 4 ? reinterpret_cast<const T*>(h->d_Ulo) : nullptr;
  HIP_TRY(launch_adj_seed<T>(static_cast<const T*>(h->d_U), lo, h->n, h->L, static_cast<T*>(h->d_Ub), h->d_node_min,
                             st));
  HIP_TRY(hipStreamSynchronize(st));
  h->adj_K = K;
  h->adj_every = every;
  h->adj_nck = nck;
  h->adj_ready = true;
  h->adj_iter_mark = h->iterations;
  if (loss) {
    // the loss is the dual bound of Eq. (3) of the final state, recomputed
    // in FP64 from the messages; it differs from sum_u min_s U_u only by the
    // edge terms, which are zero in exact arithmetic (so they add nothing to
    // the gradient) and rounding-level numbers in FP32
    HIP_TRY(launch_dual<T>(static_cast<const T*>(h->d_unaries), static_cast<const T*>(h->d_tables),
                           static_cast<const T*>(h->d_phi), h->d_node_ptr, h->d_inc, h->n, h->L, h->m, h->d_node_min,
                           h->d_edge_min, h->d_scalar, st));
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipMemcpy(loss, h->d_scalar, sizeof(double), hipMemcpyDeviceToHost));
  }
  return MPLPXX_OK;
}

template <typename T> int adjoint_backward_t(mplpxx_solver* h, void* grad_u, void* grad_pw) {
  hipStream_t st = h->stream();
  const size_t nL = (size_t)h->n * h->L, mp = (size_t)h->m * 2 * h->L, esz = sizeof(T);
  const int K = h->adj_K, every = h->adj_every, nck = h->adj_nck;
  const size_t rec_it = (size_t)h->m * 3 * h->L;
  T* lo = sizeof(T) == 4 ? reinterpret_cast<T*>(h->d_Ulo) : nullptr;
  const T* ck_lo = sizeof(T) == 4 ? reinterpret_cast<const T*>(h->d_ck_Ulo) : nullptr;
  // seed from the final state
  HIP_TRY(launch_adj_seed<T>(static_cast<const T*>((const void*)((char*)h->d_ck_U + nck * nL * esz)),
                             ck_lo ? ck_lo + nck * nL : nullptr, h->n, h->L, static_cast<T*>(h->d_Ub),
                             h->d_node_min, st));
  if (h->m) {
    HIP_TRY(hipMemsetAsync(h->d_pb, 0, mp * esz, st));
    HIP_TRY(hipMemsetAsync(h->d_thb, 0, (size_t)h->m * h->L * h->L * esz, st));
  }
  const bool pers = adjoint_persistent<T>(h) && h->d_mb64 && h->d_contrib;
  if (pers) {
    // Persistent pipeline: launch c runs the reverse of segment c beside
    // the recomputation (with argmin records) of segment c - 1, which needs
    // only its checkpoint; records alternate between two buffers.  The
    // first launch recomputes the last segment alone, the last reverses
    // segment 0 alone.
    unsigned long long* mb_fwd = h->d_mb64;
    unsigned long long* mb_rev = h->d_mb64 + 2 * nL;
    auto rec_of = [&](int c) { return h->d_rec + (size_t)(c & 1) * every * rec_it; };
    auto seg_of = [&](int c) { return std::min(every, K - c * every); };
    auto restore = [&](int c) -> hipError_t {
      hipError_t e = hipMemcpyAsync(h->d_U, (char*)h->d_ck_U + c * nL * esz, nL * esz, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(h->d_phi, (char*)h->d_ck_phi + c * mp * esz, mp * esz, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess) e = launch_mb64_init(static_cast<const double*>(h->d_U), mb_fwd, nL, st);
      return e;
    };
    for (int c = nck; c >= 0; --c) {
      // reverse of segment c (c < nck), recomputation of segment c - 1 (c >= 1)
      const bool rev = c < nck, fwd = c >= 1;
      if (fwd) HIP_TRY(restore(c - 1));
      if (rev) HIP_TRY(launch_mb64_init(static_cast<const double*>(h->d_Ub), mb_rev, nL, st));
      const bool both = rev && fwd;
      HIP_TRY(launch_adj64(static_cast<const double*>(h->d_tables), static_cast<double*>(h->d_phi), mb_fwd,
                           fwd ? seg_of(c - 1) : 0, fwd ? rec_of(c - 1) : nullptr, adjoint_grid(h, both),
                           rev ? rec_of(c) : nullptr, mb_rev, static_cast<double*>(h->d_pb), h->d_contrib,
                           static_cast<double*>(h->d_thb), rev ? seg_of(c) : 0, adjoint_grid(h, both), h->d_slots,
                           h->L, h->m, h->d_err, h->spin_limit, st));
      if (rev) HIP_TRY(launch_mb64_fini(static_cast<double*>(h->d_Ub), mb_rev, nL, st));
      const int rc = sync_and_check(h);
      if (rc != MPLPXX_OK) return rc;
    }
  }
  for (int c = nck - 1; c >= 0 && h->m > 0 && !pers; --c) {
    const int seg = std::min(every, K - c * every);
    HIP_TRY(hipMemcpyAsync(h->d_U, (char*)h->d_ck_U + c * nL * esz, nL * esz, hipMemcpyDeviceToDevice, st));
    if (lo) HIP_TRY(hipMemcpyAsync(lo, ck_lo + c * nL, nL * esz, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(h->d_phi, (char*)h->d_ck_phi + c * mp * esz, mp * esz, hipMemcpyDeviceToDevice, st));
    for (int i = 0; i < seg; ++i)
      for (int s = 0; s < h->S; ++s)
        HIP_TRY(launch_step_record<T>(static_cast<const T*>(h->d_tables), static_cast<T*>(h->d_phi),
                                      static_cast<T*>(h->d_U), lo, h->d_slots, h->L, h->step_ptr[s],
                                      h->step_ptr[s + 1] - h->step_ptr[s], h->d_rec + i * rec_it, st));
    for (int i = seg - 1; i >= 0; --i)
      for (int s = h->S - 1; s >= 0; --s)
        HIP_TRY(launch_adj_step<T>(h->d_slots, h->L, h->step_ptr[s], h->step_ptr[s + 1] - h->step_ptr[s],
                                   h->d_rec + i * rec_it, static_cast<T*>(h->d_Ub), static_cast<T*>(h->d_pb),
                                   static_cast<T*>(h->d_thb), st));
  }
  // outputs in the caller's layout; the handle's state back to the forward's end
  if (grad_u) HIP_TRY(hipMemcpyAsync(grad_u, h->d_Ub, nL * esz, hipMemcpyDeviceToDevice, st));
  if (grad_pw && h->m)
    HIP_TRY(launch_pack_tables<T>(static_cast<const T*>(h->d_thb), static_cast<T*>(grad_pw), h->d_slot_of_edge,
                                  h->d_edge_flip, h->m, h->L, st));
  HIP_TRY(hipMemcpyAsync(h->d_U, (char*)h->d_ck_U + nck * nL * esz, nL * esz, hipMemcpyDeviceToDevice, st));
  if (lo) HIP_TRY(hipMemcpyAsync(lo, ck_lo + nck * nL, nL * esz, hipMemcpyDeviceToDevice, st));
  if (h->m) HIP_TRY(hipMemcpyAsync(h->d_phi, (char*)h->d_ck_phi + nck * mp * esz, mp * esz, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  return MPLPXX_OK;
}

}  // namespace

namespace {
// FP64 twin of an FP32 handle: the same graph and costs widened exactly, in
// the caller's layout (tables unpacked from slot order), created on the
// handle's stream
int make_shadow(mplpxx_solver* h) {
  hipStream_t st = h->stream();
  const size_t nL = (size_t)h->n * h->L, mLL = (size_t)h->m * h->L * h->L;
  std::vector<int32_t> edges(2 * (size_t)h->m);
  for (int e = 0; e < h->m; ++e) {
    const SlotInfo& si = h->slots[h->slot_of_edge[e]];
    edges[2 * e] = h->flip[e] ? si.v : si.u;
    edges[2 * e + 1] = h->flip[e] ? si.u : si.v;
  }
  double* u64 = nullptr;
  double* t64 = nullptr;
  double* p64 = nullptr;
  int* d_soe = nullptr;
  int* d_flip = nullptr;
  auto cleanup = [&]() {
    for (void* p : {(void*)u64, (void*)t64, (void*)p64, (void*)d_soe, (void*)d_flip})
      if (p) (void)hipFree(p);
  };
  hipError_t e = hipMalloc(&u64, std::max<size_t>(1, nL) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&t64, std::max<size_t>(1, mLL) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&p64, std::max<size_t>(1, mLL) * sizeof(double));
  if (e == hipSuccess && h->m) e = hipMalloc(&d_soe, h->m * sizeof(int));
  if (e == hipSuccess && h->m) e = hipMalloc(&d_flip, h->m * sizeof(int));
  if (e == hipSuccess && h->m)
    e = hipMemcpyAsync(d_soe, h->slot_of_edge.data(), h->m * sizeof(int), hipMemcpyHostToDevice, st);
  if (e == hipSuccess && h->m) e = hipMemcpyAsync(d_flip, h->flip.data(), h->m * sizeof(int), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_convert(static_cast<const float*>(h->d_unaries), u64, nL, st);
  if (e == hipSuccess && h->m) e = launch_convert(static_cast<const float*>(h->d_tables), t64, mLL, st);
  if (e == hipSuccess && h->m) e = launch_pack_tables<double>(t64, p64, d_soe, d_flip, h->m, h->L, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    cleanup();
    return fail(e == hipErrorOutOfMemory ? MPLPXX_ENOMEM : MPLPXX_EDEVICE, "FP64 twin: %s", hipGetErrorString(e));
  }
  const int rc = create_impl(h->n, h->L, h->m, h->m ? edges.data() : nullptr, u64, h->m ? p64 : nullptr, MPLPXX_F64,
                             true, st, &h->shadow, h->sched);
  cleanup();
  return rc;
}

// nearest bf16 value, ties to even (the rounding the device applies to U_comp)
float bf16_round_host(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  std::memcpy(&x, &u, 4);
  return x;
}
}  // namespace

extern "C" {

int mplpxx_create(int32_t n, int32_t L, int64_t m, const int32_t* edges, const void* unaries, const void* pairwise,
                  int32_t dtype, mplpxx_solver** out) {
  return create_impl(n, L, m, edges, unaries, pairwise, dtype, false, nullptr, out);
}

int mplpxx_create_potts(int32_t n, int32_t L, int64_t m, const int32_t* edges, const float* unaries, const float* weights,
                        mplpxx_solver** out) {
  return create_impl(n, L, m, edges, unaries, weights, MPLPXX_F32, false, nullptr, out, MPLPXX_SCHED_AUTO,
                     MPLPXX_COST_POTTS);
}

int mplpxx_create_structured(int32_t n, int32_t L, int64_t m, const int32_t* edges, const float* unaries, int32_t kind,
                             const float* params, mplpxx_solver** out) {
  if (out) *out = nullptr;
  if (!known_cost_kind(kind)) return fail(MPLPXX_EINVAL, "unknown cost kind %d", kind);
  if (m > 0 && !params) return fail(MPLPXX_EINVAL, "params is NULL");
  if (m > 0 && m <= 0x3fffffff) {
    const int rc = check_structured_params(kind, params, m);
    if (rc != MPLPXX_OK) return rc;
  }
  return create_impl(n, L, m, edges, unaries, params, MPLPXX_F32, false, nullptr, out, MPLPXX_SCHED_AUTO, kind);
}

int mplpxx_create_device(int32_t n, int32_t L, int64_t m, const int32_t* edges, const void* unaries_dev,
                         const void* pairwise_dev, int32_t dtype, void* hip_stream, mplpxx_solver** out) {
  return create_impl(n, L, m, edges, unaries_dev, pairwise_dev, dtype, true, static_cast<hipStream_t>(hip_stream), out);
}

int mplpxx_create_sched(int32_t n, int32_t L, int64_t m, const int32_t* edges, const void* unaries,
                        const void* pairwise, int32_t dtype, int32_t schedule, mplpxx_solver** out) {
  return create_impl(n, L, m, edges, unaries, pairwise, dtype, false, nullptr, out, schedule);
}

int mplpxx_iterate(mplpxx_solver* h, int32_t k) {
  if (!h) return fail(MPLPXX_EINVAL, "handle is NULL");
  if (k < 0) return fail(MPLPXX_EINVAL, "k must be >= 0");
  return h->dtype == MPLPXX_F32 ? iterate_t<float>(h, k, nullptr) : iterate_t<double>(h, k, nullptr);
}

int mplpxx_iterate_trace(mplpxx_solver* h, int32_t k, double* trace) {
  if (!h) return fail(MPLPXX_EINVAL, "handle is NULL");
  if (h->potts) return fail(MPLPXX_EINVAL, "per-iteration traces are not available for structured costs (use mplpxx_iterate_gap)");
  if (k < 0) return fail(MPLPXX_EINVAL, "k must be >= 0");
  if (k > 0 && !trace) return fail(MPLPXX_EINVAL, "trace is NULL");
  return h->dtype == MPLPXX_F32 ? iterate_t<float>(h, k, trace) : iterate_t<double>(h, k, trace);
}

int mplpxx_adjoint_forward(mplpxx_solver* h, int32_t K, int32_t every, double* loss) {
  if (!h) return fail(MPLPXX_EINVAL, "handle is NULL");
  if (h->potts) return fail(MPLPXX_EINVAL, "the adjoint takes dense tables");
  if (K < 1 || every < 1) return fail(MPLPXX_EINVAL, "K and every must be >= 1");
  if (h->rule != MPLPXX_RULE_H) return fail(MPLPXX_EINVAL, "the adjoint takes the (H) update only");
  h->adj_ready = false;
  if (h->dtype == MPLPXX_F32 && h->adjoint_f64) {
    if (!h->shadow) {
      const int rc = make_shadow(h);
      if (rc != MPLPXX_OK) return rc;
    }
    h->shadow->engine_opt = h->engine_opt;  // (one launch per matching, or persistent)
    h->shadow->spin_limit = h->spin_limit;
    int rc = adjoint_forward_t<double>(h->shadow, K, every, loss);
    if (rc != MPLPXX_OK) return rc;
    // the handle's own FP32 run of K iterations from phi = 0
    hipStream_t st = h->stream();
    const size_t nL = (size_t)h->n * h->L;
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipMemsetAsync(h->d_phi, 0, (size_t)h->m * 2 * h->L * sizeof(float), st));
    HIP_TRY(hipMemcpyAsync(h->d_U, h->d_unaries, nL * sizeof(float), hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemsetAsync(h->d_Ulo, 0, nL * sizeof(float), st));
    h->iterations = 0;
    rc = iterate_t<float>(h, K, nullptr);
    if (rc != MPLPXX_OK) return rc;
    rc = sync_and_check(h);
    if (rc != MPLPXX_OK) return rc;
    h->adj_ready = true;
    h->adj_iter_mark = h->iterations;
    return MPLPXX_OK;
  }
  return h->dtype == MPLPXX_F32 ? adjoint_forward_t<float>(h, K, every, loss) : adjoint_forward_t<double>(h, K, every, loss);
}

int mplpxx_adjoint_backward(mplpxx_solver* h, void* grad_unaries, void* grad_pairwise) {
  if (!h) return fail(MPLPXX_EINVAL, "handle is NULL");
  if (!h->adj_ready || h->iterations != h->adj_iter_mark)
    return fail(MPLPXX_ESTATE, "no adjoint forward to differentiate (call mplpxx_adjoint_forward first)");
  if (h->dtype == MPLPXX_F32 && h->adjoint_f64) {
    // FP64 gradients of the twin, narrowed into the caller's FP32 buffers
    hipStream_t st = h->stream();
    const size_t nL = (size_t)h->n * h->L, mLL = (size_t)h->m * h->L * h->L;
    double* gu = nullptr;
    double* gp = nullptr;
    HIP_TRY(hipMalloc(&gu, std::max<size_t>(1, nL) * sizeof(double)));
    if (hipMalloc(&gp, std::max<size_t>(1, mLL) * sizeof(double)) != hipSuccess) {
      (void)hipFree(gu);
      return fail(MPLPXX_ENOMEM, "gradient buffers");
    }
    int rc = adjoint_backward_t<double>(h->shadow, grad_unaries ? gu : nullptr, grad_pairwise ? gp : nullptr);
    hipError_t e = hipSuccess;
    if (rc == MPLPXX_OK) {
      HIP_TRY(hipStreamSynchronize(h->shadow->stream()));
      if (grad_unaries) e = launch_convert(gu, static_cast<float*>(grad_unaries), nL, st);
      if (e == hipSuccess && grad_pairwise && mLL) e = launch_convert(gp, static_cast<float*>(grad_pairwise), mLL, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    (void)hipFree(gu);
    (void)hipFree(gp);
    if (rc != MPLPXX_OK) return rc;
    if (e != hipSuccess) return fail(MPLPXX_EDEVICE, "gradient narrowing: %s", hipGetErrorString(e));
    return MPLPXX_OK;
  }
  return h->dtype == MPLPXX_F32 ? adjoint_backward_t<float>(h, grad_unaries, grad_pairwise)
                                : adjoint_backward_t<double>(h, grad_unaries, grad_pairwise);
}

int mplpxx_dual_bound(mplpxx_solver* h, double* out) {
  if (!h || !out) return fail(MPLPXX_EINVAL, "NULL argument");
  hipStream_t st = h->stream();
  if (h->dtype == MPLPXX_F32)
    HIP_TRY(launch_dual<float>((const float*)h->d_unaries, (const float*)h->d_tables, (const float*)h->d_phi,
                               h->d_node_ptr, h->d_inc, h->n, h->L, h->m, h->d_node_min, h->d_edge_min, h->d_scalar, st,
                               h->potts));
  else
    HIP_TRY(launch_dual<double>((const double*)h->d_unaries, (const double*)h->d_tables, (const double*)h->d_phi,
                                h->d_node_ptr, h->d_inc, h->n, h->L, h->m, h->d_node_min, h->d_edge_min, h->d_scalar, st));
  int rc = sync_and_check(h);
  if (rc != MPLPXX_OK) return rc;
  HIP_TRY(hipMemcpy(out, h->d_scalar, sizeof(double), hipMemcpyDeviceToHost));
  return MPLPXX_OK;
}

int mplpxx_decode(mplpxx_solver* h, int32_t* labels, double* energy) {
  if (!h || !labels) return fail(MPLPXX_EINVAL, "NULL argument");
  hipStream_t st = h->stream();
  if (h->dtype == MPLPXX_F32)
    HIP_TRY(launch_decode<float>((const float*)h->d_unaries, (const float*)h->d_tables, (const float*)h->d_phi,
                                 h->d_slots, h->d_node_ptr, h->d_inc, h->n, h->L, h->m, h->d_labels, h->d_scalar + 1, st,
                                 h->potts));
  else
    HIP_TRY(launch_decode<double>((const double*)h->d_unaries, (const double*)h->d_tables, (const double*)h->d_phi,
                                  h->d_slots, h->d_node_ptr, h->d_inc, h->n, h->L, h->m, h->d_labels, h->d_scalar + 1, st));
  int rc = sync_and_check(h);
  if (rc != MPLPXX_OK) return rc;
  HIP_TRY(hipMemcpy(labels, h->d_labels, (size_t)h->n * sizeof(int), hipMemcpyDeviceToHost));
  if (energy) HIP_TRY(hipMemcpy(energy, h->d_scalar + 1, sizeof(double), hipMemcpyDeviceToHost));
  return MPLPXX_OK;
}

int mplpxx_iterate_gap(mplpxx_solver* h, int32_t k, double* dual, double* energy, int32_t* best_labels) {
  if (!h) return fail(MPLPXX_EINVAL, "handle is NULL");
  if (k < 1) return fail(MPLPXX_EINVAL, "k must be >= 1");
  if (!dual || !energy) return fail(MPLPXX_EINVAL, "dual or energy is NULL");
  hipStream_t st = h->stream();
  double* d_gap = nullptr;  // [k] duals, then [k] energies
  int* d_lab = nullptr;     // [k][n] labellings
  auto release = [&]() {
    (void)hipStreamSynchronize(st);
    if (d_gap) (void)hipFree(d_gap);
    if (d_lab) (void)hipFree(d_lab);
  };
  if (hipMalloc(&d_gap, (size_t)2 * k * sizeof(double)) != hipSuccess ||
      hipMalloc(&d_lab, (size_t)k * h->n * sizeof(int)) != hipSuccess) {
    release();
    return fail(MPLPXX_ENOMEM, "no device memory for the gap trace");
  }
  for (int it = 0; it < k; ++it) {
    int rc = h->dtype == MPLPXX_F32 ? iterate_t<float>(h, 1, nullptr) : iterate_t<double>(h, 1, nullptr);
    if (rc != MPLPXX_OK) {
      release();
      return rc;
    }
    hipError_t e;
    if (h->dtype == MPLPXX_F32) {
      e = launch_dual<float>((const float*)h->d_unaries, (const float*)h->d_tables, (const float*)h->d_phi,
                             h->d_node_ptr, h->d_inc, h->n, h->L, h->m, h->d_node_min, h->d_edge_min, d_gap + it, st,
                             h->potts);
      if (e == hipSuccess)
        e = launch_decode<float>((const float*)h->d_unaries, (const float*)h->d_tables, (const float*)h->d_phi,
                                 h->d_slots, h->d_node_ptr, h->d_inc, h->n, h->L, h->m, d_lab + (size_t)it * h->n,
                                 d_gap + k + it, st, h->potts);
    } else {
      e = launch_dual<double>((const double*)h->d_unaries, (const double*)h->d_tables, (const double*)h->d_phi,
                              h->d_node_ptr, h->d_inc, h->n, h->L, h->m, h->d_node_min, h->d_edge_min, d_gap + it, st);
      if (e == hipSuccess)
        e = launch_decode<double>((const double*)h->d_unaries, (const double*)h->d_tables, (const double*)h->d_phi,
                                  h->d_slots, h->d_node_ptr, h->d_inc, h->n, h->L, h->m, d_lab + (size_t)it * h->n,
                                  d_gap + k + it, st);
    }
    if (e != hipSuccess) {
      release();
      return fail(MPLPXX_EDEVICE, "gap trace: %s", hipGetErrorString(e));
    }
  }
  int rc = sync_and_check(h);
  if (rc != MPLPXX_OK) {
    release();
    return rc;
  }
  std::vector<double> buf((size_t)2 * k);
  hipError_t e = hipMemcpy(buf.data(), d_gap, buf.size() * sizeof(double), hipMemcpyDeviceToHost);
  int best = 0;
  for (int it = 0; it < k; ++it) {
    dual[it] = buf[it];
    energy[it] = buf[k + it];
    if (energy[it] < energy[best]) best = it;
  }
  if (e == hipSuccess && best_labels)
    e = hipMemcpy(best_labels, d_lab + (size_t)best * h->n, (size_t)h->n * sizeof(int), hipMemcpyDeviceToHost);
  release();
  if (e != hipSuccess) return fail(MPLPXX_EDEVICE, "gap trace copy: %s", hipGetErrorString(e));
  return MPLPXX_OK;
}

void mplpxx_destroy(mplpxx_solver* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream());
  if (h->shadow) mplpxx_destroy(h->shadow);
  free_all(h);
  delete h;
}

const char* mplpxx_error_string(int code) {
  switch (code) {
    case MPLPXX_OK: return "ok";
    case MPLPXX_EINVAL: return "invalid argument";
    case MPLPXX_ENOMEM: return "out of memory";
    case MPLPXX_EDEVICE: return "device error";
    case MPLPXX_ETIMEOUT: return "device wait timed out";
    case MPLPXX_ESTATE: return "invalid state";
    default: return "unknown error";
  }
}

const char* mplpxx_last_error(void) { return g_last_error.c_str(); }

int mplpxx_set_stream(mplpxx_solver* h, void* hip_stream) {
  if (!h) return fail(MPLPXX_EINVAL, "handle is NULL");
  HIP_TRY(hipStreamSynchronize(h->stream()));
  h->user_stream = static_cast<hipStream_t>(hip_stream);
  return MPLPXX_OK;
}

int mplpxx_get_schedule(mplpxx_solver* h, int32_t* n_steps, int32_t* step_ptr, int32_t* order) {
  if (!h) return fail(MPLPXX_EINVAL, "handle is NULL");
  if (n_steps) *n_steps = h->S;
  if (step_ptr) std::memcpy(step_ptr, h->step_ptr.data(), h->step_ptr.size() * sizeof(int));
  if (order && h->m) std::memcpy(order, h->order.data(), h->order.size() * sizeof(int));
  return MPLPXX_OK;
}

int mplpxx_schedule(int32_t n, int64_t m, const int32_t* edges, int32_t* n_steps, int32_t* step_ptr,
                    int32_t* order) {
  return mplpxx_schedule_kind(n, m, edges, MPLPXX_SCHED_AUTO, n_steps, step_ptr, order);
}

int mplpxx_schedule_kind(int32_t n, int64_t m, const int32_t* edges, int32_t schedule, int32_t* n_steps,
                         int32_t* step_ptr, int32_t* order) {
  if (schedule != MPLPXX_SCHED_AUTO && schedule != MPLPXX_SCHED_GREEDY && schedule != MPLPXX_SCHED_COLOR)
    return fail(MPLPXX_EINVAL, "unknown schedule kind %d", schedule);
  if (n < 1) return fail(MPLPXX_EINVAL, "n must be >= 1 (got %d)", n);
  if (m < 0 || m > (int64_t)n * (n - 1) / 2 || m > 0x3fffffff)
    return fail(MPLPXX_EINVAL, "m must be in [0, n(n-1)/2] (got %lld)", (long long)m);
  if (m > 0 && !edges) return fail(MPLPXX_EINVAL, "edges is NULL");
  mplpxx_solver tmp;
  tmp.n = n;
  tmp.m = (int)m;
  tmp.sched = schedule;
  int rc = prepare_solver_graph(&tmp, edges);
  if (rc != MPLPXX_OK) return rc;
  if (n_steps) *n_steps = tmp.S;
  if (step_ptr) std::memcpy(step_ptr, tmp.step_ptr.data(), tmp.step_ptr.size() * sizeof(int));
  if (order && m) std::memcpy(order, tmp.order.data(), tmp.order.size() * sizeof(int));
  return MPLPXX_OK;
}

int mplpxx_get_state(mplpxx_solver* h, void* U, void* phi, float* U_comp) {
  if (!h) return fail(MPLPXX_EINVAL, "handle is NULL");
  HIP_TRY(hipStreamSynchronize(h->stream()));
  const size_t esz = h->esz, L = h->L;
  if (U) HIP_TRY(hipMemcpy(U, h->d_U, (size_t)h->n * L * esz, hipMemcpyDeviceToHost));
  if (U_comp) {
    if (h->d_Ulo)
      HIP_TRY(hipMemcpy(U_comp, h->d_Ulo, (size_t)h->n * L * sizeof(float), hipMemcpyDeviceToHost));
    else
      std::fill(U_comp, U_comp + (size_t)h->n * L, 0.0f);
  }
  if (phi && h->m) {
    std::vector<char> tmp((size_t)h->m * 2 * L * esz);
    HIP_TRY(hipMemcpy(tmp.data(), h->d_phi, tmp.size(), hipMemcpyDeviceToHost));
    char* dst = static_cast<char*>(phi);
    const size_t row = 2 * L * esz;
    for (int e = 0; e < h->m; ++e) std::memcpy(dst + (size_t)e * row, tmp.data() + (size_t)h->slot_of_edge[e] * row, row);
  }
  return MPLPXX_OK;
}

int mplpxx_set_state(mplpxx_solver* h, const void* U, const void* phi, const float* U_comp) {
  if (!h) return fail(MPLPXX_EINVAL, "handle is NULL");
  if (U_comp && !U) return fail(MPLPXX_EINVAL, "U_comp needs U");
  if (U_comp && !h->d_Ulo) return fail(MPLPXX_EINVAL, "U_comp is for FP32 handles only");
  HIP_TRY(hipStreamSynchronize(h->stream()));
  const size_t esz = h->esz, L = h->L, nL = (size_t)h->n * L;
  if (U) {
    if (!finite_host(U, nL, h->dtype)) return fail(MPLPXX_EINVAL, "non-finite U");
    if (U_comp && !finite_host(U_comp, nL, MPLPXX_F32)) return fail(MPLPXX_EINVAL, "non-finite U_comp");
    HIP_TRY(hipMemcpyAsync(h->d_U, U, nL * esz, hipMemcpyHostToDevice, h->stream()));
    if (h->d_Ulo) {
      std::vector<float> lo(nL, 0.0f);
      if (U_comp)
        for (size_t i = 0; i < nL; ++i) lo[i] = bf16_round_host(U_comp[i]);
      HIP_TRY(hipMemcpyAsync(h->d_Ulo, lo.data(), nL * sizeof(float), hipMemcpyHostToDevice, h->stream()));
      HIP_TRY(hipStreamSynchronize(h->stream()));
    }
    HIP_TRY(hipStreamSynchronize(h->stream()));
  }
  if (phi && h->m) {
    if (!finite_host(phi, (size_t)h->m * 2 * L, h->dtype)) return fail(MPLPXX_EINVAL, "non-finite phi");
    std::vector<char> tmp((size_t)h->m * 2 * L * esz);
    const char* src = static_cast<const char*>(phi);
    const size_t row = 2 * L * esz;
    for (int e = 0; e < h->m; ++e) std::memcpy(tmp.data() + (size_t)h->slot_of_edge[e] * row, src + (size_t)e * row, row);
    HIP_TRY(hipMemcpyAsync(h->d_phi, tmp.data(), tmp.size(), hipMemcpyHostToDevice, h->stream()));
    HIP_TRY(hipStreamSynchronize(h->stream()));
  }
  h->iterations = 0;
  h->adj_ready = false;
  return MPLPXX_OK;
}

int mplpxx_set_option(mplpxx_solver* h, int32_t key, int64_t value) {
  if (!h) return fail(MPLPXX_EINVAL, "handle is NULL");
  switch (key) {
    case MPLPXX_OPT_ENGINE:
      if (value < 0 || value > 2) return fail(MPLPXX_EINVAL, "engine must be 0, 1 or 2");
      if (h->potts && value == ENGINE_STEP) return fail(MPLPXX_EINVAL, "Potts models run on the persistent engine only");
      h->engine_opt = (int)value;
      return MPLPXX_OK;
    case MPLPXX_OPT_THREADS:
      if (h->potts) {
        if (value != 0 && value != 64 && value != 256)
          return fail(MPLPXX_EINVAL, "structured costs run 64 threads (label order) or 256 (tiles formed from "
                                     "the parameters)");
        h->threads_opt = (int)value;
        return MPLPXX_OK;
      }
      if (value != 0 && !valid_threads(h->LT(), (int)value))
        return fail(MPLPXX_EINVAL, "threads %lld not valid for L=%d", (long long)value, h->L);
      h->threads_opt = (int)value;
      return MPLPXX_OK;
    case MPLPXX_OPT_GRID: {
      if (value < 0) return fail(MPLPXX_EINVAL, "grid must be >= 0");
      const int nb = h->potts && !h->gen_tiles() ? max_blocks_per_cu_mb_potts()
                     : h->mb_engine() ? max_blocks_per_cu_mb(h->LT(), h->NT())
                     : h->dtype == MPLPXX_F32 ? max_blocks_per_cu<float>(ENGINE_PERSISTENT, h->LT(), h->NT())
                                              : max_blocks_per_cu<double>(ENGINE_PERSISTENT, h->LT(), h->NT());
      if (value > (int64_t)nb * h->num_cus) return fail(MPLPXX_EINVAL, "grid %lld exceeds co-resident limit %d", (long long)value, nb * h->num_cus);
      h->grid_opt = (int)value;
      return MPLPXX_OK;
    }
    case MPLPXX_OPT_SPIN_LIMIT:
      if (value < 0) return fail(MPLPXX_EINVAL, "spin limit must be >= 0");
      h->spin_limit = value ? value : (1ll << 22);
      return MPLPXX_OK;
    case MPLPXX_OPT_PROFILE:
      h->profile = value != 0;
      return MPLPXX_OK;
    case MPLPXX_OPT_PHI:
      if (value < 0 || value > 2) return fail(MPLPXX_EINVAL, "phi placement must be 0, 1 or 2");
      h->phi_opt = (int)value;
      return MPLPXX_OK;
    case MPLPXX_OPT_PREFETCH:
      if (value < 0 || value > 2) return fail(MPLPXX_EINVAL, "prefetch must be 0, 1 or 2");
      h->prefetch_opt = (int)value;
      return MPLPXX_OK;
    case MPLPXX_OPT_ADJOINT_F64:
      h->adjoint_f64 = value != 0;
      h->adj_ready = false;
      return MPLPXX_OK;
    case MPLPXX_OPT_RULE:
      if (value != MPLPXX_RULE_H && value != MPLPXX_RULE_M && value != MPLPXX_RULE_U)
        return fail(MPLPXX_EINVAL, "rule must be MPLPXX_RULE_H, _M or _U");
      if (h->potts && value != MPLPXX_RULE_H) return fail(MPLPXX_EINVAL, "Potts models take the (H) update only");
      h->rule = (int)value;
      h->adj_ready = false;
      return MPLPXX_OK;
    default:
      return fail(MPLPXX_EINVAL, "unknown option %d", key);
  }
}

int mplpxx_get_info(mplpxx_solver* h, int32_t key, int64_t* value) {
  if (!h || !value) return fail(MPLPXX_EINVAL, "NULL argument");
  switch (key) {
    case MPLPXX_INFO_N: *value = h->n; return MPLPXX_OK;
    case MPLPXX_INFO_L: *value = h->L; return MPLPXX_OK;
    case MPLPXX_INFO_M: *value = h->m; return MPLPXX_OK;
    case MPLPXX_INFO_STEPS: *value = h->S; return MPLPXX_OK;
    case MPLPXX_INFO_DTYPE: *value = h->dtype; return MPLPXX_OK;
    case MPLPXX_INFO_ENGINE: *value = h->engine(); return MPLPXX_OK;
    case MPLPXX_INFO_GRID: *value = h->grid(); return MPLPXX_OK;
    case MPLPXX_INFO_THREADS: *value = h->NT(); return MPLPXX_OK;
    case MPLPXX_INFO_ITERATIONS: *value = h->iterations; return MPLPXX_OK;
    case MPLPXX_INFO_WALLCLOCK_KHZ: *value = h->wallclock_khz; return MPLPXX_OK;
    case MPLPXX_INFO_ADJOINT_BYTES: {
      // the handle's own adjoint buffers, plus, for an FP32 handle that
      // differentiates its FP64 twin, the twin's costs, state and buffers
      size_t b = h->adj_bytes;
      if (const mplpxx_solver* t = h->shadow)
        b += t->adj_bytes + (size_t)t->n * t->L * 8 * 2 + (size_t)t->m * t->L * t->L * 8 + (size_t)t->m * 2 * t->L * 8;
      *value = (int64_t)b;
      return MPLPXX_OK;
    }
    default: return fail(MPLPXX_EINVAL, "unknown info key %d", key);
  }
}

int mplpxx_get_step_profile(mplpxx_solver* h, int64_t* stamps) {
  if (!h || !stamps) return fail(MPLPXX_EINVAL, "NULL argument");
  if (!h->d_stamps) return fail(MPLPXX_ESTATE, "no profile recorded (set MPLPXX_OPT_PROFILE and iterate first)");
  HIP_TRY(hipStreamSynchronize(h->stream()));
  HIP_TRY(hipMemcpy(stamps, h->d_stamps, (size_t)h->m * kStampStride * sizeof(long long), hipMemcpyDeviceToHost));
  return MPLPXX_OK;
}

int mplpxx_last_iterate_ms(mplpxx_solver* h, double* ms) {
  if (!h || !ms) return fail(MPLPXX_EINVAL, "NULL argument");
  if (h->user_stream && h->timed) {
    HIP_TRY(hipEventSynchronize(h->ev1));
    float f = 0.f;
    HIP_TRY(hipEventElapsedTime(&f, h->ev0, h->ev1));
    h->last_ms = f;
  }
  *ms = h->last_ms;
  return MPLPXX_OK;
}

}  // extern "C"
