// Internal declarations shared by the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mplpxx.h"

namespace mplpxx {

enum { ENGINE_AUTO = 0, ENGINE_STEP = 1, ENGINE_PERSISTENT = 2 };

// Pairwise cost of a model: a dense L x L table per edge, or a structured
// cost given by a few parameters per edge (MPLPXX_COST_* of the header):
// Potts w [s != t] (1 parameter: w), truncated linear w min(|s - t|, tau)
// and truncated quadratic w min((s - t)^2, tau) (2 parameters: w, tau).  The
// parameters of slot i sit at tables[i * cost_params(kind)].
constexpr int kCostDense = 0;
__host__ __device__ constexpr int cost_params(int kind) {
  return kind == MPLPXX_COST_TRUNC_LINEAR || kind == MPLPXX_COST_TRUNC_QUAD ? 2 : 1;
}
// fl(w * min(d, tau)) for a distance term d that is exact in FP32: the
// entry of the expanded table of the truncated kinds
__host__ __device__ inline float truncated_cost(float w, float tau, float d) { return w * (d < tau ? d : tau); }
// th(s, t) of a structured cost from its parameters (the expanded table)
__host__ __device__ inline float structured_cost(int kind, const float* prm, int s, int t) {
  if (kind == MPLPXX_COST_TRUNC_LINEAR || kind == MPLPXX_COST_TRUNC_QUAD) {
    const float d = (float)(s > t ? s - t : t - s);
    return truncated_cost(prm[0], prm[1], kind == MPLPXX_COST_TRUNC_QUAD ? d * d : d);
  }
  return s == t ? 0.0f : prm[0];
}

// timestamps per slot: 4 in normal builds; a diagnostics build
// (-DMPLPXX_FINE_STAMPS=1) records 4 more points inside the edge update
#ifndef MPLPXX_FINE_STAMPS
#define MPLPXX_FINE_STAMPS 0
#endif
constexpr int kStampStride = MPLPXX_FINE_STAMPS ? 8 : 4;

// One entry per schedule slot (slot i = i-th edge of the schedule queue).
// Elements allocated (zeroed) past the end of every tables and messages
// array: the FP32 engines load whole tile rows without clamping the column
// index, so a row of a table (or of a slot's messages) may read up to LT
// elements into whatever follows it.
constexpr size_t kTailPad = 256;

struct SlotInfo {
  int e;       // index of the edge in the caller's edge list
  int u, v;    // its nodes, u < v
  int pos_u;   // number of edges of u that precede this one in the queue
  int pos_v;   // same for v
  int deg_u;   // degree of u (updates of u per iteration)
  int deg_v;   // degree of v
  int step;    // index of its matching in the schedule
};

template <typename T> struct HsArgs {
  const T* tables;        // [m][L][L] slot order, read-only (Potts models: [m] weights)
  T* phi;                 // [m][2][L] slot order
  T* U;                   // [n][L]
  T* Ulo;                 // [n][L] FP32 only: bf16 correction of U (U = U + Ulo), else null
  const SlotInfo* slots;  // [m]
  const int* deg;         // [n]
  int* ver;               // [n] per-node update counters (persistent engine)
  int* err;               // device error word
  double* trace;          // [iters][n] per-node minima after the node's last update, or null
  float* trace_e;         // [iters][m][W] FP32 mailbox engine: per-wave minima of the edge terms, or null
  long long* stamps;      // [m][4] wall-clock stamps of the last iteration, or null
  unsigned long long* sink;  // FP32 mailbox engine: [grid][NT + 128] scratch words
  int L, m, n;
  long long spin_limit;
};

// ---------------------------------------------------------------------------
// Batched engine: many independent FP32 models in one persistent launch.
// ---------------------------------------------------------------------------
struct BatchModel {
  long long table_off;  // floats into the concatenated tables
  long long phi_off;    // floats into the concatenated messages
  long long u_off;      // entries into U / mailboxes / unaries (n*L per model)
  int slot_off;         // first slot of the model in the concatenated SlotInfo
  int node_off;         // first node of the model (degrees, node maps)
  int n, L, m, lt;      // sizes and register tile (16, 32, 64 or 128)
  int csr_off;          // first node_ptr entry (n+1 per model)
  int inc_off;          // first incidence entry (2m per model)
  int potts;            // cost kind (0 dense; MPLPXX_COST_*: parameters per slot at table_off + slot * cost_params)
};
struct BatchTask {
  int model;   // which model
  int first;   // first slot of the model this workgroup owns
  int stride;  // team size: the workgroup owns slots first, first+stride, ...
  int lds;     // 1: a whole model whose unaries live in this workgroup's LDS for the launch
};
struct BatchArgs {
  const float* tables;
  float* phi;
  unsigned long long* mb;
  const SlotInfo* slots;
  const int* deg;
  const BatchModel* models;
  const BatchTask* tasks;
  const int* task_ptr;    // [G+1] task range of each logical workgroup
  int* ticket;            // [0] start-order counter, [1] queue head (both zeroed before each launch)
  int qbegin, qlen;       // tasks[qbegin, qbegin + qlen): single-workgroup tasks taken in order by free workgroups
  unsigned long long* sink;  // scratch words of the workgroups (stores of lanes without an output)
  long long* wg_time;        // [grid][2] start and end clock of each logical workgroup
  int* err;
  long long spin_limit;
};
hipError_t launch_batch(const BatchArgs& b, int max_lt, int grid, int iters, size_t dyn_lds, hipStream_t st);
int batch_blocks_per_cu(int max_lt, size_t dyn_lds);
size_t batch_lds_limit(int max_lt);
// LDS-resident unaries of one model in the batched engine: n*L hi values
// (FP32), then, from this byte offset, n*L bf16 corrections
__host__ __device__ inline size_t lds_lo_offset(int n, int L) { return ((size_t)n * L * 4 + 15) / 16 * 16; }
__host__ __device__ inline size_t lds_model_bytes(int n, int L) { return lds_lo_offset(n, L) + (size_t)n * L * 2; }
hipError_t launch_u_to_mb(const float* U, const float* Ulo, unsigned long long* mb, size_t count, hipStream_t st);
hipError_t launch_mb_to_u(float* U, float* Ulo, const unsigned long long* mb, size_t count, hipStream_t st);
hipError_t launch_batch_dual(const float* unaries, const float* tables, const float* phi, const BatchModel* models,
                             const int* node_model, const int* slot_model, const int* node_ptr, const int* inc,
                             int total_nodes, int total_slots, int count, double* node_min, double* edge_min,
                             double* out, hipStream_t st);

// adjoint (adjoint.hip)
template <typename T>
hipError_t launch_step_record(const T* tables, T* phi, T* U, T* Ulo, const SlotInfo* slots, int L, int slot_begin,
                              int count, unsigned char* rec, hipStream_t st);
template <typename T>
hipError_t launch_adj_step(const SlotInfo* slots, int L, int slot_begin, int count, const unsigned char* rec, T* Ub,
                           T* pb, T* thb, hipStream_t st);
template <typename T>
hipError_t launch_adj_seed(const T* U, const T* Ulo, int n, int L, T* Ub, double* node_min, hipStream_t st);
// persistent FP64 adjoint, L <= 64 (adjoint.hip): values in mailboxes of two
// tagged 64-bit words per label (mb[n][L][2]); rec = nullptr: plain forward
hipError_t launch_mb64_init(const double* x, unsigned long long* mb, size_t count, hipStream_t st);
hipError_t launch_mb64_fini(double* x, const unsigned long long* mb, size_t count, hipStream_t st);
// one launch: the reverse of `seg` recorded iterations (rev_grid workgroups,
// 0 for none) beside the forward of `iters` iterations (fwd_grid
// workgroups; fwd_rec: argmin records, or null), then the reverse
// segment's table adjoints
hipError_t launch_adj64(const double* tables, double* phi, unsigned long long* mb_fwd, int iters, unsigned char* fwd_rec,
                        int fwd_grid, const unsigned char* rev_rec, unsigned long long* mb_rev, double* pb,
                        double* contrib, double* thb, int seg, int rev_grid, const SlotInfo* slots, int L, int m,
                        int* err, long long spin_limit, hipStream_t st);

int max_blocks_per_cu_mb(int LT, int NT);
// the (M) and (U) updates on the per-matching engine (rules.hip); rule 1 = M, 2 = U
template <typename T>
hipError_t launch_step_rule(const HsArgs<T>& a, int rule, int LT, int NT, int slot_begin, int count, hipStream_t st);
template <typename T>
hipError_t launch_handshake(const HsArgs<T>& a, int engine, int LT, int NT, int slot_begin, int count, int grid,
                            int iters, hipStream_t st);
template <typename T> int max_blocks_per_cu(int engine, int LT, int NT);
// FP32 persistent engine with tagged mailboxes
// prefetch: steps the tables are loaded ahead (0 the default: 2 for tiles up
// to 64, 1 for 128; 1: one step, for tiles up to 64 without a trace)
// kind: a structured cost (MPLPXX_COST_*, NT = 256, LT <= 64) whose tiles
// are formed from the slots' parameters
// rule: MPLPXX_RULE_H, or MPLPXX_RULE_M / _U (dense tables, NT = 256, no trace)
hipError_t launch_persistent_mb(const HsArgs<float>& a, unsigned long long* mb, int LT, int NT, int grid, int iters,
                                int phi_in_lds, size_t dyn_lds, hipStream_t st, int prefetch = 0, int kind = 0,
                                int rule = 0);
// the same for Potts models (one weight per slot, L <= 64; potts_mb.h)
int max_blocks_per_cu_mb_potts();
hipError_t launch_persistent_mb_potts(const HsArgs<float>& a, unsigned long long* mb, int grid, int iters,
                                      int phi_in_lds, size_t dyn_lds, hipStream_t st, int kind = MPLPXX_COST_POTTS);
hipError_t launch_mb_init(const float* U, const float* Ulo, unsigned long long* mb, size_t count, hipStream_t st);
hipError_t launch_mb_fini(float* U, float* Ulo, const unsigned long long* mb, int n, int L, double* trace_row,
                          hipStream_t st);

// dual bound, traces, decode (dual.hip)
template <typename T>
hipError_t launch_dual(const T* unaries, const T* tables, const T* phi, const int* node_ptr, const int* inc, int n,
                       int L, int m, double* node_min, double* edge_min, double* out, hipStream_t st, int potts = 0);
template <typename T>
hipError_t launch_trace_nodes(const T* U, const T* Ulo, int n, int L, double* row, hipStream_t st);
template <typename T>
hipError_t launch_trace_edges(const T* tables, const T* phi, int m, int L, float* out, hipStream_t st);
template <typename T>
hipError_t launch_trace_sum(double* trace_nodes, const float* trace_e, int m, int W, const T* U, const int* deg, int n,
                            int L, int iters, double* out,
                            hipStream_t st);
template <typename T>
hipError_t launch_decode(const T* unaries, const T* tables, const T* phi, const SlotInfo* slots, const int* node_ptr,
                         const int* inc, int n, int L, int m, int* labels, double* energy, hipStream_t st,
                         int potts = 0);
template <typename T>
hipError_t launch_check_finite(const T* p, size_t count, int* flag, hipStream_t st);
template <typename T>
hipError_t launch_pack_tables(const T* src, T* dst, const int* slot_edge, const int* slot_flip, int m, int L,
                              hipStream_t st);
hipError_t launch_fill_int(int* p, int value, size_t count, hipStream_t st);
hipError_t launch_convert(const float* src, double* dst, size_t count, hipStream_t st);
hipError_t launch_convert(const double* src, float* dst, size_t count, hipStream_t st);

}  // namespace mplpxx
