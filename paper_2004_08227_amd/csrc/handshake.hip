// Handshake (H) edge-block update of MPLP++ on gfx950.
//
// Paper: Tourani et al., "MPLP++: Fast, Parallel Dual Block-Coordinate Ascent
// for Dense Graphical Models", ECCV 2018, Sec. 4 (updates (M), (H) and the
// "message passing" subroutine) and Sec. 6 (parallel processing of the edges
// of one matching, a barrier between consecutive matchings).
//
// State kept per model (all device memory):
//   tables  [m][L][L]  input pairwise costs, read-only, packed in schedule
//                      order (slot i holds edge order[i]);
//   phi     [m][2][L]  messages of the edge in slot i: phi[i][0] into the
//                      lower node u, phi[i][1] into the upper node v;
//   U       [n][L]     reparametrized unaries theta^phi_u.
//
// One (H) update of edge (u, v) with original table th.  The aggregated cost
// of Sec. 4 is g(s,t) = th(s,t) + a_u(s) + a_v(t) with a_u = U_u - phi[0] and
// a_v = U_v - phi[1].  Evaluating (H) on g with the three-minimization form
// the paper gives right after (H):
//   p(s) = min_t [th(s,t) + a_v(t)]           MPLP half for u: (a_u + p) / 2
//   b(s) = (a_u(s) - p(s)) / 2                so that a_u - theta^H_u = b
//   q(t) = min_s [th(s,t) + b(s)]             theta^H_v = a_v + q
//   r(s) = min_t [th(s,t) - q(t)]             theta^H_u = a_u + r
//   phi[1] := q, phi[0] := r, U_v := a_v + q, U_u := a_u + r.
// Each pass is the paper's message-passing primitive min_t [th(s,t) + x(t)]
// with the table fixed, so the tables are never written.
//
// Work mapping: one workgroup per edge update.  The L x L table (padded to
// an LT x LT tile, pads = +inf) lives in registers as a grid of
// RB x 16 thread blocks; thread (rb, cb) holds rows rb*BR .. rb*BR+BR-1 and
// columns cb*BC .. cb*BC+BC-1.  Row minima reduce across the 16 lanes of a
// DPP row, column minima across the RB row blocks (lanes 16 and 32 apart,
// then across waves through LDS).  Every entry of a pass is one IEEE add
// followed by an exact minimum, so results do not depend on LT, NT, the
// reduction tree or the engine.
#include <algorithm>
#include <type_traits>

#include "step_common.h"
#include "potts_mb.h"

namespace mplpxx {
// The three passes on a register tile; a_u / a_v must be in smem.  Writes
// the new messages and unaries to global memory (coherent stores when
// `shared_nodes`).  Returns after all writes of this workgroup completed.
template <typename T, int LT, int NT, bool kCoherent>
__device__ __forceinline__ void handshake_passes(const T (&x)[TileShape<T, LT, NT>::BR][TileShape<T, LT, NT>::BC],
                                                 Smem<T, LT, NT>& sm, int L, T* __restrict__ phi_slot,
                                                 T* __restrict__ Uu, T* __restrict__ Uv, T* __restrict__ Lu,
                                                 T* __restrict__ Lv, bool keep_new) {
  using S = TileShape<T, LT, NT>;
  const int tid = threadIdx.x;
  const int rb = tid >> 4, cb = tid & 15;
  const int wave = tid >> 6;
  const int lane = tid & 63;

  T av[S::BC];
#pragma unroll
  for (int j = 0; j < S::BC; ++j) {
    const int t = cb * S::BC + j;
    av[j] = (t < L) ? sm.av[t] : T(0);
  }
  // pass 1: p(s) = min_t [th(s,t) + a_v(t)],  b(s) = (a_u(s) - p(s)) / 2
  T b[S::BR];
#pragma unroll
  for (int i = 0; i < S::BR; ++i) {
    T mn = x[i][0] + av[0];
#pragma unroll
    for (int j = 1; j < S::BC; ++j) mn = vmin(mn, x[i][j] + av[j]);
    mn = row16_min(mn);
    const int s = rb * S::BR + i;
    b[i] = (s < L) ? T(0.5) * (sm.au[s] - mn) : T(0);
  }
  // pass 2: q(t) = min_s [th(s,t) + b(s)]
  T q[S::BC];
#pragma unroll
  for (int j = 0; j < S::BC; ++j) {
    T mn = x[0][j] + b[0];
#pragma unroll
    for (int i = 1; i < S::BR; ++i) mn = vmin(mn, x[i][j] + b[i]);
    mn = col4_min(mn);
    q[j] = mn;
  }
  if constexpr (S::W > 1) {
    if (lane < 16) {
#pragma unroll
      for (int j = 0; j < S::BC; ++j) sm.red[wave][cb * S::BC + j] = q[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < S::BC; ++j) {
      const int t = cb * S::BC + j;
      T mn = sm.red[0][t];
#pragma unroll
      for (int w = 1; w < S::W; ++w) mn = vmin(mn, sm.red[w][t]);
      q[j] = mn;
    }
  }
#pragma unroll
  for (int j = 0; j < S::BC; ++j) {
    const int t = cb * S::BC + j;
    if (t >= L) q[j] = T(0);
  }
  // pass 3: r(s) = min_t [th(s,t) - q(t)]
  T r[S::BR];
#pragma unroll
  for (int i = 0; i < S::BR; ++i) {
    T mn = x[i][0] - q[0];
#pragma unroll
    for (int j = 1; j < S::BC; ++j) mn = vmin(mn, x[i][j] - q[j]);
    r[i] = row16_min(mn);
  }
  // push back: phi[1] = q, U_v = a_v + q (threads of row block 0);
  //            phi[0] = r, U_u = a_u + r (threads of column block 0)
  // (FP32: centred passes shifted back by delta, compensated U + Ulo, see
  // device_common.h; FP64: plain, one rounding)
  T delta = T(0);
  if constexpr (kComp<T>) delta = T(0.5) * (sm.cu - sm.cv);
  if (rb == 0) {
#pragma unroll
    for (int j = 0; j < S::BC; ++j) {
      const int t = cb * S::BC + j;
      if (t < L) {
        T nvv, nvl = T(0);
        const T qs = q[j] + delta;
        if constexpr (kComp<T>) comp_update(sm.hv[t], sm.lv[t], sm.ov[t], qs, nvv, nvl);
        else nvv = av[j] + q[j];
        phi_slot[L + t] = qs;
        if (kCoherent) stv_dev(Uv + t, nvv); else Uv[t] = nvv;
        if constexpr (kComp<T>) { if (kCoherent) stv_dev(Lv + t, nvl); else Lv[t] = nvl; }
        if (keep_new) sm.nv[t] = nvv + nvl;
      }
    }
  }
  if (cb == 0) {
#pragma unroll
    for (int i = 0; i < S::BR; ++i) {
      const int s = rb * S::BR + i;
      if (s < L) {
        T nuu, nul = T(0);
        const T rs = r[i] - delta;
        if constexpr (kComp<T>) comp_update(sm.hu[s], sm.lu[s], sm.ou[s], rs, nuu, nul);
        else nuu = sm.au[s] + r[i];
        phi_slot[s] = rs;
        if (kCoherent) stv_dev(Uu + s, nuu); else Uu[s] = nuu;
        if constexpr (kComp<T>) { if (kCoherent) stv_dev(Lu + s, nul); else Lu[s] = nul; }
        if (keep_new) sm.nu[s] = nuu + nul;
      }
    }
  }
  __syncthreads();
}

// min over the L entries of sm.nu / sm.nv in FP64 (wave `w` of the block),
// written by its lane 0
template <typename T, int LT, int NT>
__device__ __forceinline__ void node_min_to(const T* v, int L, double* out) {
  const int lane = threadIdx.x & 63;
  double mn = __builtin_inf();
  for (int s = lane; s < L; s += 64) mn = __builtin_fmin(mn, (double)v[s]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mn = __builtin_fmin(mn, __shfl_xor(mn, o, 64));
  if (lane == 0) *out = mn;
}

// ---------------------------------------------------------------------------
// Engine 1: one launch per matching.  Grid = edges of the matching.  Kernel
// boundaries order the matchings (the paper's barrier between matchings).
// ---------------------------------------------------------------------------
template <typename T, int LT, int NT>
__global__ void __launch_bounds__(NT) k_step(HsArgs<T> a, int slot_begin) {
  using S = TileShape<T, LT, NT>;
  __shared__ Smem<T, LT, NT> sm;
  const int slot = slot_begin + blockIdx.x;
  const SlotInfo si = a.slots[slot];
  const int L = a.L;
  T x[S::BR][S::BC];
  load_tile<T, LT, NT>(a.tables + (size_t)slot * L * L, L, x);
  T* phi_slot = a.phi + (size_t)slot * 2 * L;
  T* Uu = a.U + (size_t)si.u * L;
  T* Uv = a.U + (size_t)si.v * L;
  T* Lu = a.Ulo ? a.Ulo + (size_t)si.u * L : nullptr;
  T* Lv = a.Ulo ? a.Ulo + (size_t)si.v * L : nullptr;
  gather<T, LT, NT, false>(sm, L, phi_slot, Uu, Uv, Lu, Lv);
  handshake_passes<T, LT, NT, false>(x, sm, L, phi_slot, Uu, Uv, Lu, Lv, false);
}

// ---------------------------------------------------------------------------
// Engine 2: persistent.  Workgroup w owns the slots w, w+G, w+2G, ... (a
// static map, so an edge's messages never leave one workgroup) and visits
// them in schedule order for every iteration.  Before updating edge (u, v) it
// waits until u and v have seen exactly the updates that precede this one in
// the schedule (per-node version counters); afterwards it publishes the new
// unaries and bumps both versions.  This is the paper's barrier between
// matchings reduced to the two nodes an edge depends on.  The versions carry
// the ordering: thread 0 stores them after the workgroup barrier that ends
// the passes (so every thread's unary stores happen before it) and a
// device-scope release; a waiter reads one with relaxed polls followed by a
// device-scope acquire, before the barrier that lets its workgroup read the
// unaries.
// ---------------------------------------------------------------------------
template <typename T, int LT, int NT>
__global__ void __launch_bounds__(NT) k_persistent(HsArgs<T> a, int iters) {
  using S = TileShape<T, LT, NT>;
  __shared__ Smem<T, LT, NT> sm;
  const int tid = threadIdx.x;
  const int L = a.L;
  const int G = gridDim.x;
  if (tid == 0) sm.abort_flag = 0;
  __syncthreads();
  int slot = blockIdx.x;
  if (slot >= a.m) return;
  T x[S::BR][S::BC];
  load_tile<T, LT, NT>(a.tables + (size_t)slot * L * L, L, x);
  for (int it = 0; it < iters; ++it) {
    for (slot = blockIdx.x; slot < a.m; slot += G) {
      const SlotInfo si = a.slots[slot];
      // wait for the two nodes (thread 0: u, thread 64 or 1: v)
      const int waiter_v = (NT >= 128) ? 64 : 1;
      if (tid == 0 || tid == waiter_v) {
        const int node = (tid == 0) ? si.u : si.v;
        // (counts modulo 2^32; a waiter is fewer than deg updates behind, so
        // the signed difference orders them)
        const unsigned want = (unsigned)it * (unsigned)a.deg[node] + (unsigned)((tid == 0) ? si.pos_u : si.pos_v);
        long long spins = 0;
        while ((int)((unsigned)ld_dev(a.ver + node) - want) < 0) {
          if (++spins > a.spin_limit || ((spins & 1023) == 0 && ld_dev(a.err) != 0)) {
            atomicCAS(a.err, 0, MPLPXX_ETIMEOUT);
            sm.abort_flag = 1;
            break;
          }
        }
        // acquire at device scope: the unaries published before the
        // version this wait saw are read after it (the barrier below
        // orders every other thread's reads after this fence)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      __syncthreads();
      if (sm.abort_flag) return;
      T* phi_slot = a.phi + (size_t)slot * 2 * L;
      T* Uu = a.U + (size_t)si.u * L;
      T* Uv = a.U + (size_t)si.v * L;
      T* Lu = a.Ulo ? a.Ulo + (size_t)si.u * L : nullptr;
      T* Lv = a.Ulo ? a.Ulo + (size_t)si.v * L : nullptr;
      gather<T, LT, NT, true>(sm, L, phi_slot, Uu, Uv, Lu, Lv);
      const bool last_u = a.trace && si.pos_u == a.deg[si.u] - 1;
      const bool last_v = a.trace && si.pos_v == a.deg[si.v] - 1;
      handshake_passes<T, LT, NT, true>(x, sm, L, phi_slot, Uu, Uv, Lu, Lv, last_u || last_v);
      if (tid == 0) {
        // release at device scope, then the two versions: a waiter that
        // reads either one and acquires sees every unary this workgroup
        // wrote before the barrier at the end of the passes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        st_dev(a.ver + si.u, (int)((unsigned)it * (unsigned)a.deg[si.u] + (unsigned)si.pos_u + 1u));
        st_dev(a.ver + si.v, (int)((unsigned)it * (unsigned)a.deg[si.v] + (unsigned)si.pos_v + 1u));
      }
      // next table of this workgroup (the same slot again in the next
      // iteration when it owns a single slot)
      int nxt = slot + G;
      if (nxt >= a.m) nxt = blockIdx.x;
      if (nxt != slot && (it + 1 < iters || nxt > slot)) load_tile<T, LT, NT>(a.tables + (size_t)nxt * L * L, L, x);
      if (last_u && (tid >> 6) == 0) node_min_to<T, LT, NT>(sm.nu, L, a.trace + (size_t)it * a.n + si.u);
      if (last_v && (tid >> 6) == (S::W > 1 ? 1 : 0)) node_min_to<T, LT, NT>(sm.nv, L, a.trace + (size_t)it * a.n + si.v);
      __syncthreads();
    }
  }
}

template <int LT, int NT, bool PHI_LDS, bool FULL, bool TRACE, bool PHI_FAR, int DEPTH = (LT <= 64 ? 2 : 1),
          int KIND = kCostDense, int RULE = MPLPXX_RULE_H>
__global__ void __launch_bounds__(NT + 128) k_persistent_mb(HsArgs<float> a, unsigned long long* __restrict__ mb,
                                                            int iters) {
  __shared__ SmemMB<LT, NT> sm;
  extern __shared__ float phi_lds[];
  const int tid = threadIdx.x;
  const int L = FULL ? LT : a.L;
  const int G = gridDim.x;
  if ((int)blockIdx.x >= a.m) return;
  if (tid == 0) sm.abort_flag = 0;
  if (PHI_LDS) {
    for (int slot = blockIdx.x, j = 0; slot < a.m; slot += G, ++j)
      for (int k = tid; k < 2 * L; k += NT + 128) phi_lds[j * 2 * L + k] = a.phi[(size_t)slot * 2 * L + k];
  }
  __syncthreads();
  MbView v{a.tables, a.phi, mb, a.slots, a.deg, a.trace, a.trace_e, a.stamps, L, a.m, a.n, nullptr, nullptr,
           a.sink + (size_t)blockIdx.x * (NT + 128)};
  if (!mb_run<LT, NT, PHI_LDS, FULL, TRACE, false, PHI_FAR, DEPTH, KIND, RULE>(v, blockIdx.x, G, iters, sm, phi_lds,
                                                                         a.spin_limit, a.err))
    return;
  __syncthreads();
  if (PHI_LDS) {
    for (int slot = blockIdx.x, j = 0; slot < a.m; slot += G, ++j)
      for (int k = tid; k < 2 * L; k += NT + 128) a.phi[(size_t)slot * 2 * L + k] = phi_lds[j * 2 * L + k];
  }
}

// Potts models (one weight per slot, L <= 64): one compute wave in label
// order plus the two sync waves (potts_mb.h)
template <bool PHI_LDS, int KIND>
__global__ void __launch_bounds__(kPottsNT + 128) k_persistent_mb_potts(HsArgs<float> a, unsigned long long* __restrict__ mb,
                                                                       int iters) {
  __shared__ SmemMB<64, kPottsNT> sm;
  extern __shared__ float phi_lds[];
  const int tid = threadIdx.x;
  const int L = a.L;
  const int G = gridDim.x;
  if ((int)blockIdx.x >= a.m) return;
  if (tid == 0) sm.abort_flag = 0;
  if (PHI_LDS) {
    for (int slot = blockIdx.x, j = 0; slot < a.m; slot += G, ++j)
      for (int k = tid; k < 2 * L; k += kPottsNT + 128) phi_lds[j * 2 * L + k] = a.phi[(size_t)slot * 2 * L + k];
  }
  __syncthreads();
  MbView v{a.tables, a.phi, mb, a.slots, a.deg, nullptr, nullptr, a.stamps, L, a.m, a.n, nullptr, nullptr,
           a.sink + (size_t)blockIdx.x * (kPottsNT + 128)};
  if (!mb_run_potts<PHI_LDS, KIND>(v, blockIdx.x, G, iters, sm, phi_lds, a.spin_limit, a.err)) return;
  __syncthreads();
  if (PHI_LDS) {
    for (int slot = blockIdx.x, j = 0; slot < a.m; slot += G, ++j)
      for (int k = tid; k < 2 * L; k += kPottsNT + 128) a.phi[(size_t)slot * 2 * L + k] = phi_lds[j * 2 * L + k];
  }
}

// mailbox <- (U, Ulo, version 0)
__global__ void k_mb_init(const float* __restrict__ U, const float* __restrict__ Ulo,
                          unsigned long long* __restrict__ mb, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    mb[i] = mb_pack(U[i], Ulo[i], 0u);
}

// U, Ulo <- mailbox values; trace row of the last iteration from the final values
__global__ void k_mb_fini(float* __restrict__ U, float* __restrict__ Ulo, const unsigned long long* __restrict__ mb,
                          int n, int L, double* __restrict__ trace_row) {
  const int u = blockIdx.x;
  double mn = __builtin_inf();
  for (int s = threadIdx.x; s < L; s += 64) {
    const unsigned long long w = mb[(size_t)u * L + s];
    U[(size_t)u * L + s] = mb_hi(w);
    Ulo[(size_t)u * L + s] = mb_lo(w);
    mn = __builtin_fmin(mn, (double)mb_hi(w) + (double)mb_lo(w));
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mn = __builtin_fmin(mn, __shfl_xor(mn, o, 64));
  if (trace_row && threadIdx.x == 0) trace_row[u] = mn;
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <typename T, int LT, int NT>
static hipError_t launch_one(const HsArgs<T>& a, int engine, int slot_begin, int count, int grid, int iters,
                             hipStream_t st) {
  if (engine == ENGINE_STEP) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_step<T, LT, NT>), dim3(count), dim3(NT), 0, st, a, slot_begin);
    return hipGetLastError();
  }
  void* args[] = {(void*)&a, (void*)&iters};
  const hipError_t e = hipLaunchCooperativeKernel((const void*)k_persistent<T, LT, NT>, dim3(grid), dim3(NT), args, 0, st);
  if (e != hipSuccess) (void)hipGetLastError();  // (see launch_mb_one)
  return e;
}

// structured costs on the dense mailbox engine, the tiles formed from the
// slots' parameters (TRACE off, default prefetch)
template <int LT, int NT, int KIND>
static const void* mb_gen_kernel(bool phi_in_lds, bool full, bool far) {
#define MPLPXX_G(P, F, A) (const void*)k_persistent_mb<LT, NT, P, F, false, A, (LT <= 64 ? 2 : 1), KIND>
  return phi_in_lds ? (full ? (far ? MPLPXX_G(true, true, true) : MPLPXX_G(true, true, false))
                            : (far ? MPLPXX_G(true, false, true) : MPLPXX_G(true, false, false)))
                    : (full ? (far ? MPLPXX_G(false, true, true) : MPLPXX_G(false, true, false))
                            : (far ? MPLPXX_G(false, false, true) : MPLPXX_G(false, false, false)));
#undef MPLPXX_G
}

// the (M) and (U) updates on the dense engine (four compute waves, no trace)
template <int LT, int RULE>
static const void* mb_rule_kernel(bool phi_in_lds, bool full, bool far) {
#define MPLPXX_G(P, F, A) (const void*)k_persistent_mb<LT, 256, P, F, false, A, (LT <= 64 ? 2 : 1), kCostDense, RULE>
  return phi_in_lds ? (full ? (far ? MPLPXX_G(true, true, true) : MPLPXX_G(true, true, false))
                            : (far ? MPLPXX_G(true, false, true) : MPLPXX_G(true, false, false)))
                    : (full ? (far ? MPLPXX_G(false, true, true) : MPLPXX_G(false, true, false))
                            : (far ? MPLPXX_G(false, false, true) : MPLPXX_G(false, false, false)));
#undef MPLPXX_G
}

template <int LT, int NT>
static hipError_t launch_mb_one(const HsArgs<float>& a, unsigned long long* mb, int grid, int iters, int phi_in_lds,
                                size_t dyn_lds, hipStream_t st, int prefetch, int kind, int rule) {
  void* args[] = {(void*)&a, (void*)&mb, (void*)&iters};
  if (rule != MPLPXX_RULE_H) {
    if constexpr (NT == 256) {
      if ((rule != MPLPXX_RULE_M && rule != MPLPXX_RULE_U) || kind != kCostDense || a.trace)
        return hipErrorInvalidValue;
      const bool far = (a.m / grid) >= (LT <= 64 ? 2 : 1) + 2;
      const void* f = rule == MPLPXX_RULE_M ? mb_rule_kernel<LT, MPLPXX_RULE_M>(phi_in_lds, a.L == LT, far)
                                            : mb_rule_kernel<LT, MPLPXX_RULE_U>(phi_in_lds, a.L == LT, far);
      const hipError_t e = hipLaunchCooperativeKernel(f, dim3(grid), dim3(NT + 128), args, dyn_lds, st);
      if (e != hipSuccess) (void)hipGetLastError();
      return e;
    }
    return hipErrorInvalidValue;
  }
  if (kind != kCostDense) {
    // (four compute waves up to 64 labels; one compute wave at 16 labels)
    if constexpr ((NT == 256 && LT <= 64) || (NT == 64 && LT == 16)) {
      const bool far = (a.m / grid) >= 4;
      const void* f = kind == MPLPXX_COST_POTTS ? mb_gen_kernel<LT, NT, MPLPXX_COST_POTTS>(phi_in_lds, a.L == LT, far)
                      : kind == MPLPXX_COST_TRUNC_LINEAR
                          ? mb_gen_kernel<LT, NT, MPLPXX_COST_TRUNC_LINEAR>(phi_in_lds, a.L == LT, far)
                          : mb_gen_kernel<LT, NT, MPLPXX_COST_TRUNC_QUAD>(phi_in_lds, a.L == LT, far);
      const hipError_t e = hipLaunchCooperativeKernel(f, dim3(grid), dim3(NT + 128), args, dyn_lds, st);
      if (e != hipSuccess) (void)hipGetLastError();
      return e;
    }
    return hipErrorInvalidValue;
  }
  const bool full = a.L == LT;
  // tables prefetched DEPTH steps ahead (2 for tiles up to 64 unless one
  // step is asked for; 1 for 128 and for traces); messages prefetched with
  // them when every workgroup owns at least DEPTH + 2 slots
  const int depth = (LT <= 64 && !a.trace && prefetch != 1) || (LT <= 64 && a.trace) ? 2 : 1;
  const bool far = (a.m / grid) >= depth + 2;
#define MPLPXX_PICK(TR, FA, D)                                                                       \
  (phi_in_lds ? (full ? (const void*)k_persistent_mb<LT, NT, true, true, TR, FA, D>                  \
                      : (const void*)k_persistent_mb<LT, NT, true, false, TR, FA, D>)                \
              : (full ? (const void*)k_persistent_mb<LT, NT, false, true, TR, FA, D>                 \
                      : (const void*)k_persistent_mb<LT, NT, false, false, TR, FA, D>))
  constexpr int D0 = LT <= 64 ? 2 : 1;
  const void* f = a.trace ? (far ? MPLPXX_PICK(true, true, D0) : MPLPXX_PICK(true, false, D0))
                  : depth == D0 ? (far ? MPLPXX_PICK(false, true, D0) : MPLPXX_PICK(false, false, D0))
                                : (far ? MPLPXX_PICK(false, true, 1) : MPLPXX_PICK(false, false, 1));
#undef MPLPXX_PICK
  const hipError_t e = hipLaunchCooperativeKernel(f, dim3(grid), dim3(NT + 128), args, dyn_lds, st);
  // a refused launch returns its error here; clear the runtime's copy so
  // that it is not reported again by the next call's error check
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}

// Workgroups of a persistent kernel that the dispatcher can always place on
// one compute unit together.  The occupancy query assumes a workgroup's
// waves spread evenly over the four SIMDs; a placement may put ceil(W/4) of
// its W waves on one SIMD, so at most (waves one SIMD holds) / ceil(W/4)
// workgroups are certain to be resident at once.  A cooperative launch
// beyond that can leave workgroups waiting for a free slot that persistent
// workgroups never release.
static int placeable_per_cu(const void* f, int threads, int nb) {
  int one_wave = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&one_wave, f, 64, 0) != hipSuccess) {
    (void)hipGetLastError();  // (not left for a later launch check)
    return nb;
  }
  if (one_wave < 4) return nb;
  const int per_simd = one_wave / 4;
  const int per_wg = ((threads + 63) / 64 + 3) / 4;
  return std::min(nb, std::max(1, per_simd / per_wg));
}

// workgroups of the FP32 mailbox kernel that fit on one compute unit (no
// dynamic LDS)
int max_blocks_per_cu_mb(int LT, int NT) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define MPLPXX_CASE(lt, nt)                                                                                  \
  if (LT == lt && NT == nt) {                                                                                \
    const void* f = (const void*)k_persistent_mb<lt, nt, false, false, false, true>;                         \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, nt + 128, 0);                                   \
    if (e == hipSuccess) nb = placeable_per_cu(f, nt + 128, nb);                                             \
  }
  MPLPXX_CASE(16, 64)
  MPLPXX_CASE(16, 256)
  MPLPXX_CASE(32, 64)
  MPLPXX_CASE(32, 256)
  MPLPXX_CASE(32, 512)
  MPLPXX_CASE(64, 256)
  MPLPXX_CASE(64, 512)
  MPLPXX_CASE(128, 256)
  MPLPXX_CASE(128, 512)
#undef MPLPXX_CASE
  return e == hipSuccess ? nb : 0;
}

hipError_t launch_persistent_mb(const HsArgs<float>& a, unsigned long long* mb, int LT, int NT, int grid, int iters,
                                int phi_in_lds, size_t dyn_lds, hipStream_t st, int prefetch, int kind, int rule) {
#define MPLPXX_CASE(lt, nt) \
  if (LT == lt && NT == nt) return launch_mb_one<lt, nt>(a, mb, grid, iters, phi_in_lds, dyn_lds, st, prefetch, kind, rule);
  MPLPXX_CASE(16, 64)
  MPLPXX_CASE(16, 256)
  MPLPXX_CASE(32, 64)
  MPLPXX_CASE(32, 256)
  MPLPXX_CASE(32, 512)
  MPLPXX_CASE(64, 256)
  MPLPXX_CASE(64, 512)
  MPLPXX_CASE(128, 256)
  MPLPXX_CASE(128, 512)
#undef MPLPXX_CASE
  return hipErrorInvalidValue;
}

int max_blocks_per_cu_mb_potts() {
  int nb = 0;
  const void* f = (const void*)k_persistent_mb_potts<false, MPLPXX_COST_POTTS>;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kPottsNT + 128, 0);
  return e == hipSuccess ? placeable_per_cu(f, kPottsNT + 128, nb) : 0;
}

hipError_t launch_persistent_mb_potts(const HsArgs<float>& a, unsigned long long* mb, int grid, int iters,
                                      int phi_in_lds, size_t dyn_lds, hipStream_t st, int kind) {
  void* args[] = {(void*)&a, (void*)&mb, (void*)&iters};
  const void* f = kind == MPLPXX_COST_TRUNC_QUAD
                      ? (phi_in_lds ? (const void*)k_persistent_mb_potts<true, MPLPXX_COST_TRUNC_QUAD>
                                    : (const void*)k_persistent_mb_potts<false, MPLPXX_COST_TRUNC_QUAD>)
                  : kind == MPLPXX_COST_TRUNC_LINEAR
                      ? (phi_in_lds ? (const void*)k_persistent_mb_potts<true, MPLPXX_COST_TRUNC_LINEAR>
                                    : (const void*)k_persistent_mb_potts<false, MPLPXX_COST_TRUNC_LINEAR>)
                      : (phi_in_lds ? (const void*)k_persistent_mb_potts<true, MPLPXX_COST_POTTS>
                                    : (const void*)k_persistent_mb_potts<false, MPLPXX_COST_POTTS>);
  const hipError_t e = hipLaunchCooperativeKernel(f, dim3(grid), dim3(kPottsNT + 128), args, dyn_lds, st);
  if (e != hipSuccess) (void)hipGetLastError();  // (see launch_mb_one)
  return e;
}

hipError_t launch_mb_init(const float* U, const float* Ulo, unsigned long long* mb, size_t count, hipStream_t st) {
  size_t blocks = (count + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mb_init, dim3((unsigned)blocks), dim3(256), 0, st, U, Ulo, mb, count);
  return hipGetLastError();
}

hipError_t launch_mb_fini(float* U, float* Ulo, const unsigned long long* mb, int n, int L, double* trace_row,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_mb_fini, dim3(n), dim3(64), 0, st, U, Ulo, mb, n, L, trace_row);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_handshake(const HsArgs<T>& a, int engine, int LT, int NT, int slot_begin, int count, int grid,
                            int iters, hipStream_t st) {
#define MPLPXX_CASE(lt, nt) \
  if (LT == lt && NT == nt) return launch_one<T, lt, nt>(a, engine, slot_begin, count, grid, iters, st);
  MPLPXX_CASE(16, 256)
  MPLPXX_CASE(32, 256)
  MPLPXX_CASE(32, 512)
  MPLPXX_CASE(64, 256)
  MPLPXX_CASE(64, 512)
  MPLPXX_CASE(64, 1024)
  MPLPXX_CASE(128, 256)
  MPLPXX_CASE(128, 512)
  MPLPXX_CASE(128, 1024)
#undef MPLPXX_CASE
  return hipErrorInvalidValue;
}

template <typename T>
int max_blocks_per_cu(int engine, int LT, int NT) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define MPLPXX_CASE(lt, nt)                                                                           \
  if (LT == lt && NT == nt) {                                                                         \
    const void* f = engine == ENGINE_STEP ? (const void*)k_step<T, lt, nt> : (const void*)k_persistent<T, lt, nt>; \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, nt, 0);                                  \
    if (e == hipSuccess && engine != ENGINE_STEP) nb = placeable_per_cu(f, nt, nb);                   \
  }
  MPLPXX_CASE(16, 256)
  MPLPXX_CASE(32, 256)
  MPLPXX_CASE(32, 512)
  MPLPXX_CASE(64, 256)
  MPLPXX_CASE(64, 512)
  MPLPXX_CASE(64, 1024)
  MPLPXX_CASE(128, 256)
  MPLPXX_CASE(128, 512)
  MPLPXX_CASE(128, 1024)
#undef MPLPXX_CASE
  return e == hipSuccess ? nb : 0;
}

template hipError_t launch_handshake<float>(const HsArgs<float>&, int, int, int, int, int, int, int, hipStream_t);
template hipError_t launch_handshake<double>(const HsArgs<double>&, int, int, int, int, int, int, int, hipStream_t);
template int max_blocks_per_cu<float>(int, int, int);
template int max_blocks_per_cu<double>(int, int, int);

}  // namespace mplpxx
