// Device building blocks shared by the MPLP++ kernels: exact min
// reductions across lanes, register tiles of an L x L pairwise table, and the
// mailbox engine that runs handshake updates over the slots a workgroup owns.
// (Paper: Tourani et al., MPLP++, ECCV 2018, Sec. 4 and Sec. 6.)
#pragma once
#include "common.h"

namespace mplpxx {


template <typename T> __device__ __forceinline__ T inf_v();
template <> __device__ __forceinline__ float inf_v<float>() { return __builtin_inff(); }
template <> __device__ __forceinline__ double inf_v<double>() { return __builtin_inf(); }

__device__ __forceinline__ float vmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double vmin(double a, double b) { return __builtin_fmin(a, b); }

// Cross-lane minima without LDS traffic.  DPP row operations stay inside a
// 16-lane row: quad_perm [1,0,3,2] and [2,3,0,1] combine lanes of a quad,
// row_half_mirror joins the two quads of each half row, row_mirror the two
// halves.  gfx950's v_permlane16_swap / v_permlane32_swap exchange rows
// (lanes 16 and 32 apart).  Min is exact and order-free, so every lane ends
// with the same bits whatever the exchange pattern.
template <int CTRL> __device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double dpp_f(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(v & 0xffffffff), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// minimum over the 16 lanes of a row (lanes 16k .. 16k+15), result in all 16
template <typename T> __device__ __forceinline__ T row16_min(T x) {
  x = vmin(x, dpp_f<0xB1>(x));   // quad_perm [1,0,3,2]
  x = vmin(x, dpp_f<0x4E>(x));   // quad_perm [2,3,0,1]
  x = vmin(x, dpp_f<0x141>(x));  // row_half_mirror
  x = vmin(x, dpp_f<0x140>(x));  // row_mirror
  return x;
}

// the same for N independent values at once (interleaved for ILP)
template <int N, typename T> __device__ __forceinline__ void row16_min_n(T (&x)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) x[k] = vmin(x[k], dpp_f<0xB1>(x[k]));
#pragma unroll
  for (int k = 0; k < N; ++k) x[k] = vmin(x[k], dpp_f<0x4E>(x[k]));
#pragma unroll
  for (int k = 0; k < N; ++k) x[k] = vmin(x[k], dpp_f<0x141>(x[k]));
#pragma unroll
  for (int k = 0; k < N; ++k) x[k] = vmin(x[k], dpp_f<0x140>(x[k]));
}

// minimum over lanes l, l^16, l^32, l^48 (the 4 row blocks of one wave)
__device__ __forceinline__ float col4_min(float x) {
  auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  x = vmin(__uint_as_float(a[0]), __uint_as_float(a[1]));
  auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return vmin(__uint_as_float(b[0]), __uint_as_float(b[1]));
}
__device__ __forceinline__ double col4_min(double x) {
  x = vmin(x, __shfl_xor(x, 16, 64));
  x = vmin(x, __shfl_xor(x, 32, 64));
  return x;
}

// coherent (device-scope) accesses for data shared between workgroups
__device__ __forceinline__ int ld_dev(const int* p) {
  return __hip_atomic_load(const_cast<int*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> __device__ __forceinline__ T ldv_dev(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> __device__ __forceinline__ void stv_dev(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// wait until this wave's memory operations have completed
__device__ __forceinline__ void wait_vmem() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <typename T, int LT, int NT> struct TileShape {
  static constexpr int RB = NT / 16;   // row blocks
  static constexpr int BR = LT / RB;   // rows per thread
  static constexpr int BC = LT / 16;   // columns per thread
  static constexpr int W = NT / 64;    // waves
  static_assert(BR >= 1 && BC >= 1 && RB * BR == LT, "tile shape");
};

// Loads the table of one slot into the register tile; pads are +inf.
template <typename T, int LT, int NT>
__device__ __forceinline__ void load_tile(const T* __restrict__ tab, int L, T (&x)[TileShape<T, LT, NT>::BR][TileShape<T, LT, NT>::BC]) {
  using S = TileShape<T, LT, NT>;
  const int tid = threadIdx.x;
  const int rb = tid >> 4, cb = tid & 15;
  if (L == LT && (S::BC % 4) == 0 && sizeof(T) == 4) {
    // full tile, 16-byte aligned rows: vector loads
#pragma unroll
    for (int i = 0; i < S::BR; ++i) {
      const int s = rb * S::BR + i;
#pragma unroll
      for (int j = 0; j < S::BC; j += 4) {
        const float4 v = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(tab) + s * LT + cb * S::BC + j);
        x[i][j] = v.x;
        x[i][j + 1] = v.y;
        x[i][j + 2] = v.z;
        x[i][j + 3] = v.w;
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < S::BR; ++i) {
      const int s = rb * S::BR + i;
#pragma unroll
      for (int j = 0; j < S::BC; ++j) {
        const int t = cb * S::BC + j;
        x[i][j] = (s < L && t < L) ? tab[s * L + t] : inf_v<T>();
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Engine 2, FP32: persistent with tagged mailboxes.
//
// The reparametrized unaries travel between workgroups through a mailbox
// array MB[n][L] of 64-bit words: low half = the FP32 bits of U_u(s), high
// half = the number of updates node u has seen in this launch.  A consumer
// polls the words it needs until every one carries the version it expects,
// so the data is its own ready flag: no separate flag store, no wait for
// store completion on the producer side.  Each word is written and read with
// one 64-bit device-scope atomic access, so a value and its version can
// never be seen torn.
//
// Two extra "sync" waves (threads NT .. NT+127) do all polling and gathering:
// they issue no other loads, so a poll never queues behind a table prefetch
// in the in-order memory counter of the compute waves.  The messages of the
// slots a workgroup owns stay in LDS for the whole launch when they fit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long mb_pack(float v, unsigned ver) {
  return ((unsigned long long)ver << 32) | (unsigned long long)__float_as_uint(v);
}
__device__ __forceinline__ unsigned long long mb_load(const unsigned long long* p) {
  return __hip_atomic_load(const_cast<unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void mb_store(unsigned long long* p, unsigned long long w) {
  __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int LT, int NT> struct SmemMB {
  float uu[2][LT];   // raw U_u delivered by the sync wave (double buffered by slot parity)
  float uv[2][LT];
  float red[TileShape<float, LT, NT>::W][LT];
  int abort_flag;
};

// the sync wave: poll MB[node] until all L words carry `want`, deliver values
// On a timed-out wait: err[0] = MPLPXX_ETIMEOUT and, for the first waiter
// that gives up, err[1..5] = (workgroup, slot, node, expected version,
// version seen).
__device__ __forceinline__ void report_timeout(int* err, int slot, int node, unsigned want, unsigned seen) {
  if (atomicCAS(err, 0, MPLPXX_ETIMEOUT) == 0) {
    err[1] = blockIdx.x;
    err[2] = slot;
    err[3] = node;
    err[4] = (int)want;
    err[5] = (int)seen;
  }
}

template <int LT>
__device__ __forceinline__ bool sync_gather(const unsigned long long* __restrict__ mb_row, int L, unsigned want,
                                            float* dst, long long spin_limit, const int* err, unsigned* seen_out) {
  const int lane = threadIdx.x & 63;
  constexpr int PER = (LT + 63) / 64;
  bool have[PER];
  float val[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) have[k] = (lane + 64 * k) >= L;
  long long spins = 0;
  for (;;) {
    bool all = true;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      if (!have[k]) {
        const unsigned long long w = mb_load(mb_row + lane + 64 * k);
        if ((unsigned)(w >> 32) == want) {
          have[k] = true;
          val[k] = __uint_as_float((unsigned)w);
        } else {
          all = false;
        }
      }
    }
    if (__all(all)) break;
    if (++spins > spin_limit || ((spins & 255) == 0 && ld_dev(err) != 0)) {
      unsigned seen = want;
#pragma unroll
      for (int k = 0; k < PER; ++k)
        if (!have[k]) seen = (unsigned)(mb_load(mb_row + lane + 64 * k) >> 32);
      // smallest version still missing in the wave
      for (int o = 32; o >= 1; o >>= 1) seen = min(seen, (unsigned)__shfl_xor((int)seen, o, 64));
      *seen_out = seen;
      return false;
    }
  }
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (lane + 64 * k < L) dst[lane + 64 * k] = val[k];
  return true;
}

// One model as the mailbox engine sees it.
struct MbView {
  const float* tables;          // [m][L][L] slot order
  float* phi;                   // [m][2][L] slot order
  unsigned long long* mb;       // [n][L] mailboxes
  const SlotInfo* slots;        // [m]
  const int* deg;               // [n]
  double* trace;                // [iters][n] or null
  long long* stamps;            // [m][kStampStride] or null
  int L, m, n;
};

// Messages of one slot for this thread's rows (into u) and columns (into v).
template <int LT, int NT, bool PHI_LDS, bool FULL>
__device__ __forceinline__ void load_phi(const float* src, int L, float (&pu)[TileShape<float, LT, NT>::BR],
                                         float (&pv)[TileShape<float, LT, NT>::BC]) {
  using S = TileShape<float, LT, NT>;
  const int rb = threadIdx.x >> 4, cb = threadIdx.x & 15;
#pragma unroll
  for (int i = 0; i < S::BR; ++i) {
    const int s = rb * S::BR + i;
    pu[i] = src[(FULL || s < L) ? s : L - 1];
  }
#pragma unroll
  for (int jj = 0; jj < S::BC; ++jj) {
    const int t = cb * S::BC + jj;
    pv[jj] = src[L + ((FULL || t < L) ? t : L - 1)];
  }
}

// Runs `iters` iterations over the slots first, first+stride, ... of one
// model.  Compute threads [0, NT) hold the table of the current slot in
// registers and prefetch the next one together with its messages; threads
// [NT, NT+128) are the two sync waves.  Returns false if a wait timed out
// (the error word is set); every thread of the block returns the same value.
template <int LT, int NT, bool PHI_LDS, bool FULL>
__device__ __forceinline__ bool mb_run(const MbView& v, int first, int stride, int iters, SmemMB<LT, NT>& sm,
                                       float* phi_lds, long long spin_limit, int* err) {
  using S = TileShape<float, LT, NT>;
  const int tid = threadIdx.x;
  const int L = FULL ? LT : v.L;
  const int wave = tid >> 6;
  const bool is_compute = tid < NT;
  const bool is_sync_u = wave == NT / 64;
  const int rb = tid >> 4, cb = tid & 15, lane = tid & 63;
  if (first >= v.m) return true;
  auto phi_of = [&](int slot, int j) -> float* {
    return PHI_LDS ? phi_lds + (size_t)j * 2 * L : v.phi + (size_t)slot * 2 * L;
  };
  float x[S::BR][S::BC], y[S::BR][S::BC];
  float pu[S::BR], pv[S::BC], npu[S::BR], npv[S::BC];
  if (is_compute) {
    load_tile<float, LT, NT>(v.tables + (size_t)first * L * L, L, x);
    load_phi<LT, NT, PHI_LDS, FULL>(phi_of(first, 0), L, pu, pv);
  }
  SlotInfo si = v.slots[first];
  // slots owned: 1 -> the next slot is this one (its messages are the r, q
  // just computed); 2 -> the next slot is the previous one, whose messages
  // this workgroup wrote during the last slot: they are read after this
  // slot's first barrier; >= 3 -> the next slot's messages were written two
  // or more slots ago, behind two barriers, and are prefetched with its table
  const int owned = (v.m - first + stride - 1) / stride;
  int parity = 0;
  for (int it = 0; it < iters; ++it) {
    int j = 0;
    for (int slot = first; slot < v.m; slot += stride, ++j, parity ^= 1) {
      const unsigned want_u = (unsigned)(it * si.deg_u + si.pos_u);
      const unsigned want_v = (unsigned)(it * si.deg_v + si.pos_v);
      int nxt = slot + stride, jn = j + 1;
      if (nxt >= v.m) { nxt = first; jn = 0; }
      const bool pref = nxt != slot && (it + 1 < iters || nxt > slot);
      const bool last_iter = it == iters - 1;
      // metadata of the next owned slot, off the dependency chain
      const SlotInfo si_next = v.slots[nxt];
      if (is_compute) {
        // table of the next owned slot (its messages follow after the barrier,
        // once this workgroup's earlier writes to them are ordered)
        if (pref) {
          load_tile<float, LT, NT>(v.tables + (size_t)nxt * L * L, L, y);
          // (the very first slot's successor has not been written in this launch)
          if (owned >= 3 || (it == 0 && j == 0)) load_phi<LT, NT, PHI_LDS, FULL>(phi_of(nxt, jn), L, npu, npv);
        }
#if MPLPXX_FINE_STAMPS
        if (v.stamps && last_iter && tid == 0) v.stamps[(size_t)slot * kStampStride + 4] = wall_clock64();
#endif
      } else {
        if (v.stamps && last_iter && lane == 0 && is_sync_u) v.stamps[(size_t)slot * kStampStride + 0] = wall_clock64();
        const int node = is_sync_u ? si.u : si.v;
        const unsigned want = is_sync_u ? want_u : want_v;
        float* dst = is_sync_u ? sm.uu[parity] : sm.uv[parity];
        unsigned seen = 0;
        if (!sync_gather<LT>(v.mb + (size_t)node * L, L, want, dst, spin_limit, err, &seen)) {
          if (lane == 0) {
            // a wait may also end because another workgroup reported first
            if (ld_dev(err) == 0 || seen != want) report_timeout(err, slot, node, want, seen);
            sm.abort_flag = 1;
          }
        }
        if (v.stamps && last_iter && lane == 0) v.stamps[(size_t)slot * kStampStride + (is_sync_u ? 1 : 2)] = wall_clock64();
      }
      __syncthreads();
      if (sm.abort_flag) return false;
      if (is_compute && pref && owned == 2 && !(it == 0 && j == 0))
        load_phi<LT, NT, PHI_LDS, FULL>(phi_of(nxt, jn), L, npu, npv);
      if (is_compute) {
#if MPLPXX_FINE_STAMPS
        if (v.stamps && last_iter && tid == 0) v.stamps[(size_t)slot * kStampStride + 5] = wall_clock64();
#endif
        // a = U - phi; unconditional LDS reads at clamped indices, then a
        // select, so the reads issue as one batch
        float av[S::BC], au[S::BR];
#pragma unroll
        for (int jj = 0; jj < S::BC; ++jj) {
          const int t = cb * S::BC + jj;
          const int tc = (FULL || t < L) ? t : L - 1;
          av[jj] = (FULL || t < L) ? sm.uv[parity][tc] - pv[jj] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < S::BR; ++i) {
          const int s = rb * S::BR + i;
          const int sc = (FULL || s < L) ? s : L - 1;
          au[i] = (FULL || s < L) ? sm.uu[parity][sc] - pu[i] : 0.f;
        }
        // pass 1: p(s) = min_t [th(s,t) + a_v(t)], b = (a_u - p) / 2
        float b[S::BR];
        {
          float pm[S::BR];
#pragma unroll
          for (int i = 0; i < S::BR; ++i) {
            float mn = x[i][0] + av[0];
#pragma unroll
            for (int jj = 1; jj < S::BC; ++jj) mn = vmin(mn, x[i][jj] + av[jj]);
            pm[i] = mn;
          }
          row16_min_n<S::BR>(pm);
#pragma unroll
          for (int i = 0; i < S::BR; ++i) {
            const int s = rb * S::BR + i;
            b[i] = (FULL || s < L) ? 0.5f * (au[i] - pm[i]) : 0.f;
          }
        }
        // pass 2: q(t) = min_s [th(s,t) + b(s)]
        float q[S::BC];
#pragma unroll
        for (int jj = 0; jj < S::BC; ++jj) {
          float mn = x[0][jj] + b[0];
#pragma unroll
          for (int i = 1; i < S::BR; ++i) mn = vmin(mn, x[i][jj] + b[i]);
          q[jj] = col4_min(mn);
        }
        if (lane < 16) {
#pragma unroll
          for (int jj = 0; jj < S::BC; ++jj) sm.red[wave][cb * S::BC + jj] = q[jj];
        }
#if MPLPXX_FINE_STAMPS
        if (v.stamps && last_iter && tid == 0) v.stamps[(size_t)slot * kStampStride + 6] = wall_clock64();
#endif
        __syncthreads();  // matched by the sync waves' barrier below
#if MPLPXX_FINE_STAMPS
        if (v.stamps && last_iter && tid == 0) v.stamps[(size_t)slot * kStampStride + 7] = wall_clock64();
#endif
#pragma unroll
        for (int jj = 0; jj < S::BC; ++jj) {
          const int t = cb * S::BC + jj;
          float mn = sm.red[0][t];
#pragma unroll
          for (int w = 1; w < S::W; ++w) mn = vmin(mn, sm.red[w][t]);
          q[jj] = (FULL || t < L) ? mn : 0.f;
        }
        // pass 3: r(s) = min_t [th(s,t) - q(t)]
        float r[S::BR];
#pragma unroll
        for (int i = 0; i < S::BR; ++i) {
          float mn = x[i][0] - q[0];
#pragma unroll
          for (int jj = 1; jj < S::BC; ++jj) mn = vmin(mn, x[i][jj] - q[jj]);
          r[i] = mn;
        }
        row16_min_n<S::BR>(r);
        // push back: new unaries through the mailboxes, messages to memory
        float* phi_w = phi_of(slot, j);
        if (rb == 0) {
#pragma unroll
          for (int jj = 0; jj < S::BC; ++jj) {
            const int t = cb * S::BC + jj;
            if (FULL || t < L) {
              mb_store(v.mb + (size_t)si.v * L + t, mb_pack(av[jj] + q[jj], want_v + 1));
              phi_w[L + t] = q[jj];
            }
          }
        }
        if (cb == 0) {
#pragma unroll
          for (int i = 0; i < S::BR; ++i) {
            const int s = rb * S::BR + i;
            if (FULL || s < L) {
              mb_store(v.mb + (size_t)si.u * L + s, mb_pack(au[i] + r[i], want_u + 1));
              phi_w[s] = r[i];
            }
          }
        }
        if (v.stamps && last_iter && tid == 0) v.stamps[(size_t)slot * kStampStride + 3] = wall_clock64();
        if (pref) {
#pragma unroll
          for (int i = 0; i < S::BR; ++i) {
            pu[i] = npu[i];
#pragma unroll
            for (int jj = 0; jj < S::BC; ++jj) x[i][jj] = y[i][jj];
          }
#pragma unroll
          for (int jj = 0; jj < S::BC; ++jj) pv[jj] = npv[jj];
        } else {
          // the same slot comes next: its messages are the ones just made
#pragma unroll
          for (int i = 0; i < S::BR; ++i) pu[i] = r[i];
#pragma unroll
          for (int jj = 0; jj < S::BC; ++jj) pv[jj] = q[jj];
        }
      } else {
        // the sync waves take part in the compute waves' mid-slot barrier
        __syncthreads();
        // per-iteration trace: the first update of a node in iteration it
        // sees the node's value at the end of iteration it-1
        if (v.trace && it > 0) {
          const bool first_upd = is_sync_u ? (si.pos_u == 0) : (si.pos_v == 0);
          if (first_upd) {
            const float* src = is_sync_u ? sm.uu[parity] : sm.uv[parity];
            double mn = __builtin_inf();
            for (int s2 = lane; s2 < L; s2 += 64) mn = __builtin_fmin(mn, (double)src[s2]);
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) mn = __builtin_fmin(mn, __shfl_xor(mn, o, 64));
            if (lane == 0) v.trace[(size_t)(it - 1) * v.n + (is_sync_u ? si.u : si.v)] = mn;
          }
        }
      }
      si = si_next;
    }
  }
  return true;
}

}  // namespace mplpxx
