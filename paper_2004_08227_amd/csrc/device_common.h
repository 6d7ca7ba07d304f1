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
// (STEPS < 4 stops early: after 3 steps each lane holds the minimum over its
// half row)
template <int N, int STEPS = 4, typename T> __device__ __forceinline__ void row16_min_n(T (&x)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) x[k] = vmin(x[k], dpp_f<0xB1>(x[k]));
#pragma unroll
  for (int k = 0; k < N; ++k) x[k] = vmin(x[k], dpp_f<0x4E>(x[k]));
#pragma unroll
  for (int k = 0; k < N; ++k) x[k] = vmin(x[k], dpp_f<0x141>(x[k]));
  if constexpr (STEPS == 4) {
#pragma unroll
    for (int k = 0; k < N; ++k) x[k] = vmin(x[k], dpp_f<0x140>(x[k]));
  }
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

// Column minima over the wave's four row blocks for BC columns per lane,
// stored to red[cb * BC + jj].  The swaps carry two different columns each:
// a 16-lane swap of columns a and b leaves row blocks 0..3 holding the
// pairwise minima (rows 0-1 of a, rows 0-1 of b, rows 2-3 of a, rows 2-3 of
// b), and a 32-lane swap of two such results joins rows 0-1 with rows 2-3,
// so with four columns row block k ends with the minimum of column k: three
// swaps and three minima where a swap of each column with itself needs
// eight of each and eight copies.
__device__ __forceinline__ float pair16_min(float a, float b) {
  auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return vmin(__uint_as_float(r[0]), __uint_as_float(r[1]));
}
__device__ __forceinline__ float join32_min(float a, float b) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return vmin(__uint_as_float(r[0]), __uint_as_float(r[1]));
}
template <int BC>
__device__ __forceinline__ void col4_min_store(const float (&x)[BC], float* red, int cb, int lane) {
  const int k = lane >> 4;
  if constexpr (BC == 1) {
    const float m = col4_min(x[0]);
    if (lane < 16) red[cb] = m;
  } else if constexpr (BC == 2) {
    // row blocks 0..3 end with columns 0, 1, 0, 1
    const float m = pair16_min(x[0], x[1]);
    const float f = join32_min(m, m);
    if (lane < 32) red[cb * 2 + k] = f;
  } else {
    static_assert(BC % 4 == 0, "columns per lane");
#pragma unroll
    for (int g = 0; g < BC; g += 4)
      red[cb * BC + g + k] = join32_min(pair16_min(x[g], x[g + 1]), pair16_min(x[g + 2], x[g + 3]));
  }
}

// ---------------------------------------------------------------------------
// Compensated FP32 unaries.  U_u = theta_u + (sum of the messages into u) is
// a running sum: every update of an incident edge replaces one message,
// U_u := (U_u - phi_old) + phi_new (Sec. 4, (H)).  Rounding the new value to
// FP32 each time would let the error grow with the number of updates a node
// has seen.  In FP32 the state therefore keeps U = hi + lo, hi in FP32 and lo
// a correction rounded to bf16 (8 significant bits), and updates it with
// error-free sums (Knuth's TwoSum):
//   d  = hi - phi_old        (the a_u of the three passes, unchanged)
//   s  = d + phi_new
//   c  = (err(d) + err(s)) + lo
//   hi' = s + c,  lo' = bf16(err(hi'))
// so the error left per update is the bf16 rounding of lo', at most 2^-9 of
// an ulp of hi.  Every engine uses this one function, so they agree bitwise.
//
// Centred passes.  The messages (about 0.07 on the pose workload) come out
// of b = (a_u - p)/2, a difference of two O(|U|) numbers (about 2), so FP32
// a_u and a_v would cost each message a few 1e-7 of absolute error, and the
// block-coordinate ascent amplifies that over the iterations.  The FP32
// engines therefore take per node the reference c_u = min_s hi_u(s) (exact)
// and run the passes on a'_u = ((hi_u - c_u) + lo_u) - phi[0], which is
// small exactly where the minima are taken.  (H) is invariant under such
// shifts: with delta = (c_u - c_v)/2 the messages are r = r' - delta and
// q = q' + delta, where r', q' are the passes' results on a'.
// ---------------------------------------------------------------------------
// exact error of s = fl(a + b): a + b = s + two_sum_err(a, b, s)
__device__ __forceinline__ float two_sum_err(float a, float b, float s) {
  const float bb = s - a;
  return (a - (s - bb)) + (b - bb);
}
// nearest bf16 value (ties to even); finite inputs
__device__ __forceinline__ float bf16_round(float x) {
  const unsigned u = __float_as_uint(x);
  return __uint_as_float((u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u);
}
__device__ __forceinline__ void comp_update(float hi, float lo, float phi_old, float phi_new, float& nhi, float& nlo) {
  const float d = hi - phi_old;
  const float e1 = two_sum_err(hi, -phi_old, d);
  const float s = d + phi_new;
  const float e2 = two_sum_err(d, phi_new, s);
  const float c = (e1 + e2) + lo;
  nhi = s + c;
  nlo = bf16_round(two_sum_err(s, c, nhi));
}
// comp_update in two parts with the same operations in the same order (so
// the same bits): the head needs only the old value and message, the tail
// adds the new message.
__device__ __forceinline__ void comp_update_head(float hi, float phi_old, float& d, float& e1) {
  d = hi - phi_old;
  e1 = two_sum_err(hi, -phi_old, d);
}
__device__ __forceinline__ void comp_update_tail(float d, float e1, float lo, float phi_new, float& nhi, float& nlo) {
  const float s = d + phi_new;
  const float e2 = two_sum_err(d, phi_new, s);
  const float c = (e1 + e2) + lo;
  nhi = s + c;
  nlo = bf16_round(two_sum_err(s, c, nhi));
}

// Values every lane of the wave holds the same: readfirstlane tells the
// compiler so, and loads through such pointers and indices become scalar
// loads (scalar cache, lgkmcnt) instead of vector loads that share vmcnt with
// the table prefetches.
// (Offsets, not pointers: a pointer rebuilt from integers would lose its
// address space and turn every access into a FLAT one.)
//
// ld_const: a load from data no thread writes during the kernel, through the
// constant address space, so that a uniform address becomes one scalar load.
__device__ __forceinline__ SlotInfo ld_const(const SlotInfo* p) {
  const __attribute__((address_space(4))) int* q = (const __attribute__((address_space(4))) int*)p;
  SlotInfo r;
  r.e = q[0];
  r.u = q[1];
  r.v = q[2];
  r.pos_u = q[3];
  r.pos_v = q[4];
  r.deg_u = q[5];
  r.deg_v = q[6];
  r.step = q[7];
  return r;
}
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ long long uni(long long x) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(unsigned long long)x);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)x >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
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

template <typename T, int LT, int NT> struct TileShape {
  static constexpr int RB = NT / 16;   // row blocks
  static constexpr int BR = LT / RB;   // rows per thread
  static constexpr int BC = LT / 16;   // columns per thread
  static constexpr int W = NT / 64;    // waves
  static_assert(BR >= 1 && BC >= 1 && RB * BR == LT, "tile shape");
};

// Table pad of the mailbox engine.  With pads = BIG = 2^126 and every real
// value below 2^100 in magnitude, the three passes need no masks: a padded
// column never wins a row minimum (BIG + a_v rounds to BIG); a padded row
// gets p = BIG, b = -BIG/2 exactly, so it never wins a column minimum of a
// real column (BIG - BIG/2 = BIG/2) and makes q = BIG/2 in every padded
// column, which in turn never wins pass 3 (BIG - BIG/2).  All values stay
// finite and every real minimum is the one over the real entries, so the
// results are bitwise those of the unpadded tile.
constexpr float kPadBig = 0x1p126f;

// Loads the table of one slot into the register tile; pads take `pad`.
template <typename T, int LT, int NT>
__device__ __forceinline__ void load_tile(const T* __restrict__ tab, int L, T (&x)[TileShape<T, LT, NT>::BR][TileShape<T, LT, NT>::BC],
                                          T pad = inf_v<T>()) {
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
        x[i][j] = (s < L && t < L) ? tab[s * L + t] : pad;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Engine 2, FP32: persistent with tagged mailboxes.
//
// The reparametrized unaries travel between workgroups through a mailbox
// array MB[n][L] of 64-bit words: bits 0..31 = hi of U_u(s) (FP32), bits
// 32..47 = its bf16 correction lo, bits 48..63 = the number of updates node u
// has seen in this launch, modulo 2^16.  A waiter for version w can only see
// versions w - deg(u) + 1 .. w (it made version w - deg(u) + 1 itself one
// iteration earlier, and nobody makes w + 1 before it), so 16 bits identify
// the version when every degree is below 2^16.  A consumer
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
__device__ __forceinline__ unsigned long long mb_pack(float hi, float lo, unsigned ver) {
  const unsigned top = (ver << 16) | (__float_as_uint(lo) >> 16);
  return ((unsigned long long)top << 32) | (unsigned long long)__float_as_uint(hi);
}
__device__ __forceinline__ unsigned mb_ver(unsigned long long w) { return (unsigned)(w >> 48); }
__device__ __forceinline__ float mb_hi(unsigned long long w) { return __uint_as_float((unsigned)w); }
__device__ __forceinline__ float mb_lo(unsigned long long w) { return __uint_as_float((unsigned)(w >> 32) << 16); }
__device__ __forceinline__ unsigned long long mb_load(const unsigned long long* p) {
  return __hip_atomic_load(const_cast<unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void mb_store(unsigned long long* p, unsigned long long w) {
  __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int LT, int NT> struct SmemMB {
  float uu[2][LT];   // centred (hi - c) + lo of U_u from the sync wave (double buffered by slot parity)
  float uv[2][LT];
  float uh[2][LT];   // hi of U_u
  float vh[2][LT];
  float ul[2][LT];   // lo of U_u
  float vl[2][LT];
  float cc[2][2];    // references c_u, c_v
  alignas(16) float red[TileShape<float, LT, NT>::W][LT];
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

// On success delivers hi, lo, the centred values (hi - c) + lo and the
// reference c = min_s hi(s) of the node.
template <int LT>
__device__ __forceinline__ bool sync_gather(const unsigned long long* __restrict__ mb_row, int L, unsigned want,
                                            float* dst_un, float* dst_hi, float* dst_lo, float* dst_c,
                                            long long spin_limit, const int* err, unsigned* seen_out) {
  const int lane = threadIdx.x & 63;
  constexpr int PER = (LT + 63) / 64;
  want &= 0xFFFFu;
  // Every lane reloads its words until the whole wave sees the version:
  // no word can move past it meanwhile, since this workgroup makes the
  // node's next update (lanes past L read word L - 1).
  // (one exit from the loop, so that the delivery follows a hit directly)
  unsigned long long val[PER];
  long long spins = 0;
  bool done;
  do {
    bool all = true;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int s = lane + 64 * k;
      val[k] = mb_load(mb_row + (s < L ? s : L - 1));
      all &= mb_ver(val[k]) == want;
    }
    done = __all(all);
  } while (!done && ++spins <= spin_limit && ((spins & 255) != 0 || ld_dev(err) == 0));
  if (!done) {
    unsigned seen = want;
#pragma unroll
    for (int k = 0; k < PER; ++k)
      if (mb_ver(val[k]) != want) seen = mb_ver(val[k]);
    // smallest version still missing in the wave
    for (int o = 32; o >= 1; o >>= 1) seen = min(seen, (unsigned)__shfl_xor((int)seen, o, 64));
    *seen_out = seen;
    return false;
  }
  float c = __builtin_inff();
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (lane + 64 * k < L) c = vmin(c, mb_hi(val[k]));
  c = col4_min(row16_min(c));
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (lane + 64 * k < L) {
      const float hi = mb_hi(val[k]), lo = mb_lo(val[k]);
      dst_hi[lane + 64 * k] = hi;
      dst_lo[lane + 64 * k] = lo;
      dst_un[lane + 64 * k] = (hi - c) + lo;
    }
  if (lane == 0) *dst_c = c;
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
  float* trace_e;               // [iters][m][W] per-wave minima of the edge terms, or null
  long long* stamps;            // [m][kStampStride] or null
  int L, m, n;
  float* lds_hi;                // LDS-resident unaries (hi [n][L], lo as bf16 bits), or null
  unsigned short* lds_lo;
  unsigned long long* sink;     // this workgroup's scratch words [NT + 128] (see the output stores)
};

// The gather of the LDS-resident mode: hi, lo, centred values and reference
// of one node from this workgroup's LDS copy of the unaries (no wait: the
// workgroup itself produced them, ordered by its barriers).
template <int LT>
__device__ __forceinline__ void lds_gather(const float* hi_row, const unsigned short* lo_row, int L, float* dst_un,
                                           float* dst_hi, float* dst_lo, float* dst_c) {
  const int lane = threadIdx.x & 63;
  constexpr int PER = (LT + 63) / 64;
  float h[PER], l[PER];
  float c = __builtin_inff();
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int s = lane + 64 * k;
    const int sc = s < L ? s : L - 1;
    h[k] = hi_row[sc];
    l[k] = __uint_as_float((unsigned)lo_row[sc] << 16);
    if (s < L) c = vmin(c, h[k]);
  }
  c = col4_min(row16_min(c));
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int s = lane + 64 * k;
    if (s < L) {
      dst_hi[s] = h[k];
      dst_lo[s] = l[k];
      dst_un[s] = (h[k] - c) + l[k];
    }
  }
  if (lane == 0) *dst_c = c;
}

// Raw tile load for the mailbox engine: every lane loads, at clamped indices
// (always inside the table), so no load is predicated and no destination
// register is written twice; the pads are applied when the tile is used
// (pad_tile).  A predicated load into a register that the pad value was
// written to makes the compiler wait for every load in flight.
template <int LT, int NT, bool FULL>
__device__ __forceinline__ void load_tile_raw(const float* __restrict__ tab, int L,
                                              float (&x)[TileShape<float, LT, NT>::BR][TileShape<float, LT, NT>::BC]) {
  using S = TileShape<float, LT, NT>;
  const int rb = threadIdx.x >> 4, cb = threadIdx.x & 15;
  if (FULL && (S::BC % 4) == 0) {
#pragma unroll
    for (int i = 0; i < S::BR; ++i) {
      const int s = rb * S::BR + i;
#pragma unroll
      for (int j = 0; j < S::BC; j += 4) {
        const float4 v = *reinterpret_cast<const float4*>(tab + s * LT + cb * S::BC + j);
        x[i][j] = v.x;
        x[i][j + 1] = v.y;
        x[i][j + 2] = v.z;
        x[i][j + 3] = v.w;
      }
    }
  } else {
    // rows clamped, columns not: a row segment runs on into the next row
    // (or past the table, into the allocation's zeroed tail); those entries
    // are replaced by the pad in pad_tile.  One address per row, immediate
    // offsets for the columns.
#pragma unroll
    for (int i = 0; i < S::BR; ++i) {
      const int s = rb * S::BR + i;
      const float* row = tab + ((FULL || s < L) ? s : L - 1) * L + cb * S::BC;
#pragma unroll
      for (int j = 0; j < S::BC; ++j) x[i][j] = row[j];
    }
  }
}
template <int LT, int NT, bool FULL>
__device__ __forceinline__ void pad_tile(int L, float (&x)[TileShape<float, LT, NT>::BR][TileShape<float, LT, NT>::BC]) {
  using S = TileShape<float, LT, NT>;
  if (FULL) return;
  const int rb = threadIdx.x >> 4, cb = threadIdx.x & 15;
#pragma unroll
  for (int i = 0; i < S::BR; ++i) {
    const int s = rb * S::BR + i;
#pragma unroll
    for (int j = 0; j < S::BC; ++j) {
      const int t = cb * S::BC + j;
      x[i][j] = (s < L && t < L) ? x[i][j] : kPadBig;
    }
  }
}

// A +0 the compiler cannot see (a visible constant would let it rewrite
// fl(0 - q) under a minimum as -q, which is -0 for q = +0).
__device__ __forceinline__ float opaque_zero() {
  float z = 0.0f;
  asm volatile("" : "+v"(z));
  return z;
}
// scalar load of read-only data through the constant address space
__device__ __forceinline__ float ld_const_f(const float* p) {
  return *(const __attribute__((address_space(4))) float*)p;
}

// The register tile of a structured cost, formed from the slot's
// parameters instead of loaded: entry (s, t) is exactly the expanded
// table's value (Potts: +0 on the diagonal, w off it; truncated linear:
// fl(w min(|s - t|, tau)); truncated quadratic: fl(w min((s - t)^2, tau))),
// so the passes give the dense engine's bits.
// Entries outside L x L are replaced by the pad at use (pad_tile).
template <int LT, int NT, int KIND>
__device__ __forceinline__ void gen_tile(const float* prm, float (&x)[TileShape<float, LT, NT>::BR][TileShape<float, LT, NT>::BC]) {
  using S = TileShape<float, LT, NT>;
  const int rb = threadIdx.x >> 4, cb = threadIdx.x & 15;
  const float w = ld_const_f(prm);
  if constexpr (KIND == MPLPXX_COST_POTTS) {
    const float z = opaque_zero();
#pragma unroll
    for (int i = 0; i < S::BR; ++i)
#pragma unroll
      for (int j = 0; j < S::BC; ++j) x[i][j] = (rb * S::BR + i == cb * S::BC + j) ? z : w;
  } else {
    static_assert(KIND == MPLPXX_COST_TRUNC_LINEAR || KIND == MPLPXX_COST_TRUNC_QUAD, "structured cost kind");
    const float tau = ld_const_f(prm + 1);
#pragma unroll
    for (int i = 0; i < S::BR; ++i)
#pragma unroll
      for (int j = 0; j < S::BC; ++j) {
        const int dd = rb * S::BR + i - cb * S::BC - j;
        const float d = (float)(dd < 0 ? -dd : dd);
        x[i][j] = truncated_cost(w, tau, KIND == MPLPXX_COST_TRUNC_QUAD ? d * d : d);
      }
  }
}

// Messages of one slot for this thread's rows (into u) and columns (into v).
template <int LT, int NT, bool PHI_LDS, bool FULL>
__device__ __forceinline__ void load_phi(const float* src, int L, float (&pu)[TileShape<float, LT, NT>::BR],
                                         float (&pv)[TileShape<float, LT, NT>::BC]) {
  using S = TileShape<float, LT, NT>;
  const int rb = threadIdx.x >> 4, cb = threadIdx.x & 15;
  if (PHI_LDS) {
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
  } else {
    // global messages: no clamping (padded labels read the following
    // messages or the allocation's zeroed tail; any finite value will do)
#pragma unroll
    for (int i = 0; i < S::BR; ++i) pu[i] = src[rb * S::BR + i];
#pragma unroll
    for (int jj = 0; jj < S::BC; ++jj) pv[jj] = src[L + cb * S::BC + jj];
  }
}

// Runs `iters` iterations over the slots first, first+stride, ... of one
// model: a flat sequence of owned*iters steps.  Compute threads [0, NT) hold
// the table of the current step in registers; the tables of the next DEPTH
// steps are in flight in a ring of DEPTH+1 register tiles whose roles rotate
// (the loop is unrolled by the ring size, so no tile is ever copied and each
// load has DEPTH steps to land).  The messages of the next step are
// prefetched one step ahead.  Threads [NT, NT+128) are the two sync waves.
// Returns false if a wait timed out (the error word is set); every thread of
// the block returns the same value.
//
// Each new unary value (with its message) is finished by one compute lane:
// row s = rb*BR + i by lane cb = i of row block rb, which holds r and the old
// message for that row; the columns are shared out over the other lanes of
// each wave, LT/W per wave, and each column lane keeps the old message of its
// column in a register of its own.
//
// LDSU: the whole model runs on this workgroup (first = 0, stride = 1) with
// its unaries in LDS (v.lds_hi / v.lds_lo) instead of the mailboxes.  The
// sync waves then read the next slot's nodes from LDS while the current slot
// computes; that is safe inside a matching (its edges share no node), and
// before the first slot of every matching all threads meet at one more
// barrier, after the previous slot's results are written.
// KIND: 0 dense tables; MPLPXX_COST_POTTS or _TRUNC_QUAD: the tile of each
// slot is formed from its parameters (v.tables holds cost_params(KIND)
// floats per slot) by gen_tile, the rest is the dense engine.
template <int LT, int NT, bool PHI_LDS, bool FULL, bool TRACE, bool LDSU, bool PHI_FAR, int DEPTH = (LT <= 64 ? 2 : 1),
          int KIND = kCostDense, int RULE = MPLPXX_RULE_H>
__device__ __forceinline__ bool mb_run(const MbView& v_in, int first_in, int stride_in, int iters_in,
                                       SmemMB<LT, NT>& sm, float* phi_lds, long long spin_limit, int* err) {
  using S = TileShape<float, LT, NT>;
  // sizes and positions are uniform over the workgroup (the pointers are
  // formed from uniform offsets by the caller)
  MbView v = v_in;
  v.L = uni(v.L);
  v.m = uni(v.m);
  v.n = uni(v.n);
  const int first = uni(first_in), stride = uni(stride_in), iters = uni(iters_in);
  const int tid = threadIdx.x;
  const int L = FULL ? LT : v.L;
  const int wave = tid >> 6;
  const int rb = tid >> 4, cb = tid & 15, lane = tid & 63;
  if (first >= v.m) return true;
  const int owned = (v.m - first + stride - 1) / stride;
  const int total = owned * iters;
  auto phi_of = [&](int slot, int j) -> float* {
    return PHI_LDS ? phi_lds + (size_t)j * 2 * L : v.phi + (size_t)slot * 2 * L;
  };
  // The two kinds of waves run separate loops with the same barriers per
  // step (first barrier, mid-step barrier, and in the LDS-resident mode one
  // more before each matching), so the compiler accounts for each loop's
  // memory operations on their own.
  if (tid >= NT) {
    // ---- sync waves: wait for (or read) the step's two nodes ----
    const bool is_sync_u = wave == NT / 64;
    SlotInfo si = ld_const(v.slots + first);
    int parity = 0, it = 0, j = 0;
    for (int q = 0; q < total; ++q) {
      const int slot = first + j * stride;
      const unsigned want_u = (unsigned)it * (unsigned)si.deg_u + (unsigned)si.pos_u;
      const unsigned want_v = (unsigned)it * (unsigned)si.deg_v + (unsigned)si.pos_v;
      int nxt = slot + stride;
      if (nxt >= v.m) nxt = first;
      nxt = uni(nxt);
      const bool last_iter = it == iters - 1;
      const SlotInfo si_next = ld_const(v.slots + nxt);
      if (v.stamps && last_iter && lane == 0 && is_sync_u) v.stamps[(size_t)slot * kStampStride + 0] = wall_clock64();
      const int node = is_sync_u ? si.u : si.v;
      const unsigned want = is_sync_u ? want_u : want_v;
      float* dst = is_sync_u ? sm.uu[parity] : sm.uv[parity];
      float* dst_hi = is_sync_u ? sm.uh[parity] : sm.vh[parity];
      float* dst_lo = is_sync_u ? sm.ul[parity] : sm.vl[parity];
      unsigned seen = 0;
      if (LDSU) {
        lds_gather<LT>(v.lds_hi + (size_t)node * L, v.lds_lo + (size_t)node * L, L, dst, dst_hi, dst_lo,
                       &sm.cc[parity][is_sync_u ? 0 : 1]);
      } else if (!sync_gather<LT>(v.mb + (size_t)node * L, L, want, dst, dst_hi, dst_lo,
                                  &sm.cc[parity][is_sync_u ? 0 : 1], spin_limit, err, &seen)) {
        if (lane == 0) {
          // a wait may also end because another workgroup reported first
          if (ld_dev(err) == 0 || seen != (want & 0xFFFFu)) report_timeout(err, slot, node, want & 0xFFFFu, seen);
          sm.abort_flag = q + 1;  // tagged with the step, so a later step's flag is not taken for this one's
        }
      }
      if (v.stamps && last_iter && lane == 0) v.stamps[(size_t)slot * kStampStride + (is_sync_u ? 1 : 2)] = wall_clock64();
      __syncthreads();
      __syncthreads();  // the compute waves' mid-step barrier
      // (a timed-out wait of this step is seen by every wave after the
      // mid-step barrier)
      if (sm.abort_flag == q + 1) return false;
      // per-iteration trace: the first update of a node in iteration it
      // sees the node's value at the end of iteration it-1
      if (TRACE && it > 0) {
        const bool first_upd = is_sync_u ? (si.pos_u == 0) : (si.pos_v == 0);
        if (first_upd) {
          const float* src = is_sync_u ? sm.uh[parity] : sm.vh[parity];
          const float* src_lo = is_sync_u ? sm.ul[parity] : sm.vl[parity];
          double mn = __builtin_inf();
          for (int s2 = lane; s2 < L; s2 += 64) mn = __builtin_fmin(mn, (double)src[s2] + (double)src_lo[s2]);
#pragma unroll
          for (int o = 32; o >= 1; o >>= 1) mn = __builtin_fmin(mn, __shfl_xor(mn, o, 64));
          if (lane == 0) v.trace[(size_t)(it - 1) * v.n + (is_sync_u ? si.u : si.v)] = mn;
        }
      }
      // LDS-resident mode: the next slot starts a matching (or the next
      // iteration) and may read what this slot wrote
      if (LDSU && (si_next.step != si.step || nxt <= slot)) __syncthreads();
      si = si_next;
      parity ^= 1;
      if (++j == owned) { j = 0; ++it; }
    }
    return true;
  }

  // ---- compute waves ----
  // output lane of this thread
  constexpr int VPW = LT / S::W;
  static_assert(VPW <= 4 * (16 - S::BR), "column outputs per wave");
  static_assert(S::BR <= 8, "row outputs in the first half of a row block");
  const bool out_u = cb < S::BR;
  const int out_s = rb * S::BR + cb;
  const int lw = (rb & 3) * (16 - S::BR) + (cb - S::BR);
  const int out_t = wave * VPW + lw;
  const bool out_v = !out_u && lw < VPW && (FULL || out_t < L);
  const bool out_uk = out_u && (FULL || out_s < L);
  const int out_i = out_u ? out_s : out_t;     // label of the output
  const int out_ic = out_i < L ? out_i : L - 1;  // in range for every lane
  static_assert(DEPTH == 1 || DEPTH == 2, "prefetch depth");
  constexpr int RING = DEPTH + 1;
  float t0[S::BR][S::BC], t1[S::BR][S::BC], t2[S::BR][S::BC];
  // old messages of a step: this thread's rows (into u) and columns (into
  // v), and its output column's
  struct PhiSet {
    float pu[S::BR], pv[S::BC], pvo;
  };
  PhiSet f0, f1, f2;
  auto load_phiset = [&](PhiSet& f, int jq) __attribute__((always_inline)) {
    const float* src = phi_of(first + jq * stride, jq);
    load_phi<LT, NT, PHI_LDS, FULL>(src, L, f.pu, f.pv);
    f.pvo = src[L + out_ic];  // (used by column lanes only)
  };
  // The messages of step q + DEPTH are last written by this workgroup at
  // step q + DEPTH - owned.  PHI_FAR (the caller guarantees owned >= DEPTH
  // + 2): that step's writes are behind a barrier when step q starts, so
  // they are prefetched DEPTH steps ahead with the tables.  Otherwise each
  // step reads its own messages right after its first barrier.
  // Positions (iteration, owned index) of the current step and of the step
  // DEPTH ahead, advanced without divisions.
  int it = 0, j = 0, jp = 0;
  {
    const int j1 = owned > 1 ? 1 : 0;
    if constexpr (KIND == kCostDense) {
      load_tile_raw<LT, NT, FULL>(v.tables + (size_t)first * L * L, L, t0);
      if (DEPTH == 2) load_tile_raw<LT, NT, FULL>(v.tables + (size_t)(first + j1 * stride) * L * L, L, t1);
    } else {
      gen_tile<LT, NT, KIND>(v.tables + (size_t)first * cost_params(KIND), t0);
      if (DEPTH == 2) gen_tile<LT, NT, KIND>(v.tables + (size_t)(first + j1 * stride) * cost_params(KIND), t1);
    }
    if (PHI_FAR) {
      load_phiset(f0, 0);
      if (DEPTH == 2) load_phiset(f1, j1);
    }
    jp = DEPTH % owned;
  }
  SlotInfo si = ld_const(v.slots + first);
  int parity = 0;
  // one step: compute on tile xc with messages fc, start loading the table
  // and messages of step q + DEPTH into xp, fp (the ring position used one
  // step earlier, free again)
  auto step = [&](float (&xc)[S::BR][S::BC], float (&xp)[S::BR][S::BC], PhiSet& fc, PhiSet& fp, int q)
                  __attribute__((always_inline)) -> bool {
    float (&pu)[S::BR] = fc.pu;
    float (&pv)[S::BC] = fc.pv;
    const int slot = first + j * stride;
    const unsigned want_u = (unsigned)it * (unsigned)si.deg_u + (unsigned)si.pos_u;
    const unsigned want_v = (unsigned)it * (unsigned)si.deg_v + (unsigned)si.pos_v;
    int nxt = slot + stride;
    if (nxt >= v.m) nxt = first;
    nxt = uni(nxt);
    const bool last_iter = it == iters - 1;
    // metadata of the next owned slot, off the dependency chain
    const SlotInfo si_next = ld_const(v.slots + nxt);
    {
      // (past the end: a harmless reload of the last step's table)
      const int jq = q + DEPTH < total ? jp : owned - 1;
      if constexpr (KIND == kCostDense) load_tile_raw<LT, NT, FULL>(v.tables + (size_t)(first + jq * stride) * L * L, L, xp);
      else gen_tile<LT, NT, KIND>(v.tables + (size_t)(first + jq * stride) * cost_params(KIND), xp);
      if (PHI_FAR) load_phiset(fp, jq);
    }
    // This lane's mailbox target and version need no result of the passes:
    // formed here, before the step's barriers (the empty asm keeps them here
    // rather than at their use, on the step's critical path).
    const int node = out_u ? si.u : si.v;
    const bool outk = out_uk || out_v;
    unsigned long long* mb_dst = nullptr;
    unsigned ver = 0;
    if (!LDSU) {
      mb_dst = outk ? v.mb + (size_t)node * L + out_i : v.sink + (tid & ~63);
      ver = (out_u ? want_u : want_v) + 1;
      asm volatile("" ::"v"(mb_dst), "v"(ver));
    }
    // (and the next slot's metadata is loaded here, not late in the step)
    asm volatile("" ::"s"(si_next.u), "s"(si_next.v), "s"(si_next.pos_u), "s"(si_next.pos_v), "s"(si_next.deg_u),
                 "s"(si_next.deg_v));
#if MPLPXX_FINE_STAMPS
    if (v.stamps && last_iter && tid == 0) v.stamps[(size_t)slot * kStampStride + 4] = wall_clock64();
#endif
    __syncthreads();
    if (!PHI_FAR) load_phiset(fc, j);
    pad_tile<LT, NT, FULL>(L, xc);
#if MPLPXX_FINE_STAMPS
    if (v.stamps && last_iter && tid == 0) v.stamps[(size_t)slot * kStampStride + 5] = wall_clock64();
#endif
    // a' = centred U - phi (padded labels read label L-1: any finite value works)
    float av[S::BC], au[S::BR];
#pragma unroll
    for (int jj = 0; jj < S::BC; ++jj) {
      const int t = cb * S::BC + jj;
      av[jj] = sm.uv[parity][(FULL || t < L) ? t : L - 1] - pv[jj];
    }
#pragma unroll
    for (int i = 0; i < S::BR; ++i) {
      const int s = rb * S::BR + i;
      au[i] = sm.uu[parity][(FULL || s < L) ? s : L - 1] - pu[i];
    }
    // the old value (hi, lo) and message of this lane's output; the shift
    // between the centred passes and the messages
    const float ohi = out_u ? sm.uh[parity][out_ic] : sm.vh[parity][out_ic];
    const float olo = out_u ? sm.ul[parity][out_ic] : sm.vl[parity][out_ic];
    const float delta = 0.5f * (sm.cc[parity][0] - sm.cc[parity][1]);
    float ophi = fc.pvo;
    if (out_u) {
      ophi = pu[0];
#pragma unroll
      for (int i = 1; i < S::BR; ++i)
        if (cb == i) ophi = pu[i];
    }
    // pass 1: p(s) = min_t [th(s,t) + a_v(t)], b = (a_u - p) / 2
    // ((M), Sec. 4: the column pass takes a_u itself, b = a_u)
    static_assert(RULE == MPLPXX_RULE_H || ((RULE == MPLPXX_RULE_M || RULE == MPLPXX_RULE_U) && !TRACE), "update rule");
    float b[S::BR], pm[S::BR];
    {
#pragma unroll
      for (int i = 0; i < S::BR; ++i) {
        float mn = xc[i][0] + av[0];
#pragma unroll
        for (int jj = 1; jj < S::BC; ++jj) mn = vmin(mn, xc[i][jj] + av[jj]);
        pm[i] = mn;
      }
      row16_min_n<S::BR>(pm);
#pragma unroll
      for (int i = 0; i < S::BR; ++i) b[i] = RULE == MPLPXX_RULE_M ? au[i] : 0.5f * (au[i] - pm[i]);
    }
    // pass 2: q(t) = min_s [th(s,t) + b(s)]  ((M): p'(t) = min_s [th(s,t) + a_u(s)];
    // (U): instead this wave's part of G = min over real rows of a'_u(s) + p(s))
    float qv[S::BC];
    if constexpr (RULE == MPLPXX_RULE_U) {
      float gm = __builtin_inff();
#pragma unroll
      for (int i = 0; i < S::BR; ++i)
        if (FULL || rb * S::BR + i < L) gm = vmin(gm, au[i] + pm[i]);
      gm = col4_min(gm);
      if (lane == 0) sm.red[wave][0] = gm;
#pragma unroll
      for (int jj = 0; jj < S::BC; ++jj) qv[jj] = 0.0f;
    } else {
#pragma unroll
      for (int jj = 0; jj < S::BC; ++jj) {
        float mn = xc[0][jj] + b[0];
#pragma unroll
        for (int i = 1; i < S::BR; ++i) mn = vmin(mn, xc[i][jj] + b[i]);
        qv[jj] = mn;
      }
      col4_min_store<S::BC>(qv, sm.red[wave], cb, lane);
    }
    // The head of this lane's compensated update needs only the old value
    // and message: done before the mid-step barrier (the empty asm keeps it
    // there; the compiler would otherwise sink it to its use after the
    // barrier, on the step's critical path).
    float cd, ce1;
    comp_update_head(ohi, ophi, cd, ce1);
    asm volatile("" : "+v"(cd), "+v"(ce1));
#if MPLPXX_FINE_STAMPS
    if (v.stamps && last_iter && tid == 0) v.stamps[(size_t)slot * kStampStride + 6] = wall_clock64();
#endif
    __syncthreads();  // mid-step barrier (the sync waves take part)
#if MPLPXX_FINE_STAMPS
    if (v.stamps && last_iter && tid == 0) v.stamps[(size_t)slot * kStampStride + 7] = wall_clock64();
#endif
    // The waves' partial column minima, every read issued before the first
    // use (one LDS round trip), and the abort flag with them.
    float part[S::W][S::BC], opart[S::W];
#pragma unroll
    for (int w = 0; w < S::W; ++w) {
#pragma unroll
      for (int jj = 0; jj < S::BC; ++jj) part[w][jj] = sm.red[w][cb * S::BC + jj];
      opart[w] = sm.red[w][out_ic];
    }
    const int aborted = sm.abort_flag;
    __builtin_amdgcn_sched_barrier(0);
    if (aborted == q + 1) return false;
#pragma unroll
    for (int jj = 0; jj < S::BC; ++jj) {
      float mn = part[0][jj];
#pragma unroll
      for (int w = 1; w < S::W; ++w) mn = vmin(mn, part[w][jj]);
      qv[jj] = mn;
    }
    // the output column's message q' + delta, q' reduced the same way
    // ((M): (p' - a'_v)/2 + delta; (U): (G/2 - a'_v) + delta)
    float omsg;
    float ghalf = 0.0f;
    if constexpr (RULE == MPLPXX_RULE_U) {
      float gm = sm.red[0][0];
#pragma unroll
      for (int w = 1; w < S::W; ++w) gm = vmin(gm, sm.red[w][0]);
      ghalf = 0.5f * gm;
      omsg = (ghalf - (sm.uv[parity][out_ic] - fc.pvo)) + delta;
    } else {
      float mn = opart[0];
#pragma unroll
      for (int w = 1; w < S::W; ++w) mn = vmin(mn, opart[w]);
      if constexpr (RULE == MPLPXX_RULE_M) omsg = 0.5f * (mn - (sm.uv[parity][out_ic] - fc.pvo)) + delta;
      else omsg = mn + delta;
    }
    // pass 3: r(s) = min_t [th(s,t) - q(t)]  ((M), (U): none; the row message
    // is (p - a'_u)/2 - delta, or (G/2 - a'_u) - delta)
    float r[S::BR];
    if constexpr (RULE == MPLPXX_RULE_M) {
#pragma unroll
      for (int i = 0; i < S::BR; ++i) r[i] = 0.5f * (pm[i] - au[i]);
    } else if constexpr (RULE == MPLPXX_RULE_U) {
#pragma unroll
      for (int i = 0; i < S::BR; ++i) r[i] = ghalf - au[i];
    } else {
#pragma unroll
      for (int i = 0; i < S::BR; ++i) {
        float mn = xc[i][0] - qv[0];
#pragma unroll
        for (int jj = 1; jj < S::BC; ++jj) mn = vmin(mn, xc[i][jj] - qv[jj]);
        r[i] = mn;
      }
      if (TRACE) {
        row16_min_n<S::BR>(r);  // (the trace needs every row's minimum)
      } else {
        // Only lane cb = i of a row block needs row i's minimum: three
        // exchanges leave each lane the minimum over its half row, then
        // lanes cb and 15 - cb both take row min(cb, 15 - cb) and one
        // mirrored exchange joins the halves (BR <= 8: every output lane
        // is in the first half).
        row16_min_n<S::BR, 3>(r);
        // (every lane finishes every half-row minimum first, so the choice
        // below stays a select instead of becoming divergent branches)
#pragma unroll
        for (int i = 0; i < S::BR; ++i) asm volatile("" : "+v"(r[i]));
        const int half_row = cb < 8 ? cb : 15 - cb;
        float sel = r[0];
#pragma unroll
        for (int i = 1; i < S::BR; ++i) sel = half_row == i ? r[i] : sel;
        r[0] = vmin(sel, dpp_f<0x140>(sel));
      }
    }
    if (TRACE) {
      // edge term of Eq. (3) after this update from the stored messages
      // rs = r' - delta, qs = q' + delta: min over real rows of
      // (fl(th - qs) - rs) + err(th - qs), exact up to one rounding of a
      // number near zero; padded rows are skipped, padded columns stay
      // near BIG/2
      float em = __builtin_inff();
#pragma unroll
      for (int i = 0; i < S::BR; ++i) {
        const int s = rb * S::BR + i;
        const float rs = r[i] - delta;
        if (FULL || s < L) {
#pragma unroll
          for (int jj = 0; jj < S::BC; ++jj) {
            const float qs = qv[jj] + delta;
            const float d = xc[i][jj] - qs;
            em = vmin(em, (d - rs) + two_sum_err(xc[i][jj], -qs, d));
          }
        }
      }
      em = col4_min(row16_min(em));
      if (lane == 0) v.trace_e[((size_t)it * v.m + slot) * S::W + wave] = em;
    }
    if (out_u) {
      float rr = r[0];
      if (RULE != MPLPXX_RULE_H || TRACE) {
#pragma unroll
        for (int i = 1; i < S::BR; ++i)
          if (cb == i) rr = r[i];
      }
      omsg = rr - delta;
    }
    // push back: the new unary through the mailbox, the message to memory.
    // Every lane issues the same global stores (lanes without an output
    // write one scratch word per wave, so that a store instruction touches
    // no more cache lines than its real outputs need): a store that only
    // some waves skip would leave the compiler unsure how many memory
    // operations are in flight, and it would then wait for all of them,
    // prefetches too.
    float* phi_w = phi_of(slot, j);
    float nhi, nlo;
    comp_update_tail(cd, ce1, olo, omsg, nhi, nlo);
    if (LDSU) {
      if (outk) {
        v.lds_hi[(size_t)node * L + out_i] = nhi;
        v.lds_lo[(size_t)node * L + out_i] = (unsigned short)(__float_as_uint(nlo) >> 16);
      }
    } else {
      mb_store(mb_dst, mb_pack(nhi, nlo, ver));
    }
    if (PHI_LDS) {
      if (outk) phi_w[(out_u ? 0 : L) + out_i] = omsg;
    } else {
      *(outk ? phi_w + (out_u ? 0 : L) + out_i : reinterpret_cast<float*>(v.sink + NT + (tid >> 6))) = omsg;
    }
    {
      const bool st = v.stamps && last_iter && tid == 0;
      long long* dst = st ? v.stamps + (size_t)slot * kStampStride + 3
                          : reinterpret_cast<long long*>(v.sink + NT + 64 + (tid >> 6));
      *dst = st ? (long long)wall_clock64() : 0;
    }
    // LDS-resident mode: the next slot starts a matching (or the next
    // iteration) and may read what this slot wrote
    if (LDSU && (si_next.step != si.step || nxt <= slot)) __syncthreads();
    si = si_next;
    parity ^= 1;
    if (++j == owned) { j = 0; ++it; }
    if (++jp == owned) jp = 0;
    return true;
  };
  // whole turns of the ring in the loop (every path through its body issues
  // the same memory operations, so the compiler can count the loads in
  // flight exactly), then the remaining steps
  int q = 0;
  if (RING == 2) {
    for (; q + 2 <= total; q += 2) {
      if (!step(t0, t1, f0, f1, q)) return false;
      if (!step(t1, t0, f1, f0, q + 1)) return false;
    }
    if (q < total && !step(t0, t1, f0, f1, q)) return false;
  } else {
    for (; q + 3 <= total; q += 3) {
      if (!step(t0, t2, f0, f2, q)) return false;
      if (!step(t1, t0, f1, f0, q + 1)) return false;
      if (!step(t2, t1, f2, f1, q + 2)) return false;
    }
    if (q < total && !step(t0, t2, f0, f2, q)) return false;
    if (q + 1 < total && !step(t1, t0, f1, f0, q + 1)) return false;
  }
  return true;
}

}  // namespace mplpxx
