// Wave engine: one wavefront performs one whole handshake update (Sec. 4,
// (H)) on its own, with no workgroup barrier inside an update.  A workgroup
// of NW waves is NW independent workers, so a compute unit keeps many edge
// updates in flight at once (the mailbox engine runs one at a time per
// workgroup and waits on two barriers per update).  Used by the batched
// solver for models with L <= 64.
//
// Lane layout.  The L x L table (padded to LT = 16, 32 or 64) sits on an 8 x 8
// grid of lanes: lane = 8 rb + cb holds rows rb B .. rb B + B - 1 and columns
// cb B .. cb B + B - 1, B = LT / 8, in registers.  A minimum over t of a row
// is an in-register minimum and one over the 8 lanes of an octet (lane bits
// 0..2); a minimum over s of a column is an in-register minimum and one over
// the 8 lanes with the same cb (lane bits 3..5).  Per-label vectors (the
// unaries, the messages, the results) are in "label order": lane l holds
// label l.  A small per-wave LDS area turns label order into the grid's rows
// and columns and back.
//
// Arithmetic.  Every value is formed by the same IEEE operations, in the same
// order, as in the mailbox engine (centred passes, exact minima, the same
// compensated unary update), so both engines give bitwise the same results.
//
// Ordering between updates.  The slots of a model are dealt to the workers
// round-robin in schedule order; each worker takes its slots in order.  An
// update of edge (u, v) in iteration it waits until node u has seen exactly
// it * deg(u) + pos_u updates in this launch (and the same for v), which is
// the state the sequential schedule gives it.  Every wait is for an earlier
// slot, so the worker holding the earliest unfinished slot never waits and
// the run cannot deadlock.
//  * LDS mode (a model on one workgroup): the unaries are in LDS (hi FP32, lo
//    bf16) with one update counter per node; a worker polls the two
//    counters, and publishes an update by writing the values, waiting for
//    its LDS writes to complete, then bumping the counters.
//  * Mailbox mode (a model on a team of workgroups, or without LDS room):
//    the unaries are in the tagged 64-bit mailbox words of the mailbox
//    engine (value and version in one word), polled and written with
//    device-scope atomic accesses.
// The messages of a slot are read and written only by the worker that owns
// the slot, each label by the same lane, so they need no synchronisation.
#pragma once
#include "device_common.h"
#include "potts_passes.h"

namespace mplpxx {

// per-wave LDS: a' of both nodes in label order, and the pass results
struct WvScratch {
  float au[64];
  float av[64];
  float rr[64];
  float qq[64];
};

// Stops the compiler from moving memory operations across this point (LDS
// exchanges between the lanes of one wave need no hardware wait: a wave's
// LDS operations execute in order).
__device__ __forceinline__ void wave_sync() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// minimum over the 8 lanes of an octet (lane bits 0..2), N values at once
template <int N> __device__ __forceinline__ void oct_min_n(float (&x)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) x[k] = vmin(x[k], dpp_f<0xB1>(x[k]));   // lane ^ 1
#pragma unroll
  for (int k = 0; k < N; ++k) x[k] = vmin(x[k], dpp_f<0x4E>(x[k]));   // lane ^ 2
#pragma unroll
  for (int k = 0; k < N; ++k) x[k] = vmin(x[k], dpp_f<0x141>(x[k]));  // the other quad of the octet
}
// minimum over the 8 lanes with the same lane & 7 (lane bits 3..5)
template <int N> __device__ __forceinline__ void stripe_min_n(float (&x)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) x[k] = vmin(x[k], dpp_f<0x128>(x[k]));  // row_ror:8 = lane ^ 8
#pragma unroll
  for (int k = 0; k < N; ++k) x[k] = col4_min(x[k]);                  // lanes ^ 16, ^ 32
}
__device__ __forceinline__ float wave_min(float x) { return col4_min(row16_min(x)); }

template <int LT> struct WvShape {
  static constexpr int B = LT / 8;
  static_assert(LT == 16 || LT == 32 || LT == 64, "wave engine tile");
};

// One model as the wave engine sees it.
struct WvView {
  const float* tables;          // [m][L][L] slot order
  float* phi;                   // [m][2][L] slot order
  unsigned long long* mb;       // [n][L] mailboxes (mailbox mode)
  const SlotInfo* slots;        // [m]
  int L, m, n;
  float* lds_hi;                // LDS mode: [n][L] hi of the unaries
  unsigned short* lds_lo;       //           [n][L] bf16 bits of lo
  int* lds_ver;                 //           [n] updates of each node so far
  unsigned long long* sink;     // this wave's 192 scratch words (stores of lanes without an output)
};

// Table of one slot into the grid layout: offb[i] is the byte offset of
// this lane's segment of row rb B + i, rows clamped into the table, columns
// not (a row's segment runs on into the next row, or into the allocation's
// zeroed tail), so every entry is finite and below 2^100 in magnitude.
//
// The padded labels are masked on the vectors instead of the tile (no
// per-entry selects): a padded column gets a_v = BIG (pass 1) and q' - BIG
// = -BIG (pass 3); a padded row gets a_u = 2^127, so b = (2^127 - p)/2
// rounds to BIG (pass 2).  A padded entry then sums to BIG and never wins a
// minimum over real labels, and every real minimum is bitwise the one over
// the real entries, as with the padded tiles of the mailbox engine.
template <int LT>
__device__ __forceinline__ void wv_load_tile(const float* __restrict__ tab, int L, int rb, int cb,
                                             float (&x)[LT / 8][LT / 8]) {
  constexpr int B = LT / 8;
  const char* base = reinterpret_cast<const char*>(tab);
#pragma unroll
  for (int i = 0; i < B; ++i) {
    const int s = rb * B + i;
    const unsigned offb = (unsigned)(((s < L ? s : L - 1) * L + cb * B) * 4);
#pragma unroll
    for (int j = 0; j < B; ++j) x[i][j] = reinterpret_cast<const float*>(base + (size_t)offb)[j];
  }
}
// A copy of x that the compiler cannot see through: values derived from it
// are recomputed where they are used instead of being kept in registers for
// the whole loop.
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}


// Runs `iters` iterations over the slots first, first + stride, ... of one
// model on this wave.  Returns false if a wait timed out or another worker
// gave up (then *abort is set for the workgroup and err for the launch).
// PHI_FAR (the caller guarantees at least two owned slots): the messages of
// the next slot are loaded one slot ahead.  LT <= 32 also loads the next
// table one slot ahead (a second register tile); LT = 64 loads each table at
// the start of its own update, and other waves of the compute unit cover the
// latency.
//
// KIND: 0 dense tables; MPLPXX_COST_POTTS / _TRUNC_LINEAR: structured costs
// with their parameters per slot in v.tables (cost_params floats each); the
// passes then run in label order, no tile.
template <int LT, bool LDSU, bool PHI_FAR, int KIND = kCostDense>
__device__ __forceinline__ bool wv_run(const WvView& v_in, int first_in, int stride_in, int iters_in,
                                       WvScratch& scr, long long spin_limit, int* err, int* abort) {
  constexpr int B = WvShape<LT>::B;
  constexpr bool POTTS = KIND != kCostDense;   // (any structured cost)
  constexpr bool PRE = LT <= 32 && !POTTS;
  WvView v = v_in;
  v.L = uni(v.L);
  v.m = uni(v.m);
  v.n = uni(v.n);
  const int first = uni(first_in), stride = uni(stride_in), iters = uni(iters_in);
  if (first >= v.m) return true;
  const int L = v.L;
  const int lane = threadIdx.x & 63, rb = lane >> 3, cb = lane & 7;
  const bool lout = lane < L;                  // this lane's label is real
  const int li = lout ? lane : L - 1;          // in range for every lane
  const int owned = (v.m - first + stride - 1) / stride;
  const int total = owned * iters;
  const float kInf = __builtin_inff();

  float t0[B][B], t1[B][B];
  float f0u = 0.f, f0v = 0.f, f1u = 0.f, f1v = 0.f;
  int it = 0, j = 0, jn = owned > 1 ? 1 : 0;
  if (PRE) wv_load_tile<LT>(v.tables + (size_t)first * L * L, L, rb, cb, t0);
  if (PHI_FAR) {
    const float* p = v.phi + (size_t)first * 2 * L;
    f0u = p[li];
    f0v = p[L + li];
  }
  SlotInfo si = ld_const(v.slots + first);

  // one update on tile xc (loaded) with messages fu/fv (PHI_FAR: loaded);
  // loads the next slot's table into xn (PRE) and messages into gu/gv
  // (PHI_FAR)
  auto step = [&](float (&xc)[B][B], float (&xn)[B][B], float& fu, float& fv, float& gu, float& gv)
                  __attribute__((always_inline)) -> bool {
    const int slot = first + j * stride;
    // (lane positions recomputed per update: loop-invariant row offsets and
    // pads would hold registers the 64-label tile needs)
    const int ln = opaque(threadIdx.x) & 63, rbl = ln >> 3, cbl = ln & 7;
    const unsigned want_u = (unsigned)it * (unsigned)si.deg_u + (unsigned)si.pos_u;
    const unsigned want_v = (unsigned)it * (unsigned)si.deg_v + (unsigned)si.pos_v;
    const int nslot = uni(first + jn * stride);
    const SlotInfo si_next = ld_const(v.slots + nslot);
    auto prefetch = [&]() __attribute__((always_inline)) {
      if (PRE) wv_load_tile<LT>(v.tables + (size_t)nslot * L * L, L, rbl, cbl, xn);
      if (PHI_FAR) {
        const float* p = v.phi + (size_t)nslot * 2 * L;
        gu = p[li];
        gv = p[L + li];
      }
    };
    if (!PRE && !POTTS) wv_load_tile<LT>(v.tables + (size_t)slot * L * L, L, rbl, cbl, xc);
    const float* prm = v.tables + (size_t)slot * cost_params(KIND);
    if (!PHI_FAR) {
      const float* p = v.phi + (size_t)slot * 2 * L;
      fu = p[li];
      fv = p[L + li];
    }
    // LDS mode: the prefetches go out now (LDS polls do not wait on them);
    // mailbox mode: after the poll, so that the poll does not queue behind
    // them in the in-order memory counter
    if (LDSU) prefetch();
    // ---- wait for both nodes, read their unaries in label order ----
    float hu, lu, hv, lv;
    {
      long long spins = 0;
      if (LDSU) {
        for (;;) {
          const unsigned cu = (unsigned)__hip_atomic_load(v.lds_ver + si.u, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
          const unsigned cv = (unsigned)__hip_atomic_load(v.lds_ver + si.v, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (cu == want_u && cv == want_v) break;
          if (++spins > spin_limit || ((spins & 63) == 0 && (*(volatile int*)abort != 0 || ld_dev(err) != 0))) {
            if (lane == 0) {
              if (spins > spin_limit) report_timeout(err, slot, cu != want_u ? si.u : si.v, cu != want_u ? want_u : want_v,
                                                     cu != want_u ? cu : cv);
              *(volatile int*)abort = 1;
            }
            return false;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        wave_sync();
        hu = v.lds_hi[(size_t)si.u * L + li];
        lu = __uint_as_float((unsigned)v.lds_lo[(size_t)si.u * L + li] << 16);
        hv = v.lds_hi[(size_t)si.v * L + li];
        lv = __uint_as_float((unsigned)v.lds_lo[(size_t)si.v * L + li] << 16);
      } else {
        const unsigned long long* pu = v.mb + (size_t)si.u * L + li;
        const unsigned long long* pv = v.mb + (size_t)si.v * L + li;
        unsigned long long wu, wv;
        for (;;) {
          wu = mb_load(pu);
          wv = mb_load(pv);
          const bool ok = mb_ver(wu) == (want_u & 0xFFFFu) && mb_ver(wv) == (want_v & 0xFFFFu);
          if (__all(ok)) break;
          if (++spins > spin_limit || ((spins & 255) == 0 && (*(volatile int*)abort != 0 || ld_dev(err) != 0))) {
            if (lane == 0) {
              if (spins > spin_limit) {
                const bool bad_u = mb_ver(wu) != (want_u & 0xFFFFu);
                report_timeout(err, slot, bad_u ? si.u : si.v, (bad_u ? want_u : want_v) & 0xFFFFu,
                               bad_u ? mb_ver(wu) : mb_ver(wv));
              }
              *(volatile int*)abort = 1;
            }
            return false;
          }
        }
        hu = mb_hi(wu);
        lu = mb_lo(wu);
        hv = mb_hi(wv);
        lv = mb_lo(wv);
        prefetch();
      }
    }
    const float c_u = wave_min(lout ? hu : kInf);
    const float c_v = wave_min(lout ? hv : kInf);
    const float delta = 0.5f * (c_u - c_v);
    float phu, phv;
    if constexpr (POTTS) {
      // centred a' in label order; the three passes by min_other
      const float au = ((hu - c_u) + lu) - fu;
      const float av = ((hv - c_v) + lv) - fv;
      structured_passes<KIND>(au, av, prm, lout, L, delta, phu, phv);
    } else {
      // ---- centred a' in label order, then into the grid ----
      scr.au[lane] = lout ? ((hu - c_u) + lu) - fu : 0x1p127f;
      scr.av[lane] = lout ? ((hv - c_v) + lv) - fv : kPadBig;
      wave_sync();
      float au[B], av[B];
  #pragma unroll
      for (int i = 0; i < B; ++i) au[i] = scr.au[rb * B + i];
  #pragma unroll
      for (int jj = 0; jj < B; ++jj) av[jj] = scr.av[cb * B + jj];
      // pass 1: p(s) = min_t [th(s,t) + a_v(t)], b = (a_u - p) / 2
      float b[B];
      {
        float pm[B];
  #pragma unroll
        for (int i = 0; i < B; ++i) {
          float mn = xc[i][0] + av[0];
  #pragma unroll
          for (int jj = 1; jj < B; ++jj) mn = vmin(mn, xc[i][jj] + av[jj]);
          pm[i] = mn;
        }
        oct_min_n<B>(pm);
  #pragma unroll
        for (int i = 0; i < B; ++i) b[i] = 0.5f * (au[i] - pm[i]);
      }
      // pass 2: q(t) = min_s [th(s,t) + b(s)]
      float qv[B];
  #pragma unroll
      for (int jj = 0; jj < B; ++jj) {
        float mn = xc[0][jj] + b[0];
  #pragma unroll
        for (int i = 1; i < B; ++i) mn = vmin(mn, xc[i][jj] + b[i]);
        qv[jj] = mn;
      }
      stripe_min_n<B>(qv);
      float qm[B];
  #pragma unroll
      for (int jj = 0; jj < B; ++jj) qm[jj] = cbl * B + jj < L ? qv[jj] : -kPadBig;
      // pass 3: r(s) = min_t [th(s,t) - q(t)]
      float r[B];
  #pragma unroll
      for (int i = 0; i < B; ++i) {
        float mn = xc[i][0] - qm[0];
  #pragma unroll
        for (int jj = 1; jj < B; ++jj) mn = vmin(mn, xc[i][jj] - qm[jj]);
        r[i] = mn;
      }
      oct_min_n<B>(r);
      // ---- results back to label order ----
      {
        // (every lane of an octet holds the same r, every lane of a stripe
        // the same q: one lane of each writes its B values)
        if (cb == 0) {
  #pragma unroll
          for (int i = 0; i < B; ++i) scr.rr[rb * B + i] = r[i];
        }
        if (rb == 0) {
  #pragma unroll
          for (int jj = 0; jj < B; ++jj) scr.qq[cb * B + jj] = qv[jj];
        }
      }
      wave_sync();
      phu = scr.rr[li] - delta;   // new message into u
      phv = scr.qq[li] + delta;   // new message into v
    }
    float nhu, nlu, nhv, nlv;
    comp_update(hu, lu, fu, phu, nhu, nlu);
    comp_update(hv, lv, fv, phv, nhv, nlv);
    // ---- publish ----
    // (every lane issues the same global stores; lanes without a label
    // write this wave's scratch words, so the count of memory operations in
    // flight never depends on L)
    {
      float* pw = v.phi + (size_t)slot * 2 * L;
      float* sk = reinterpret_cast<float*>(v.sink + 128);
      *(lout ? pw + lane : sk + lane) = phu;
      *(lout ? pw + L + lane : sk + 64 + lane) = phv;
    }
    if (LDSU) {
      if (lout) {
        v.lds_hi[(size_t)si.u * L + lane] = nhu;
        v.lds_lo[(size_t)si.u * L + lane] = (unsigned short)(__float_as_uint(nlu) >> 16);
        v.lds_hi[(size_t)si.v * L + lane] = nhv;
        v.lds_lo[(size_t)si.v * L + lane] = (unsigned short)(__float_as_uint(nlv) >> 16);
      }
      // (release stores at workgroup scope: a wave whose acquire poll reads
      // these versions reads the unaries above)
      if (lane == 0) {
        __hip_atomic_store(v.lds_ver + si.u, (int)(want_u + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_store(v.lds_ver + si.v, (int)(want_v + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    } else {
      mb_store(lout ? v.mb + (size_t)si.u * L + lane : v.sink + lane, mb_pack(nhu, nlu, want_u + 1));
      mb_store(lout ? v.mb + (size_t)si.v * L + lane : v.sink + 64 + lane, mb_pack(nhv, nlv, want_v + 1));
    }
    si = si_next;
    j = jn;
    if (j == 0) ++it;
    jn = jn + 1 == owned ? 0 : jn + 1;
    return true;
  };
  int q = 0;
  if (PRE || PHI_FAR) {
    // two steps per turn: the tiles and message registers swap roles
    for (; q + 2 <= total; q += 2) {
      if (!step(t0, t1, f0u, f0v, f1u, f1v)) return false;
      if (!step(PRE ? t1 : t0, t0, f1u, f1v, f0u, f0v)) return false;
    }
  }
  for (; q < total; ++q)
    if (!step(t0, t1, f0u, f0v, f1u, f1v)) return false;
  return true;
}

}  // namespace mplpxx
