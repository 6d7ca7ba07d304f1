// The passes of (H) on an edge with a structured pairwise cost (Potts,
// truncated linear, truncated quadratic), in label order (lane l holds label l): shared by the
// wave engine and the mailbox engine's structured instance.
#pragma once
#include "device_common.h"

namespace mplpxx {

// ---------------------------------------------------------------------------
// Potts pairwise terms th(s,t) = w [s != t] (Sec. 4: the message-passing
// minimization then takes O(L)).  Every pass of (H) has the form
//   y(s) = min_t fl(th(s,t) + x(t)) = min( fl(0 + x(s)), fl(w + min_{t != s} x(t)) ),
// exactly, because fl(w + .) is monotone: the minimum over t != s of the
// rounded sums is the rounded sum with the minimum.  So the passes need,
// per label s, the minimum of x over the other labels: the smallest value
// when s is not where it is attained, else the second smallest.  Pass 3,
// min_t fl(th(s,t) - q(t)), is the same with x = -q (exact negation).  The
// results are bitwise the dense passes on the table w [s != t]: no
// candidate of either is -0 (fl(+0 + x) and fl(w + x), w != -0, never
// are), so the minima agree whatever a minimum makes of signed zeros.
// The diagonal term is added as a +0 the compiler cannot see: a visible
// constant lets it rewrite fl(0 - q) under a minimum as -q, which is -0
// for q = +0.
// ---------------------------------------------------------------------------
// (opaque_zero and ld_const_f: device_common.h)
// (m1, m2) <- the two smallest of the multiset {m1, m2} + {o1, o2}, each
// pair being the two smallest of a group of lanes (a repeated value counts
// twice)
__device__ __forceinline__ void min2_merge(float& m1, float& m2, float o1, float o2) {
  const float hi = __builtin_fmaxf(m1, o1);
  m1 = vmin(m1, o1);
  m2 = vmin(hi, vmin(m2, o2));
}
template <int CTRL> __device__ __forceinline__ void min2_dpp(float& m1, float& m2) {
  min2_merge(m1, m2, dpp_f<CTRL>(m1), dpp_f<CTRL>(m2));
}
// per lane (label) s: min over the real labels t != s of x(t) (+inf if
// none).  The two smallest values of the wave, m1 <= m2, by a butterfly
// over the lanes (DPP within rows of 16, then the row swaps); a label
// holding m1 gets m2 (equal to m1 when the minimum is repeated), any other
// label m1.  Which zero a minimum of +0 and -0 returns does not matter
// here: the result only enters fl(w + .) with w != -0.  With L <= 16 every
// label is in the first row of 16 lanes and the row swaps are skipped;
// with L <= 32, the second one (L is the same on every lane).
__device__ __forceinline__ float min_other(float x, bool real, int L) {
  const float kInf = __builtin_inff();
  float m1 = real ? x : kInf;
  float m2;
  {
    const float o = dpp_f<0xB1>(m1);   // lane ^ 1 (m2 is +inf on both sides)
    m2 = __builtin_fmaxf(m1, o);
    m1 = vmin(m1, o);
  }
  min2_dpp<0x4E>(m1, m2);              // lane ^ 2
  min2_dpp<0x141>(m1, m2);             // row_half_mirror: the other quad of the octet
  min2_dpp<0x140>(m1, m2);             // row_mirror: the other octet of the row
  if (L > 16) {
    auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(m1), __float_as_uint(m1), false, false);
    auto b = __builtin_amdgcn_permlane16_swap(__float_as_uint(m2), __float_as_uint(m2), false, false);
    m1 = __uint_as_float(a[0]);
    m2 = __uint_as_float(b[0]);
    min2_merge(m1, m2, __uint_as_float(a[1]), __uint_as_float(b[1]));
  }
  if (L > 32) {
    auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(m1), __float_as_uint(m1), false, false);
    auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(m2), __float_as_uint(m2), false, false);
    m1 = __uint_as_float(a[0]);
    m2 = __uint_as_float(b[0]);
    min2_merge(m1, m2, __uint_as_float(a[1]), __uint_as_float(b[1]));
  }
  return (real && x == m1) ? m2 : m1;
}

// New messages of one (H) update of a Potts edge, per lane (label): au, av
// are the centred a'_u, a'_v of this label, w the edge's weight, delta the
// shift between the centred passes and the messages.
__device__ __forceinline__ void potts_passes(float au, float av, float w, bool lout, int L, float delta, float& phu,
                                             float& phv) {
  const float z = opaque_zero();   // th(s,s)
  const float p = vmin(z + av, w + min_other(av, lout, L));
  const float b = 0.5f * (au - p);
  const float q = vmin(z + b, w + min_other(b, lout, L));
  const float nq = -q;
  const float r = vmin(z - q, w + min_other(nq, lout, L));
  phu = r - delta;   // new message into u
  phv = q + delta;   // new message into v
}

// ---------------------------------------------------------------------------
// Truncated linear terms th(s,t) = fl(w min(|s - t|, tau)), w, tau >= 0 (Sec.
// 4 names absolute-difference costs among those whose message passing takes
// O(|Y|)).  A pass y(s) = min_t [x(t) + th(s,t)] is the distance transform
//   y(s) = min( min_t [x(t) + w |s - t|],  min_t x(t) + fl(w tau) ):
// a label farther than tau costs x(t) + w tau >= min x + w tau, and a nearer
// one x(t) + w |s - t| <= x(t) + w tau.  The first term is a prefix minimum
// (labels t <= s) and a suffix minimum (t >= s) of x(t) + w |s - t|, formed
// by doubling distances: after the steps d = 1, 2, 4, 8 (DPP row shifts,
// adding w d, exact for these powers of two) each label holds the minimum
// over the labels of its row of 16 lanes; the rows are then joined by the
// carry of the earlier (later) rows' ends, through at most three rows.  The
// sums are rounded in a different order than fl(x(t) + fl(w |s - t|)), so
// the pass agrees with the expanded table up to a few FP32 roundings.
// ---------------------------------------------------------------------------
template <int CTRL> __device__ __forceinline__ float dpp_shift_inf(float x) {
  // lanes whose source is outside the row keep +inf
  return __int_as_float(__builtin_amdgcn_update_dpp((int)0x7f800000, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_value(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ float tl_pass(float x, bool real, float w, float wt, int L) {
  const float kInf = __builtin_inff();
  const float xs = real ? x : kInf;
  float f = xs, g = xs;   // from labels below / above
  f = vmin(f, dpp_shift_inf<0x111>(f) + w);   // row_shr:1
  g = vmin(g, dpp_shift_inf<0x101>(g) + w);   // row_shl:1
  const float w2 = 2.0f * w, w4 = 4.0f * w, w8 = 8.0f * w;
  f = vmin(f, dpp_shift_inf<0x112>(f) + w2);
  g = vmin(g, dpp_shift_inf<0x102>(g) + w2);
  f = vmin(f, dpp_shift_inf<0x114>(f) + w4);
  g = vmin(g, dpp_shift_inf<0x104>(g) + w4);
  f = vmin(f, dpp_shift_inf<0x118>(f) + w8);
  g = vmin(g, dpp_shift_inf<0x108>(g) + w8);
  float xm = row16_min(xs);
  if (L > 16) {
    const int lane = threadIdx.x & 63, row = lane >> 4, k = lane & 15;
    const float w16 = 16.0f * w;
    // c_r: min over the labels of the rows below r of x(t) + w (16 r - 1 - t)
    const float c1 = lane_value(f, 15);
    const float c2 = vmin(lane_value(f, 31), c1 + w16);
    const float c3 = vmin(lane_value(f, 47), c2 + w16);
    const float c = row == 0 ? kInf : row == 1 ? c1 : row == 2 ? c2 : c3;
    // d_r: min over the labels of the rows above r of x(t) + w (t - 16 (r + 1))
    const float d2 = lane_value(g, 48);
    const float d1 = vmin(lane_value(g, 32), d2 + w16);
    const float d0 = vmin(lane_value(g, 16), d1 + w16);
    const float d = row == 3 ? kInf : row == 2 ? d2 : row == 1 ? d1 : d0;
    f = vmin(f, c + w * (float)(k + 1));
    g = vmin(g, d + w * (float)(16 - k));
    xm = col4_min(xm);
  }
  return vmin(vmin(f, g), xm + wt);
}

// ---------------------------------------------------------------------------
// Truncated quadratic terms th(s,t) = fl(w min((s - t)^2, tau)), w, tau >= 0
// (Sec. 4 names quadratic costs among those whose message passing needs no
// L x L table).  No table is read: lane s holds the L costs of its row, each
// formed from the two parameters exactly as the expanded table's entry
// ((s - t)^2 is exact in FP32, then one rounded product), and a pass takes
// y(s) = min_t fl(x(t) + th(s,t)) over every candidate t, x(t) coming from
// lane t as a wave-uniform value.  Each candidate is the same single IEEE
// add as in the dense passes, and no candidate is -0 (the costs are >= +0
// and a sum is -0 only when both terms are), so the minimum, and with it
// every update, is bitwise that of the dense engine on the expanded table.
// The pass takes L steps with L lanes; the table's 4 L^2 bytes become 8.
// ---------------------------------------------------------------------------
// costs of this lane's row s = lane: c[t] = fl(w min((s - t)^2, tau))
__device__ __forceinline__ void tq_costs(float w, float tau, float (&c)[64]) {
  const float fs = (float)(threadIdx.x & 63);
#pragma unroll
  for (int t = 0; t < 64; ++t) {
    const float d = fs - (float)t;
    c[t] = truncated_cost(w, tau, d * d);
  }
}
// y(s) = min over the real labels t of fl(x(t) + c[t]); labels t >= L are
// visited in whole groups of 8 at most, with x = +inf
__device__ __forceinline__ float tq_pass(float x, bool real, const float (&c)[64], int L) {
  const float xs = real ? x : __builtin_inff();
  float y0 = __builtin_inff(), y1 = __builtin_inff();
#pragma unroll
  for (int g = 0; g < 8; ++g) {
    if (8 * g < L) {
#pragma unroll
      for (int k = 0; k < 8; k += 2) {
        const int t = 8 * g + k;
        y0 = vmin(y0, lane_value(xs, t) + c[t]);
        y1 = vmin(y1, lane_value(xs, t + 1) + c[t + 1]);
      }
    }
  }
  return vmin(y0, y1);
}

// The same minimum over a window of distances.  Every label t with (s -
// t)^2 >= tau has th(s,t) = fl(w tau), so
//   y(s) = min( min_{|s - t| <= D} fl(x(t) + th(s,t)),  fl(min_t x(t) + fl(w tau)) )
// exactly for any D whose square reaches tau (the second term equals the
// smallest of the omitted candidates, and is no smaller than a candidate of
// the table when tau exceeds every (s - t)^2: fl(w .) is monotone).  The
// labels at distance d come from lanes s - d and s + d by one-lane wave
// shifts (DPP wave_shr:1, wave_shl:1; lanes shifted in from outside the
// wave hold +inf); distances are taken in groups of 4 up to D, and the
// extra ones of the last group are candidates of the table too.
__device__ __forceinline__ float tq_pass_window(float x, bool real, float w, float tau, int D) {
  const float kInf = __builtin_inff();
  const float xs = real ? x : kInf;
  float y = xs + truncated_cost(w, tau, opaque_zero());   // d = 0
  float xl = xs, xr = xs;
#pragma unroll
  for (int g = 0; g < 16; ++g) {
    if (4 * g + 1 <= D) {
#pragma unroll
      for (int k = 1; k <= 4; ++k) {
        const float d = (float)(4 * g + k);
        xl = dpp_shift_inf<0x138>(xl);   // wave_shr:1, from lane s - d
        xr = dpp_shift_inf<0x130>(xr);   // wave_shl:1, from lane s + d
        const float c = truncated_cost(w, tau, d * d);
        y = vmin(y, vmin(xl + c, xr + c));
      }
    }
  }
  return vmin(y, col4_min(row16_min(xs)) + w * tau);
}

// New messages of one (H) update of a structured edge, per lane (label): au,
// av are the centred a'_u, a'_v of this label, prm the edge's parameters
// (Potts: w; truncated linear and quadratic: w, tau), delta the shift
// between the centred passes and the messages.
template <int KIND>
__device__ __forceinline__ void structured_passes(float au, float av, const float* prm, bool lout, int L, float delta,
                                                  float& phu, float& phv) {
  if constexpr (KIND == MPLPXX_COST_TRUNC_QUAD) {
    const float w = ld_const_f(prm), tau = ld_const_f(prm + 1);
    // window of distances whose square reaches tau (one more than the
    // rounded square root, so its rounding cannot matter); the whole row
    // when that is most of it.  Both forms give the same bits.
    const int D = uni(min(L - 1, (int)__builtin_sqrtf(tau) + 1));
    if (2 * D < L) {
      const float p = tq_pass_window(av, lout, w, tau, D);
      const float b = 0.5f * (au - p);
      const float q = tq_pass_window(b, lout, w, tau, D);
      const float r = tq_pass_window(-q, lout, w, tau, D);
      phu = r - delta;
      phv = q + delta;
    } else {
      float c[64];
      tq_costs(w, tau, c);
      const float p = tq_pass(av, lout, c, L);
      const float b = 0.5f * (au - p);
      const float q = tq_pass(b, lout, c, L);
      const float r = tq_pass(-q, lout, c, L);
      phu = r - delta;
      phv = q + delta;
    }
  } else if constexpr (KIND == MPLPXX_COST_TRUNC_LINEAR) {
    const float w = ld_const_f(prm), tau = ld_const_f(prm + 1);
    const float wt = w * tau;   // the table's value beyond the truncation
    const float p = tl_pass(av, lout, w, wt, L);
    const float b = 0.5f * (au - p);
    const float q = tl_pass(b, lout, w, wt, L);
    const float r = tl_pass(-q, lout, w, wt, L);
    phu = r - delta;
    phv = q + delta;
  } else {
    potts_passes(au, av, ld_const_f(prm), lout, L, delta, phu, phv);
  }
}

}  // namespace mplpxx
