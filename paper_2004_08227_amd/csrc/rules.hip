// The other BCA-updates of Sec. 4 on the per-matching engine: MPLP (M) and
// the uniform update (U), for the comparison the paper makes between them
// and MPLP++ (H) (Sec. 5: one iteration of (H) dominates (M), which
// dominates (U); Sec. 7: time to reach the dual bound).
//
// In message form, with a_u = U_u - phi[0], a_v = U_v - phi[1] and the
// aggregated cost g(s,t) = th(s,t) + a_u(s) + a_v(t) of Sec. 4:
//   p(s)  = min_t [th(s,t) + a_v(t)]      (row minima of g are a_u + p)
//   p'(t) = min_s [th(s,t) + a_u(s)]      (column minima of g are a_v + p')
//   G     = min_s [a_u(s) + p(s)]          (minimum of g)
// (M): theta_u = (a_u + p)/2, theta_v = (a_v + p')/2, so the new messages
//      are phi[0] = (p - a_u)/2 and phi[1] = (p' - a_v)/2;
// (U): theta_u = theta_v = G/2, so phi[0] = G/2 - a_u, phi[1] = G/2 - a_v.
// FP32 runs the passes on the centred a'_u = a_u - c_u, a'_v = a_v - c_v
// (c = min_s hi, as for (H)); (M) and (U) are invariant under the shift up
// to delta = (c_u - c_v)/2: phi[0] = phi'[0] - delta, phi[1] = phi'[1] +
// delta, where phi' are the formulas above on the centred values.  The new
// unaries are the same compensated sums as for (H).
//
// One workgroup per edge update, the register tile of the per-matching
// engine (pads +inf).
#include "step_common.h"

namespace mplpxx {

template <typename T, int LT, int NT, int RULE>
__device__ __forceinline__ void rule_passes(const T (&x)[TileShape<T, LT, NT>::BR][TileShape<T, LT, NT>::BC],
                                            Smem<T, LT, NT>& sm, int L, T* __restrict__ phi_slot, T* __restrict__ Uu,
                                            T* __restrict__ Uv, T* __restrict__ Lu, T* __restrict__ Lv) {
  using S = TileShape<T, LT, NT>;
  const int tid = threadIdx.x;
  const int rb = tid >> 4, cb = tid & 15;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  T av[S::BC], au[S::BR];
#pragma unroll
  for (int j = 0; j < S::BC; ++j) {
    const int t = cb * S::BC + j;
    av[j] = (t < L) ? sm.av[t] : T(0);
  }
#pragma unroll
  for (int i = 0; i < S::BR; ++i) {
    const int s = rb * S::BR + i;
    au[i] = (s < L) ? sm.au[s] : T(0);
  }
  // p(s) = min_t [th(s,t) + a_v(t)]   (padded columns: th = +inf)
  T p[S::BR];
#pragma unroll
  for (int i = 0; i < S::BR; ++i) {
    T mn = x[i][0] + av[0];
#pragma unroll
    for (int j = 1; j < S::BC; ++j) mn = vmin(mn, x[i][j] + av[j]);
    p[i] = row16_min(mn);
  }
  T delta = T(0);
  if constexpr (kComp<T>) delta = T(0.5) * (sm.cu - sm.cv);
  T out_u[S::BR], out_v[S::BC];   // new messages phi[0] (rows), phi[1] (columns)
  if constexpr (RULE == 1) {
    // p'(t) = min_s [th(s,t) + a_u(s)]   (padded rows: th = +inf)
    T pp[S::BC];
#pragma unroll
    for (int j = 0; j < S::BC; ++j) {
      T mn = x[0][j] + au[0];
#pragma unroll
      for (int i = 1; i < S::BR; ++i) mn = vmin(mn, x[i][j] + au[i]);
      pp[j] = col4_min(mn);
    }
    if constexpr (S::W > 1) {
      if (lane < 16) {
#pragma unroll
        for (int j = 0; j < S::BC; ++j) sm.red[wave][cb * S::BC + j] = pp[j];
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < S::BC; ++j) {
        const int t = cb * S::BC + j;
        T mn = sm.red[0][t];
#pragma unroll
        for (int w = 1; w < S::W; ++w) mn = vmin(mn, sm.red[w][t]);
        pp[j] = mn;
      }
    }
#pragma unroll
    for (int i = 0; i < S::BR; ++i) out_u[i] = T(0.5) * (p[i] - au[i]) - delta;
#pragma unroll
    for (int j = 0; j < S::BC; ++j) out_v[j] = T(0.5) * (pp[j] - av[j]) + delta;
  } else {
    // G = min over the real rows of a_u(s) + p(s)
    T gm = inf_v<T>();
#pragma unroll
    for (int i = 0; i < S::BR; ++i) {
      const int s = rb * S::BR + i;
      if (s < L) gm = vmin(gm, au[i] + p[i]);
    }
    gm = col4_min(gm);
    if constexpr (S::W > 1) {
      if (lane == 0) sm.red[wave][0] = gm;
      __syncthreads();
      gm = sm.red[0][0];
#pragma unroll
      for (int w = 1; w < S::W; ++w) gm = vmin(gm, sm.red[w][0]);
    }
    const T half = T(0.5) * gm;
#pragma unroll
    for (int i = 0; i < S::BR; ++i) out_u[i] = (half - au[i]) - delta;
#pragma unroll
    for (int j = 0; j < S::BC; ++j) out_v[j] = (half - av[j]) + delta;
  }
  // push back: phi[1] and U_v by row block 0, phi[0] and U_u by column block 0
  if (rb == 0) {
#pragma unroll
    for (int j = 0; j < S::BC; ++j) {
      const int t = cb * S::BC + j;
      if (t < L) {
        T nvv, nvl = T(0);
        if constexpr (kComp<T>) comp_update(sm.hv[t], sm.lv[t], sm.ov[t], out_v[j], nvv, nvl);
        else nvv = av[j] + out_v[j];
        phi_slot[L + t] = out_v[j];
        Uv[t] = nvv;
        if constexpr (kComp<T>) Lv[t] = nvl;
      }
    }
  }
  if (cb == 0) {
#pragma unroll
    for (int i = 0; i < S::BR; ++i) {
      const int s = rb * S::BR + i;
      if (s < L) {
        T nuu, nul = T(0);
        if constexpr (kComp<T>) comp_update(sm.hu[s], sm.lu[s], sm.ou[s], out_u[i], nuu, nul);
        else nuu = au[i] + out_u[i];
        phi_slot[s] = out_u[i];
        Uu[s] = nuu;
        if constexpr (kComp<T>) Lu[s] = nul;
      }
    }
  }
}

// one launch per matching, one workgroup per edge of it
template <typename T, int LT, int NT, int RULE>
__global__ void __launch_bounds__(NT) k_step_rule(HsArgs<T> a, int slot_begin) {
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
  rule_passes<T, LT, NT, RULE>(x, sm, L, phi_slot, Uu, Uv, Lu, Lv);
}

template <typename T>
hipError_t launch_step_rule(const HsArgs<T>& a, int rule, int LT, int NT, int slot_begin, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (rule != 1 && rule != 2) return hipErrorInvalidValue;
#define MPLPXX_CASE(lt, nt)                                                                           \
  if (LT == lt && NT == nt) {                                                                         \
    if (rule == 1) hipLaunchKernelGGL((k_step_rule<T, lt, nt, 1>), dim3(count), dim3(nt), 0, st, a, slot_begin); \
    else hipLaunchKernelGGL((k_step_rule<T, lt, nt, 2>), dim3(count), dim3(nt), 0, st, a, slot_begin);           \
    return hipGetLastError();                                                                         \
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
  return hipErrorInvalidValue;
}

template hipError_t launch_step_rule<float>(const HsArgs<float>&, int, int, int, int, int, hipStream_t);
template hipError_t launch_step_rule<double>(const HsArgs<double>&, int, int, int, int, int, hipStream_t);

}  // namespace mplpxx
