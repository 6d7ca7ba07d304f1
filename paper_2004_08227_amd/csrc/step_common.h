// Shared memory and gather of the one-update-per-workgroup kernels (the
// per-matching engine and its variants): a_u = U_u - phi[0] and
// a_v = U_v - phi[1] of one edge, centred in FP32 (Sec. 4, Eq. (2); the
// centring is described in device_common.h).
#pragma once
#include <type_traits>

#include "device_common.h"

namespace mplpxx {

template <typename T, int LT, int NT> struct Smem {
  T au[LT];
  T av[LT];
  T red[TileShape<T, LT, NT>::W][LT];
  T nu[LT];
  T nv[LT];
  // FP32: old hi, lo and message of each label (compensated update), and
  // the references of the centred passes (see device_common.h)
  T hu[LT], lu[LT], ou[LT];
  T hv[LT], lv[LT], ov[LT];
  T cu, cv;
  int abort_flag;
};
template <typename T> constexpr bool kComp = std::is_same<T, float>::value;

// a_u = U_u - phi[0], a_v = U_v - phi[1] into smem (FP32: the centred
// ((hi - c) + lo) - phi with c = min_s hi(s) per node, see device_common.h)
template <typename T, int LT, int NT, bool kCoherent>
__device__ __forceinline__ void gather(Smem<T, LT, NT>& sm, int L, const T* __restrict__ phi_slot, const T* Uu,
                                       const T* Uv, const T* Lu, const T* Lv) {
  const int tid = threadIdx.x;
  if constexpr (!kComp<T>) {
    for (int s = tid; s < 2 * LT; s += NT) {
      if (s < LT) {
        if (s < L) sm.au[s] = (kCoherent ? ldv_dev(Uu + s) : Uu[s]) - phi_slot[s];
      } else {
        const int t = s - LT;
        if (t < L) sm.av[t] = (kCoherent ? ldv_dev(Uv + t) : Uv[t]) - phi_slot[L + t];
      }
    }
  } else {
    for (int s = tid; s < 2 * LT; s += NT) {
      if (s < LT) {
        if (s < L) {
          sm.hu[s] = kCoherent ? ldv_dev(Uu + s) : Uu[s];
          sm.lu[s] = kCoherent ? ldv_dev(Lu + s) : Lu[s];
          sm.ou[s] = phi_slot[s];
        }
      } else {
        const int t = s - LT;
        if (t < L) {
          sm.hv[t] = kCoherent ? ldv_dev(Uv + t) : Uv[t];
          sm.lv[t] = kCoherent ? ldv_dev(Lv + t) : Lv[t];
          sm.ov[t] = phi_slot[L + t];
        }
      }
    }
    __syncthreads();
    // wave 0: c_u, wave 1: c_v (min is exact, any order)
    const int wave = tid >> 6, lane = tid & 63;
    if (wave < 2) {
      const T* h = wave == 0 ? sm.hu : sm.hv;
      T c = inf_v<T>();
      for (int s = lane; s < L; s += 64) c = vmin(c, h[s]);
      c = col4_min(row16_min(c));
      if (lane == 0) (wave == 0 ? sm.cu : sm.cv) = c;
    }
    __syncthreads();
    for (int s = tid; s < 2 * LT; s += NT) {
      if (s < LT) {
        if (s < L) sm.au[s] = ((sm.hu[s] - sm.cu) + sm.lu[s]) - sm.ou[s];
      } else {
        const int t = s - LT;
        if (t < L) sm.av[t] = ((sm.hv[t] - sm.cv) + sm.lv[t]) - sm.ov[t];
      }
    }
  }
  __syncthreads();
}

}  // namespace mplpxx
