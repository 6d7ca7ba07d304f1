// Adjoint (reverse mode) of K unrolled MPLP++ iterations.
//
// Loss: D_K = sum_u min_s U_u(s) after K iterations from phi = 0.  After an
// edge's (H) update its reparametrized pairwise term theta - r - q has row
// minima 0 (Sec. 4, after (H)), so it stays identically 0 under small input
// changes and the dual bound of Eq. (3) reduces to the node terms.
//
// Forward of one update (three-minimization form of (H)), with the argmin
// records the reverse needs (lowest index on ties); in FP32 the unaries are
// updated with the same compensated sum as in the other engines, which
// changes no derivative:
//   p(s) = min_t [th(s,t) + a_v(t)]   t1(s) = argmin
//   b(s) = (a_u(s) - p(s)) / 2
//   q(t) = min_s [th(s,t) + b(s)]     s2(t) = argmin
//   r(s) = min_t [th(s,t) - q(t)]     t3(s) = argmin
//   phi0' = r, phi1' = q, U_u' = a_u + r, U_v' = a_v + q,
//   a_u = U_u - phi0, a_v = U_v - phi1.
// Reverse, given the adjoints Ub_u', Ub_v' of the new unaries and pb0', pb1'
// of the new messages:
//   rb = pb0' + Ub_u',  qb = pb1' + Ub_v'
//   r:  thb(s, t3(s)) += rb(s);  qb(t3(s)) -= rb(s)
//   q:  thb(s2(t), t) += qb(t);  bb(s2(t)) += qb(t)
//   b:  ab_u = Ub_u' + bb / 2;   pb = -bb / 2
//   p:  thb(s, t1(s)) += pb(s);  ab_v = Ub_v' + sum over s with t1(s)=t of pb(s)
//   Ub_u = ab_u, pb0 = -ab_u, Ub_v = ab_v, pb1 = -ab_v.
// Every scatter is done by one thread per target in ascending index order, so
// the result is deterministic.  One workgroup per edge, one launch per
// matching: the edges of a matching are independent in reverse as forward.
#include <type_traits>

#include "device_common.h"

namespace mplpxx {

template <typename T> __device__ __forceinline__ T inf_of();
template <> __device__ __forceinline__ float inf_of<float>() { return __builtin_inff(); }
template <> __device__ __forceinline__ double inf_of<double>() { return __builtin_inf(); }

constexpr int kAdjNT = 256;

// Forward of one matching with argmin records: rec[slot][0..L) = t1,
// [L..2L) = s2, [2L..3L) = t3.  Same values, bit for bit, as the other engines
// (each entry one IEEE add, exact minimum).
template <typename T>
__global__ void __launch_bounds__(kAdjNT) k_step_record(const T* __restrict__ tables, T* __restrict__ phi,
                                                        T* __restrict__ U, T* __restrict__ Ulo,
                                                        const SlotInfo* __restrict__ slots, int L, int slot_begin,
                                                        unsigned char* __restrict__ rec) {
  constexpr bool kComp = std::is_same<T, float>::value;
  __shared__ T au[MPLPXX_MAX_LABELS], av[MPLPXX_MAX_LABELS], b[MPLPXX_MAX_LABELS], q[MPLPXX_MAX_LABELS];
  __shared__ T hu[MPLPXX_MAX_LABELS], lu[MPLPXX_MAX_LABELS], ou[MPLPXX_MAX_LABELS];
  __shared__ T hv[MPLPXX_MAX_LABELS], lv[MPLPXX_MAX_LABELS], ov[MPLPXX_MAX_LABELS];
  __shared__ T cuv[2];
  const int slot = slot_begin + blockIdx.x;
  const SlotInfo si = slots[slot];
  const T* th = tables + (size_t)slot * L * L;
  T* ph = phi + (size_t)slot * 2 * L;
  T* Uu = U + (size_t)si.u * L;
  T* Uv = U + (size_t)si.v * L;
  unsigned char* rc = rec + (size_t)slot * 3 * L;
  const int tid = threadIdx.x;
  T delta = T(0);
  if constexpr (!kComp) {
    for (int i = tid; i < L; i += kAdjNT) {
      au[i] = Uu[i] - ph[i];
      av[i] = Uv[i] - ph[L + i];
    }
  } else {
    // centred passes, as in the other FP32 engines (device_common.h)
    for (int i = tid; i < L; i += kAdjNT) {
      hu[i] = Uu[i];
      lu[i] = Ulo[(size_t)si.u * L + i];
      ou[i] = ph[i];
      hv[i] = Uv[i];
      lv[i] = Ulo[(size_t)si.v * L + i];
      ov[i] = ph[L + i];
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63;
    if (wave < 2) {
      const T* h = wave == 0 ? hu : hv;
      T c = inf_of<T>();
      for (int i = lane; i < L; i += 64) c = vmin(c, h[i]);
      c = col4_min(row16_min(c));
      if (lane == 0) cuv[wave] = c;
    }
    __syncthreads();
    for (int i = tid; i < L; i += kAdjNT) {
      au[i] = ((hu[i] - cuv[0]) + lu[i]) - ou[i];
      av[i] = ((hv[i] - cuv[1]) + lv[i]) - ov[i];
    }
    delta = T(0.5) * (cuv[0] - cuv[1]);
  }
  __syncthreads();
  for (int s = tid; s < L; s += kAdjNT) {  // pass 1
    T mn = inf_of<T>();
    int arg = 0;
    for (int t = 0; t < L; ++t) {
      const T x = th[(size_t)s * L + t] + av[t];
      if (x < mn) { mn = x; arg = t; }
    }
    b[s] = T(0.5) * (au[s] - mn);
    rc[s] = (unsigned char)arg;
  }
  __syncthreads();
  for (int t = tid; t < L; t += kAdjNT) {  // pass 2
    T mn = inf_of<T>();
    int arg = 0;
    for (int s = 0; s < L; ++s) {
      const T x = th[(size_t)s * L + t] + b[s];
      if (x < mn) { mn = x; arg = s; }
    }
    q[t] = mn;
    rc[L + t] = (unsigned char)arg;
  }
  __syncthreads();
  for (int s = tid; s < L; s += kAdjNT) {  // pass 3
    T mn = inf_of<T>();
    int arg = 0;
    for (int t = 0; t < L; ++t) {
      const T x = th[(size_t)s * L + t] - q[t];
      if (x < mn) { mn = x; arg = t; }
    }
    rc[2 * L + s] = (unsigned char)arg;
    const T rs = mn - delta;
    ph[s] = rs;
    if constexpr (kComp) comp_update(hu[s], lu[s], ou[s], rs, Uu[s], Ulo[(size_t)si.u * L + s]);
    else Uu[s] = au[s] + mn;
  }
  for (int t = tid; t < L; t += kAdjNT) {
    const T qs = q[t] + delta;
    ph[L + t] = qs;
    if constexpr (kComp) comp_update(hv[t], lv[t], ov[t], qs, Uv[t], Ulo[(size_t)si.v * L + t]);
    else Uv[t] = av[t] + q[t];
  }
}

// Reverse of one matching.  Ub [n][L] adjoints of the unaries, pb [m][2][L]
// of the messages (slot order), thb [m][L][L] accumulated table adjoints.
template <typename T>
__global__ void __launch_bounds__(kAdjNT) k_adj_step(const SlotInfo* __restrict__ slots, int L, int slot_begin,
                                                     const unsigned char* __restrict__ rec, T* __restrict__ Ub,
                                                     T* __restrict__ pb, T* __restrict__ thb) {
  __shared__ T rb[MPLPXX_MAX_LABELS], qb[MPLPXX_MAX_LABELS], bb[MPLPXX_MAX_LABELS], pbv[MPLPXX_MAX_LABELS];
  __shared__ T abu[MPLPXX_MAX_LABELS], abv[MPLPXX_MAX_LABELS];
  __shared__ unsigned char t1[MPLPXX_MAX_LABELS], s2[MPLPXX_MAX_LABELS], t3[MPLPXX_MAX_LABELS];
  const int slot = slot_begin + blockIdx.x;
  const SlotInfo si = slots[slot];
  T* Ubu = Ub + (size_t)si.u * L;
  T* Ubv = Ub + (size_t)si.v * L;
  T* p = pb + (size_t)slot * 2 * L;
  T* g = thb + (size_t)slot * L * L;
  const unsigned char* rc = rec + (size_t)slot * 3 * L;
  const int tid = threadIdx.x;
  for (int i = tid; i < L; i += kAdjNT) {
    t1[i] = rc[i];
    s2[i] = rc[L + i];
    t3[i] = rc[2 * L + i];
    rb[i] = p[i] + Ubu[i];
    qb[i] = p[L + i] + Ubv[i];
    abu[i] = Ubu[i];
    abv[i] = Ubv[i];
  }
  __syncthreads();
  // r = th(s, t3) - q(t3)
  for (int s = tid; s < L; s += kAdjNT) g[(size_t)s * L + t3[s]] += rb[s];
  for (int t = tid; t < L; t += kAdjNT) {
    T acc = qb[t];
    for (int s = 0; s < L; ++s)
      if (t3[s] == t) acc -= rb[s];
    qb[t] = acc;
  }
  __syncthreads();
  // q = th(s2, t) + b(s2)
  for (int t = tid; t < L; t += kAdjNT) g[(size_t)s2[t] * L + t] += qb[t];
  for (int s = tid; s < L; s += kAdjNT) {
    T acc = T(0);
    for (int t = 0; t < L; ++t)
      if (s2[t] == s) acc += qb[t];
    bb[s] = acc;
  }
  __syncthreads();
  // b = (a_u - p) / 2
  for (int s = tid; s < L; s += kAdjNT) {
    abu[s] += T(0.5) * bb[s];
    pbv[s] = -T(0.5) * bb[s];
  }
  __syncthreads();
  // p = th(s, t1) + a_v(t1)
  for (int s = tid; s < L; s += kAdjNT) g[(size_t)s * L + t1[s]] += pbv[s];
  for (int t = tid; t < L; t += kAdjNT) {
    T acc = abv[t];
    for (int s = 0; s < L; ++s)
      if (t1[s] == t) acc += pbv[s];
    abv[t] = acc;
  }
  __syncthreads();
  // a_u = U_u - phi0, a_v = U_v - phi1
  for (int i = tid; i < L; i += kAdjNT) {
    Ubu[i] = abu[i];
    p[i] = -abu[i];
    Ubv[i] = abv[i];
    p[L + i] = -abv[i];
  }
}

// Seed for D_K = sum_u min_s U_u: one-hot at the smallest minimizing label;
// loss partial per node in FP64 (FP32: U + Ulo, exact in FP64).
template <typename T>
__global__ void __launch_bounds__(64) k_adj_seed(const T* __restrict__ U, const T* __restrict__ Ulo, int L,
                                                 T* __restrict__ Ub, double* __restrict__ node_min) {
  const int u = blockIdx.x;
  const int lane = threadIdx.x;
  double best = __builtin_inf();
  int arg = 0x7fffffff;
  for (int s = lane; s < L; s += 64) {
    const size_t i = (size_t)u * L + s;
    const double x = (double)U[i] + (Ulo ? (double)Ulo[i] : 0.0);
    if (x < best) { best = x; arg = s; }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double ob = __shfl_xor(best, o, 64);
    const int oa = __shfl_xor(arg, o, 64);
    if (ob < best || (ob == best && oa < arg)) { best = ob; arg = oa; }
  }
  for (int s = lane; s < L; s += 64) Ub[(size_t)u * L + s] = (s == arg) ? T(1) : T(0);
  if (lane == 0) node_min[u] = best;
}

template <typename T>
hipError_t launch_step_record(const T* tables, T* phi, T* U, T* Ulo, const SlotInfo* slots, int L, int slot_begin,
                              int count, unsigned char* rec, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_step_record<T>, dim3(count), dim3(kAdjNT), 0, st, tables, phi, U, Ulo, slots, L, slot_begin,
                     rec);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_step(const SlotInfo* slots, int L, int slot_begin, int count, const unsigned char* rec, T* Ub,
                           T* pb, T* thb, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_step<T>, dim3(count), dim3(kAdjNT), 0, st, slots, L, slot_begin, rec, Ub, pb, thb);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_seed(const T* U, const T* Ulo, int n, int L, T* Ub, double* node_min, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_seed<T>, dim3(n), dim3(64), 0, st, U, Ulo, L, Ub, node_min);
  return hipGetLastError();
}

#define MPLPXX_INST(T)                                                                                        \
  template hipError_t launch_step_record<T>(const T*, T*, T*, T*, const SlotInfo*, int, int, int,            \
                                            unsigned char*, hipStream_t);                                     \
  template hipError_t launch_adj_step<T>(const SlotInfo*, int, int, int, const unsigned char*, T*, T*, T*,    \
                                         hipStream_t);                                                        \
  template hipError_t launch_adj_seed<T>(const T*, const T*, int, int, T*, double*, hipStream_t);
MPLPXX_INST(float)
MPLPXX_INST(double)
#undef MPLPXX_INST

}  // namespace mplpxx
