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
// the result is deterministic.  Per-matching kernels: one workgroup per
// edge, one launch per matching (the edges of a matching are independent in
// reverse as forward).  Persistent FP64 kernels (L <= 64, below): one launch
// per segment, with the same arithmetic in the same order.
#include <algorithm>
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

// ---------------------------------------------------------------------------
// Persistent FP64 adjoint (tiles up to 64 labels): one launch per segment of
// the checkpointed run for the recomputation with records, one for its
// reverse, instead of one launch per matching.
//
// Mailboxes.  A node's FP64 values (the unaries in the forward, their
// adjoints in the reverse) travel between workgroups as two 64-bit words per
// label, mb[node][label][h]: bits 0..31 hold the low (h = 0) or high (h = 1)
// half of the double, bits 32..63 the number of updates the node has had in
// this launch.  Each word is written and read with one device-scope atomic
// access, so a consumer that sees the version it waits for in both words of
// every label holds the values of that version: no flag, no fence.  (The
// FP32 engines pack value and version into one word the same way.)
//
// Slots are owned statically as in the other persistent engines: workgroup w
// runs slots w, w + G, ... in schedule order every iteration (the reverse in
// the opposite order), so an edge's messages, records and adjoints never
// leave one workgroup, and every wait is for an update earlier in the
// (forward or reverse) order: the workgroup holding the earliest unfinished
// one never waits.  Two sync waves poll the step's two nodes and deliver
// them to LDS (double buffered), as in the FP32 mailbox engine.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mb64_put(unsigned long long* row, int s, double x, unsigned ver) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned long long tag = (unsigned long long)ver << 32;
  mb_store(row + 2 * s, tag | (b & 0xffffffffull));
  mb_store(row + 2 * s + 1, tag | (b >> 32));
}

// sync wave: poll the 2L words of one node until every one carries `want`,
// then write their payloads to dst (2L 32-bit halves = L doubles)
template <int LT>
__device__ __forceinline__ bool mb64_gather(const unsigned long long* __restrict__ row, int L, unsigned want,
                                            unsigned* dst, long long spin_limit, const int* err, unsigned* seen_out) {
  const int lane = threadIdx.x & 63;
  constexpr int PER = (2 * LT + 63) / 64;
  bool have[PER];
  unsigned long long val[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) have[k] = (lane + 64 * k) >= 2 * L;
  long long spins = 0;
  for (;;) {
    bool all = true;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      if (!have[k]) {
        const unsigned long long w = mb_load(row + lane + 64 * k);
        if ((unsigned)(w >> 32) == want) {
          have[k] = true;
          val[k] = w;
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
        if (!have[k]) seen = (unsigned)(mb_load(row + lane + 64 * k) >> 32);
      for (int o = 32; o >= 1; o >>= 1) seen = min(seen, (unsigned)__shfl_xor((int)seen, o, 64));
      *seen_out = seen;
      return false;
    }
  }
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (lane + 64 * k < 2 * L) dst[lane + 64 * k] = (unsigned)val[k];
  return true;
}

__global__ void k_mb64_init(const double* __restrict__ x, unsigned long long* __restrict__ mb, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x[i]);
    mb[2 * i] = b & 0xffffffffull;
    mb[2 * i + 1] = b >> 32;
  }
}
__global__ void k_mb64_fini(double* __restrict__ x, const unsigned long long* __restrict__ mb, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    x[i] = __longlong_as_double((long long)((mb[2 * i] & 0xffffffffull) | (mb[2 * i + 1] << 32)));
}

// lowest-index minimum of (v, i) pairs: the other pair wins if smaller, or
// equal with a smaller index (its bits are kept, as a scan in index order
// keeps the first of equal values).  Written as selects: no branch.
__device__ __forceinline__ void argmin_merge(double& v, int& i, double ov, int oi) {
  const bool take = (ov < v) | ((ov == v) & (oi < i));
  v = take ? ov : v;
  i = take ? oi : i;
}
// the same when the other index is known to be the larger (a scan in index
// order): strictly smaller values win
__device__ __forceinline__ void argmin_next(double& v, int& i, double ov, int oi) {
  const bool take = ov < v;
  v = take ? ov : v;
  i = take ? oi : i;
}
template <int CTRL> __device__ __forceinline__ void argmin_dpp(double& v, int& i) {
  const double ov = dpp_f<CTRL>(v);
  const int oi = __builtin_amdgcn_update_dpp(0, i, CTRL, 0xF, 0xF, false);
  argmin_merge(v, i, ov, oi);
}
// over the 16 lanes of a row
__device__ __forceinline__ void row16_argmin(double& v, int& i) {
  argmin_dpp<0xB1>(v, i);
  argmin_dpp<0x4E>(v, i);
  argmin_dpp<0x141>(v, i);
  argmin_dpp<0x140>(v, i);
}
// over lanes l, l^16, l^32, l^48 (gfx950 permlane swaps of the two halves
// and the index: each lane gets its partner's values)
__device__ __forceinline__ double dbl_of(unsigned lo, unsigned hi) {
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ void col4_argmin(double& v, int& i) {
  {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    const auto ix = __builtin_amdgcn_permlane16_swap((unsigned)i, (unsigned)i, false, false);
    // each swap leaves this lane's own value in one half and the partner's
    // in the other; which is which is the same for all three
    const double a0 = dbl_of(lo[0], hi[0]), a1 = dbl_of(lo[1], hi[1]);
    double w = a0;
    int k = (int)ix[0];
    argmin_merge(w, k, a1, (int)ix[1]);
    v = w;
    i = k;
  }
  {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    const auto ix = __builtin_amdgcn_permlane32_swap((unsigned)i, (unsigned)i, false, false);
    double w = dbl_of(lo[0], hi[0]);
    int k = (int)ix[0];
    argmin_merge(w, k, dbl_of(lo[1], hi[1]), (int)ix[1]);
    v = w;
    i = k;
  }
}

constexpr int kF64NT = 256;  // compute threads of the FP64 mailbox forward

template <int LT> struct SmemF64 {
  double hu[2][LT];
  double hv[2][LT];
  double red[kF64NT / 64][LT];
  int redi[kF64NT / 64][LT];
  int abort_flag;
};

// Forward of `iters` iterations (FP64): the unaries in the mailboxes, the
// messages in phi (slot order).  REC: also the argmins of every update,
// rec[it][slot][0..L) = t1, [L..2L) = s2, [2L..3L) = t3, lowest index on
// ties, as the per-matching recording kernel gives them.  Every value is
// the same IEEE result as in the other FP64 kernels (one add per entry,
// exact minima, the same a_u, a_v), so the runs agree bit for bit.
struct Fwd64Args {
  const double* tables;
  double* phi;
  unsigned long long* mb;
  const SlotInfo* slots;
  int L, m, iters;
  unsigned char* rec;   // argmin records, or null (plain forward)
  int* err;
  long long spin_limit;
  int grid;             // workgroups of this role
};
template <int LT, bool REC>
__device__ __forceinline__ void fwd64_role(const Fwd64Args& a, int first, int G, SmemF64<LT>& sm) {
  const double* __restrict__ tables = a.tables;
  double* __restrict__ phi = a.phi;
  unsigned long long* __restrict__ mb = a.mb;
  const SlotInfo* __restrict__ slots = a.slots;
  unsigned char* __restrict__ rec = a.rec;
  const int L = a.L, m = a.m, iters = a.iters;
  int* err = a.err;
  const long long spin_limit = a.spin_limit;
  constexpr int NT = kF64NT;
  using S = TileShape<double, LT, NT>;
  const int tid = threadIdx.x;
  const int owned = (m - first + G - 1) / G;
  const int total = owned * iters;
  const size_t rec_it = (size_t)m * 3 * L;
  if (tid >= NT) {
    // ---- sync waves: wait for the step's two nodes ----
    const bool is_u = tid < NT + 64;
    int parity = 0, it = 0, j = 0;
    SlotInfo si = ld_const(slots + first);
    for (int q = 0; q < total; ++q) {
      const int slot = first + j * G;
      // metadata of the next owned slot, off the dependency chain
      const int nxt = uni(j + 1 == owned ? first : slot + G);
      const SlotInfo si_next = ld_const(slots + nxt);
      const int node = is_u ? si.u : si.v;
      const unsigned want = (unsigned)it * (unsigned)(is_u ? si.deg_u : si.deg_v) + (unsigned)(is_u ? si.pos_u : si.pos_v);
      unsigned seen = 0;
      unsigned* dst = reinterpret_cast<unsigned*>(is_u ? sm.hu[parity] : sm.hv[parity]);
      if (!mb64_gather<LT>(mb + (size_t)node * 2 * L, L, want, dst, spin_limit, err, &seen)) {
        if ((tid & 63) == 0) {
          if (ld_dev(err) == 0 || seen != want) report_timeout(err, slot, node, want, seen);
          sm.abort_flag = q + 1;
        }
      }
      __syncthreads();  // the step's nodes are in LDS
      __syncthreads();  // the compute waves' mid-step barrier
      if (sm.abort_flag == q + 1) return;
      si = si_next;
      parity ^= 1;
      if (++j == owned) { j = 0; ++it; }
    }
    return;
  }
  // ---- compute waves ----
  const int rb = tid >> 4, cb = tid & 15, wave = tid >> 6, lane = tid & 63;
  double x[S::BR][S::BC];
  double pu[S::BR], pv[S::BC];
  auto load_phi64 = [&](int slot) __attribute__((always_inline)) {
    const double* ph = phi + (size_t)slot * 2 * L;
#pragma unroll
    for (int i = 0; i < S::BR; ++i) {
      const int s = rb * S::BR + i;
      pu[i] = s < L ? ph[s] : 0.0;
    }
#pragma unroll
    for (int jj = 0; jj < S::BC; ++jj) {
      const int t = cb * S::BC + jj;
      pv[jj] = t < L ? ph[L + t] : 0.0;
    }
  };
  load_tile<double, LT, NT>(tables + (size_t)first * L * L, L, x);
  // (a workgroup that owns one slot reads back the messages it wrote at the
  // previous step: after the next step's first barrier)
  if (owned > 1) load_phi64(first);
  int parity = 0, it = 0, j = 0;
  SlotInfo si = ld_const(slots + first);
  for (int q = 0; q < total; ++q) {
    const int slot = first + j * G;
    const int nxt_slot = uni(j + 1 == owned ? first : slot + G);
    const SlotInfo si_next = ld_const(slots + nxt_slot);
    __syncthreads();  // the step's nodes are in LDS
    if (owned == 1) load_phi64(slot);
    double au[S::BR], av[S::BC];
#pragma unroll
    for (int jj = 0; jj < S::BC; ++jj) {
      const int t = cb * S::BC + jj;
      av[jj] = t < L ? sm.hv[parity][t] - pv[jj] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < S::BR; ++i) {
      const int s = rb * S::BR + i;
      au[i] = s < L ? sm.hu[parity][s] - pu[i] : 0.0;
    }
    // pass 1: p(s) = min_t [th(s,t) + a_v(t)], t1 = its lowest argmin
    double b[S::BR];
    int t1[S::BR];
#pragma unroll
    for (int i = 0; i < S::BR; ++i) {
      double mn = x[i][0] + av[0];
      int arg = cb * S::BC;
#pragma unroll
      for (int jj = 1; jj < S::BC; ++jj) argmin_next(mn, arg, x[i][jj] + av[jj], cb * S::BC + jj);
      row16_argmin(mn, arg);
      const int s = rb * S::BR + i;
      b[i] = s < L ? 0.5 * (au[i] - mn) : 0.0;
      t1[i] = arg;
    }
    // pass 2: q(t) = min_s [th(s,t) + b(s)], s2 = its lowest argmin
#pragma unroll
    for (int jj = 0; jj < S::BC; ++jj) {
      double mn = x[0][jj] + b[0];
      int arg = rb * S::BR;
#pragma unroll
      for (int i = 1; i < S::BR; ++i) argmin_next(mn, arg, x[i][jj] + b[i], rb * S::BR + i);
      col4_argmin(mn, arg);
      if (lane < 16) {
        sm.red[wave][cb * S::BC + jj] = mn;
        sm.redi[wave][cb * S::BC + jj] = arg;
      }
    }
    __syncthreads();  // mid-step barrier
    if (sm.abort_flag == q + 1) return;
    // waves hold ascending row ranges: merging them in order keeps the
    // lowest argmin
    double qv[S::BC];
    int s2[S::BC];
#pragma unroll
    for (int jj = 0; jj < S::BC; ++jj) {
      const int t = cb * S::BC + jj;
      double mn = sm.red[0][t];
      int arg = sm.redi[0][t];
#pragma unroll
      for (int w = 1; w < S::W; ++w) argmin_merge(mn, arg, sm.red[w][t], sm.redi[w][t]);
      qv[jj] = t < L ? mn : 0.0;
      s2[jj] = arg;
    }
    // pass 3: r(s) = min_t [th(s,t) - q(t)], t3 = its lowest argmin
    double r[S::BR];
    int t3[S::BR];
#pragma unroll
    for (int i = 0; i < S::BR; ++i) {
      double mn = x[i][0] - qv[0];
      int arg = cb * S::BC;
#pragma unroll
      for (int jj = 1; jj < S::BC; ++jj) argmin_next(mn, arg, x[i][jj] - qv[jj], cb * S::BC + jj);
      row16_argmin(mn, arg);
      r[i] = mn;
      t3[i] = arg;
    }
    // push back: U_u = a_u + r, phi[0] = r (column block 0), U_v = a_v + q,
    // phi[1] = q (row block 0)
    double* ph = phi + (size_t)slot * 2 * L;
    unsigned char* rc = rec + (size_t)it * rec_it + (size_t)slot * 3 * L;
    if (cb == 0) {
      const unsigned ver = (unsigned)it * (unsigned)si.deg_u + (unsigned)si.pos_u + 1u;
#pragma unroll
      for (int i = 0; i < S::BR; ++i) {
        const int s = rb * S::BR + i;
        if (s < L) {
          mb64_put(mb + (size_t)si.u * 2 * L, s, au[i] + r[i], ver);
          ph[s] = r[i];
          if (REC) {
            rc[s] = (unsigned char)t1[i];
            rc[2 * L + s] = (unsigned char)t3[i];
          }
        }
      }
    }
    if (rb == 0) {
      const unsigned ver = (unsigned)it * (unsigned)si.deg_v + (unsigned)si.pos_v + 1u;
#pragma unroll
      for (int jj = 0; jj < S::BC; ++jj) {
        const int t = cb * S::BC + jj;
        if (t < L) {
          mb64_put(mb + (size_t)si.v * 2 * L, t, av[jj] + qv[jj], ver);
          ph[L + t] = qv[jj];
          if (REC) rc[L + t] = (unsigned char)s2[jj];
        }
      }
    }
    si = si_next;
    parity ^= 1;
    if (++j == owned) { j = 0; ++it; }
    if (q + 1 < total && owned > 1) {
      load_tile<double, LT, NT>(tables + (size_t)nxt_slot * L * L, L, x);
      load_phi64(nxt_slot);
    }
  }
}

template <int LT> struct SmemR64 {
  double ubu[2][LT];
  double ubv[2][LT];
  int abort_flag;
};
// the double held by lane k, as a wave-uniform value
__device__ __forceinline__ double lane_double(double x, int k) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, k);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), k);
  return dbl_of(lo, hi);
}

// Reverse of `seg` recorded iterations (FP64, L <= 64): node adjoints in the
// mailboxes (version = updates of the node already reversed in this
// launch), message adjoints pb (slot order).  One compute wave, lane =
// label; the arithmetic of every adjoint is that of the per-matching reverse
// (same terms, same order), the sums over labels by wave-uniform values
// read from the other lanes, with no LDS round trip.  The table adjoints are not accumulated here:
// each reverse step writes its three scatter vectors rb, q-bar and p-bar to
// contrib[it][slot][3L] for k_thb_acc, which adds them in the per-matching
// kernel's order.
struct Rev64Args {
  const SlotInfo* slots;
  int L, m, seg;
  const unsigned char* rec;
  unsigned long long* mb;
  double* pb;
  double* contrib;
  int* err;
  long long spin_limit;
  int grid;             // workgroups of this role (0: no reverse in the launch)
};
template <int LT>
__device__ __forceinline__ void rev64_role(const Rev64Args& a, int first, int G, SmemR64<LT>& sm) {
  const SlotInfo* __restrict__ slots = a.slots;
  const unsigned char* __restrict__ rec = a.rec;
  unsigned long long* __restrict__ mb = a.mb;
  double* __restrict__ pb = a.pb;
  double* __restrict__ contrib = a.contrib;
  const int L = a.L, m = a.m, seg = a.seg;
  int* err = a.err;
  const long long spin_limit = a.spin_limit;
  const int tid = threadIdx.x;
  const int owned = (m - first + G - 1) / G;
  const int total = owned * seg;
  const size_t rec_it = (size_t)m * 3 * L;
  if (tid >= 64 && tid < kF64NT) {
    // ---- waves 1..3 are idle in this role: they take part in its barriers ----
    for (int q = 0; q < total; ++q) {
      __syncthreads();
      if (sm.abort_flag == q + 1) return;
    }
    return;
  }
  if (tid >= kF64NT) {
    // ---- sync waves ----
    const bool is_u = tid < kF64NT + 64;
    int parity = 0, done = 0, j = owned - 1;
    SlotInfo si = ld_const(slots + first + j * G);
    for (int q = 0; q < total; ++q) {
      const int slot = first + j * G;
      const int nxt = uni(j == 0 ? first + (owned - 1) * G : slot - G);
      const SlotInfo si_next = ld_const(slots + nxt);
      const int node = is_u ? si.u : si.v;
      const int deg = is_u ? si.deg_u : si.deg_v;
      const int pos = is_u ? si.pos_u : si.pos_v;
      const unsigned want = (unsigned)done * (unsigned)deg + (unsigned)(deg - 1 - pos);
      unsigned seen = 0;
      unsigned* dst = reinterpret_cast<unsigned*>(is_u ? sm.ubu[parity] : sm.ubv[parity]);
      if (!mb64_gather<LT>(mb + (size_t)node * 2 * L, L, want, dst, spin_limit, err, &seen)) {
        if ((tid & 63) == 0) {
          if (ld_dev(err) == 0 || seen != want) report_timeout(err, slot, node, want, seen);
          sm.abort_flag = q + 1;
        }
      }
      __syncthreads();
      if (sm.abort_flag == q + 1) return;
      si = si_next;
      parity ^= 1;
      if (--j < 0) { j = owned - 1; ++done; }
    }
    return;
  }
  // ---- the compute wave: lane = label ----
  const int s = tid;
  const bool real = s < L;
  const int sc = real ? s : 0;
  double p0 = 0.0, p1 = 0.0;
  int t1 = 0, s2 = 0, t3 = 0;
  auto load_step = [&](int slot, int it) __attribute__((always_inline)) {
    const unsigned char* rc = rec + (size_t)it * rec_it + (size_t)slot * 3 * L;
    t1 = rc[sc];
    s2 = rc[L + sc];
    t3 = rc[2 * L + sc];
    p0 = pb[(size_t)slot * 2 * L + sc];
    p1 = pb[(size_t)slot * 2 * L + L + sc];
  };
  int parity = 0, done = 0, j = owned - 1;
  if (owned > 1) load_step(first + j * G, seg - 1);
  SlotInfo si = ld_const(slots + first + j * G);
  for (int q = 0; q < total; ++q) {
    const int slot = first + j * G;
    const int it = seg - 1 - done;
    const int nxt_slot = uni(j == 0 ? first + (owned - 1) * G : slot - G);
    const SlotInfo si_next = ld_const(slots + nxt_slot);
    __syncthreads();  // the step's node adjoints are in LDS
    if (sm.abort_flag == q + 1) return;
    if (owned == 1) load_step(slot, it);
    const double ubu = sm.ubu[parity][sc], ubv = sm.ubv[parity][sc];
    // Each sum over the labels k with idx(k) = this lane's label takes the
    // terms in ascending k, as wave-uniform values read from lane k (labels
    // k >= L carry index -1 and never match).
    const int t3k = real ? t3 : -1, s2k = real ? s2 : -1, t1k = real ? t1 : -1;
    // r = th(s, t3) - q(t3): rb = pb0 + Ub_u
    const double rb = real ? p0 + ubu : 0.0;
    double qb = p1 + ubv;
#pragma unroll
    for (int k = 0; k < LT; ++k) {
      const double y = qb - lane_double(rb, k);
      qb = __builtin_amdgcn_readlane(t3k, k) == s ? y : qb;
    }
    // q = th(s2, t) + b(s2)
    const double qbk = real ? qb : 0.0;
    double bb = 0.0;
#pragma unroll
    for (int k = 0; k < LT; ++k) {
      const double y = bb + lane_double(qbk, k);
      bb = __builtin_amdgcn_readlane(s2k, k) == s ? y : bb;
    }
    // b = (a_u - p) / 2
    const double abu = ubu + 0.5 * bb;
    const double pbv = -0.5 * bb;
    // p = th(s, t1) + a_v(t1)
    const double pbk = real ? pbv : 0.0;
    double abv = ubv;
#pragma unroll
    for (int k = 0; k < LT; ++k) {
      const double y = abv + lane_double(pbk, k);
      abv = __builtin_amdgcn_readlane(t1k, k) == s ? y : abv;
    }
    // a_u = U_u - phi0, a_v = U_v - phi1
    if (real) {
      mb64_put(mb + (size_t)si.u * 2 * L, s, abu, (unsigned)done * (unsigned)si.deg_u + (unsigned)(si.deg_u - si.pos_u));
      mb64_put(mb + (size_t)si.v * 2 * L, s, abv, (unsigned)done * (unsigned)si.deg_v + (unsigned)(si.deg_v - si.pos_v));
      pb[(size_t)slot * 2 * L + s] = -abu;
      pb[(size_t)slot * 2 * L + L + s] = -abv;
      double* ct = contrib + ((size_t)it * m + slot) * 3 * L;
      ct[s] = rb;
      ct[L + s] = qb;
      ct[2 * L + s] = pbv;
    }
    si = si_next;
    parity ^= 1;
    if (--j < 0) { j = owned - 1; ++done; }
    if (q + 1 < total && owned > 1) load_step(nxt_slot, seg - 1 - done);
  }
}

// One launch of the persistent FP64 adjoint: workgroups [0, r.grid) run the
// reverse of one recorded segment, the others the forward of `f.iters`
// iterations (recording or not).  In the backward the two roles work on
// different segments (the reverse of segment c beside the recomputation of
// segment c - 1, which needs only its checkpoint): they share no data, so
// they run side by side on the device.  Each workgroup has kF64NT + 128
// threads; the reverse uses wave 0 and the two sync waves.
template <int LT, bool REC>
__global__ void __launch_bounds__(kF64NT + 128) k_adj64(Fwd64Args f, Rev64Args r) {
  __shared__ SmemF64<LT> smf;
  __shared__ SmemR64<LT> smr;
  const int b = blockIdx.x;
  if (b < r.grid) {
    if (b >= r.m || r.seg <= 0) return;
    if (threadIdx.x == 0) smr.abort_flag = 0;
    __syncthreads();
    rev64_role<LT>(r, b, r.grid, smr);
  } else {
    const int first = b - r.grid;
    if (first >= f.m || f.iters <= 0) return;
    if (threadIdx.x == 0) smf.abort_flag = 0;
    __syncthreads();
    fwd64_role<LT, REC>(f, first, f.grid, smf);
  }
}

// Table adjoints of one segment: thb[slot] += the reverse steps' scatters,
// iterations descending, within each r (thb(s, t3(s)) += rb(s)), then q
// (thb(s2(t), t) += q-bar(t)), then p (thb(s, t1(s)) += p-bar(s)): the
// order of the per-matching reverse.  One workgroup per slot, the slot's
// table adjoint in LDS.
template <int LT>
__global__ void __launch_bounds__(256) k_thb_acc(double* __restrict__ thb, const unsigned char* __restrict__ rec,
                                                 const double* __restrict__ contrib, int L, int m, int seg) {
  __shared__ double g[LT * LT];
  const int slot = blockIdx.x;
  const int tid = threadIdx.x;
  double* gt = thb + (size_t)slot * L * L;
  for (int k = tid; k < L * L; k += 256) g[k] = gt[k];
  __syncthreads();
  const size_t rec_it = (size_t)m * 3 * L;
  for (int it = seg - 1; it >= 0; --it) {
    const unsigned char* rc = rec + (size_t)it * rec_it + (size_t)slot * 3 * L;
    const double* ct = contrib + ((size_t)it * m + slot) * 3 * L;
    if (tid < L) g[tid * L + rc[2 * L + tid]] += ct[tid];
    __syncthreads();
    if (tid < L) g[rc[L + tid] * L + tid] += ct[L + tid];
    __syncthreads();
    if (tid < L) g[tid * L + rc[tid]] += ct[2 * L + tid];
    __syncthreads();
  }
  for (int k = tid; k < L * L; k += 256) gt[k] = g[k];
}

hipError_t launch_mb64_init(const double* x, unsigned long long* mb, size_t count, hipStream_t st) {
  const size_t blocks = std::min<size_t>(1024, (count + 255) / 256);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mb64_init, dim3((unsigned)blocks), dim3(256), 0, st, x, mb, count);
  return hipGetLastError();
}
hipError_t launch_mb64_fini(double* x, const unsigned long long* mb, size_t count, hipStream_t st) {
  const size_t blocks = std::min<size_t>(1024, (count + 255) / 256);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mb64_fini, dim3((unsigned)blocks), dim3(256), 0, st, x, mb, count);
  return hipGetLastError();
}

template <int LT>
static hipError_t adj64_one(const Fwd64Args& f, const Rev64Args& r, double* thb, hipStream_t st) {
  void* args[] = {(void*)&f, (void*)&r};
  const void* fn = f.rec ? (const void*)k_adj64<LT, true> : (const void*)k_adj64<LT, false>;
  const int grid = r.grid + f.grid;
  if (grid <= 0) return hipSuccess;
  hipError_t e = hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kF64NT + 128), args, 0, st);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e;
  }
  if (r.grid > 0 && r.seg > 0 && r.m > 0) {
    hipLaunchKernelGGL(k_thb_acc<LT>, dim3(r.m), dim3(256), 0, st, thb, r.rec, r.contrib, r.L, r.m, r.seg);
    return hipGetLastError();
  }
  return hipSuccess;
}

// One launch: the reverse of `seg` recorded iterations (rev_grid
// workgroups; 0: none) next to the forward of `iters` iterations (fwd_grid
// workgroups; iters 0: none; fwd_rec: record the argmins there), then the
// reverse segment's table adjoints.
hipError_t launch_adj64(const double* tables, double* phi, unsigned long long* mb_fwd, int iters, unsigned char* fwd_rec,
                        int fwd_grid, const unsigned char* rev_rec, unsigned long long* mb_rev, double* pb,
                        double* contrib, double* thb, int seg, int rev_grid, const SlotInfo* slots, int L, int m,
                        int* err, long long spin_limit, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  Fwd64Args f{tables, phi, mb_fwd, slots, L, m, iters, fwd_rec, err, spin_limit, iters > 0 ? fwd_grid : 0};
  Rev64Args r{slots, L, m, seg, rev_rec, mb_rev, pb, contrib, err, spin_limit, seg > 0 ? rev_grid : 0};
  if (L <= 16) return adj64_one<16>(f, r, thb, st);
  if (L <= 32) return adj64_one<32>(f, r, thb, st);
  if (L <= 64) return adj64_one<64>(f, r, thb, st);
  return hipErrorInvalidValue;
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
