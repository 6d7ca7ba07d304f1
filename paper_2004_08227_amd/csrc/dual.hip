// Dual bound (Eq. (3)), per-iteration dual traces, primal rounding (Eq. (5))
// and energy (Eq. (1)) of MPLP++ on gfx950, plus small utility kernels.
//
// The certified dual bound is recomputed from the input costs and the
// messages, never from the incrementally updated unaries:
//   node term  min_s [theta_u(s) + sum_{e incident to u} phi_{e->u}(s)]
//   edge term  min_{s,t} [theta_e(s,t) - phi_e[0](s) - phi_e[1](t)]
// with every sum in FP64 (Eq. (2) and Eq. (3)).  All reductions use a fixed
// order, so the result is deterministic.
#include <algorithm>

#include "common.h"

namespace mplpxx {

__device__ __forceinline__ double dmin(double a, double b) { return __builtin_fmin(a, b); }

// fixed-order block reduction of one double per thread (blockDim power of 2)
template <int NT, bool kMin>
__device__ __forceinline__ double block_reduce(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s >= 1; s >>= 1) {
    if (tid < s) sh[tid] = kMin ? dmin(sh[tid], sh[tid + s]) : sh[tid] + sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// node terms: one workgroup per node, one thread per label
template <typename T>
__global__ void __launch_bounds__(128) k_node_terms(const T* __restrict__ unaries, const T* __restrict__ phi,
                                                    const int* __restrict__ node_ptr, const int* __restrict__ inc,
                                                    int L, double* __restrict__ node_min) {
  __shared__ double sh[128];
  const int u = blockIdx.x;
  const int s = threadIdx.x;
  double acc = __builtin_inf();
  if (s < L) {
    acc = (double)unaries[(size_t)u * L + s];
    for (int k = node_ptr[u]; k < node_ptr[u + 1]; ++k) {
      const int code = inc[k];
      acc += (double)phi[(size_t)(code >> 1) * 2 * L + (size_t)(code & 1) * L + s];
    }
  }
  const double mn = block_reduce<128, true>(acc, sh);
  if (s == 0) node_min[u] = mn;
}

// th(s, t) of the edge in `slot`: its table, or, for structured costs (their
// parameters per slot), the expanded table entry
template <typename T>
__device__ __forceinline__ T table_at(const T* tables, int slot, int L, int s, int t, int potts) {
  if constexpr (sizeof(T) == 4) {
    if (potts) return structured_cost(potts, tables + (size_t)slot * cost_params(potts), s, t);
  }
  return tables[(size_t)slot * L * L + (size_t)s * L + t];
}

// edge terms: one workgroup per slot
template <typename T>
__global__ void __launch_bounds__(256) k_edge_terms(const T* __restrict__ tables, const T* __restrict__ phi, int L,
                                                    int potts, double* __restrict__ edge_min) {
  __shared__ double sh[256];
  const int slot = blockIdx.x;
  const T* p0 = phi + (size_t)slot * 2 * L;
  const T* p1 = p0 + L;
  double mn = __builtin_inf();
  for (int i = threadIdx.x; i < L * L; i += 256) {
    const int s = i / L, t = i - s * L;
    mn = dmin(mn, (double)table_at(tables, slot, L, s, t, potts) - (double)p0[s] - (double)p1[t]);
  }
  mn = block_reduce<256, true>(mn, sh);
  if (threadIdx.x == 0) edge_min[slot] = mn;
}

// out = sum(a[0..na)) + sum(b[0..nb)), fixed order, one workgroup
__global__ void __launch_bounds__(1024) k_sum2(const double* __restrict__ a, int na, const double* __restrict__ b,
                                               int nb, double* __restrict__ out) {
  __shared__ double sh[1024];
  double acc = 0.0;
  for (int i = threadIdx.x; i < na; i += 1024) acc += a[i];
  for (int i = threadIdx.x; i < nb; i += 1024) acc += b[i];
  acc = block_reduce<1024, false>(acc, sh);
  if (threadIdx.x == 0) *out = acc;
}

template <typename T>
hipError_t launch_dual(const T* unaries, const T* tables, const T* phi, const int* node_ptr, const int* inc, int n,
                       int L, int m, double* node_min, double* edge_min, double* out, hipStream_t st, int potts) {
  hipLaunchKernelGGL(k_node_terms<T>, dim3(n), dim3(128), 0, st, unaries, phi, node_ptr, inc, L, node_min);
  if (m > 0) hipLaunchKernelGGL(k_edge_terms<T>, dim3(m), dim3(256), 0, st, tables, phi, L, potts, edge_min);
  hipLaunchKernelGGL(k_sum2, dim3(1), dim3(1024), 0, st, node_min, n, edge_min, m, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Traces: sum_u min_s U_u(s) in FP64 per iteration.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(64) k_trace_nodes(const T* __restrict__ U, const T* __restrict__ Ulo, int L,
                                                    double* __restrict__ row) {
  const int u = blockIdx.x;
  double mn = __builtin_inf();
  for (int s = threadIdx.x; s < L; s += 64) {
    const size_t i = (size_t)u * L + s;
    mn = dmin(mn, (double)U[i] + (Ulo ? (double)Ulo[i] : 0.0));
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mn = dmin(mn, __shfl_xor(mn, o, 64));
  if (threadIdx.x == 0) row[u] = mn;
}

template <typename T>
hipError_t launch_trace_nodes(const T* U, const T* Ulo, int n, int L, double* row, hipStream_t st) {
  hipLaunchKernelGGL(k_trace_nodes<T>, dim3(n), dim3(64), 0, st, U, Ulo, L, row);
  return hipGetLastError();
}

// Edge terms of Eq. (3) for the trace of one iteration: out[slot] =
// min_{s,t} [theta(s,t) - phi[0](s) - phi[1](t)] in FP64, stored as FP32 (the
// FP32 engines' terms are rounding-level numbers, far inside FP32 range).
template <typename T>
__global__ void __launch_bounds__(256) k_trace_edges(const T* __restrict__ tables, const T* __restrict__ phi, int L,
                                                     float* __restrict__ out) {
  __shared__ double sh[256];
  const int slot = blockIdx.x;
  const T* tab = tables + (size_t)slot * L * L;
  const T* p0 = phi + (size_t)slot * 2 * L;
  const T* p1 = p0 + L;
  double mn = __builtin_inf();
  for (int i = threadIdx.x; i < L * L; i += 256) {
    const int s = i / L, t = i - s * L;
    mn = dmin(mn, ((double)tab[i] - (double)p0[s]) - (double)p1[t]);
  }
  mn = block_reduce<256, true>(mn, sh);
  if (threadIdx.x == 0) out[slot] = (float)mn;
}

template <typename T>
hipError_t launch_trace_edges(const T* tables, const T* phi, int m, int L, float* out, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trace_edges<T>, dim3(m), dim3(256), 0, st, tables, phi, L, out);
  return hipGetLastError();
}

// One workgroup per iteration: sum of the node minima (nodes without edges
// keep their input unary) plus, when trace_e is given, the edge terms (the
// minimum over the W partial minima of each slot), in a fixed order.
template <typename T>
__global__ void __launch_bounds__(256) k_trace_sum(const double* __restrict__ trace_nodes,
                                                   const float* __restrict__ trace_e, int m, int W,
                                                   const T* __restrict__ U, const int* __restrict__ deg, int n, int L,
                                                   double* __restrict__ out) {
  __shared__ double sh[256];
  const int it = blockIdx.x;
  double acc = 0.0;
  for (int u = threadIdx.x; u < n; u += 256) {
    double v;
    if (deg[u] > 0) {
      v = trace_nodes[(size_t)it * n + u];
    } else {
      v = __builtin_inf();
      for (int s = 0; s < L; ++s) v = dmin(v, (double)U[(size_t)u * L + s]);
    }
    acc += v;
  }
  if (trace_e) {
    for (int e = threadIdx.x; e < m; e += 256) {
      const float* w = trace_e + ((size_t)it * m + e) * W;
      float v = w[0];
      for (int k = 1; k < W; ++k) v = __builtin_fminf(v, w[k]);
      acc += (double)v;
    }
  }
  acc = block_reduce<256, false>(acc, sh);
  if (threadIdx.x == 0) out[it] = acc;
}

template <typename T>
hipError_t launch_trace_sum(double* trace_nodes, const float* trace_e, int m, int W, const T* U, const int* deg, int n,
                            int L, int iters, double* out, hipStream_t st) {
  if (iters <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trace_sum<T>, dim3(iters), dim3(256), 0, st, trace_nodes, trace_e, m, W, U, deg, n, L, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Primal rounding, Eq. (5), and energy, Eq. (1).  One workgroup of 1024
// threads walks the nodes in ascending order; for node u, wave w sums the
// incidences w, w+16, ... of u (lane = label), and the 16 partial sums are
// added in wave order after the reparametrized unary.  All sums in FP64.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(1024) k_decode(const T* __restrict__ unaries, const T* __restrict__ tables,
                                                 const T* __restrict__ phi, const SlotInfo* __restrict__ slots,
                                                 const int* __restrict__ node_ptr, const int* __restrict__ inc, int n,
                                                 int L, int m, int potts, int* __restrict__ labels,
                                                 double* __restrict__ energy) {
  constexpr int NW = 16;
  __shared__ double part[NW][MPLPXX_MAX_LABELS];
  __shared__ double sh[1024];
  __shared__ int best_label;
  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;
  for (int u = 0; u < n; ++u) {
    for (int x = lane; x < L; x += 64) {
      double acc = 0.0;
      for (int k = node_ptr[u] + w; k < node_ptr[u + 1]; k += NW) {
        const int code = inc[k];
        const int slot = code >> 1, side = code & 1;
        const T* p = phi + (size_t)slot * 2 * L;
        // message into u: part of the reparametrized unary of u (Eq. 2)
        acc += (double)p[(size_t)side * L + x];
        if (side == 1) {
          // u is the upper node: add theta^phi_{vu}(x*_v, x) for v < u
          const int yv = labels[slots[slot].u];
          acc += (double)table_at(tables, slot, L, yv, x, potts) - (double)p[yv] - (double)p[L + x];
        }
      }
      part[w][x] = acc;
    }
    __syncthreads();
    if (w == 0) {
      // cost and argmin over labels; ties go to the smallest label
      double best = __builtin_inf();
      int arg = 0x7fffffff;
      for (int x = lane; x < L; x += 64) {
        double c = (double)unaries[(size_t)u * L + x];
        for (int ww = 0; ww < NW; ++ww) c += part[ww][x];
        if (c < best) { best = c; arg = x; }
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oa = __shfl_xor(arg, o, 64);
        if (ob < best || (ob == best && oa < arg)) { best = ob; arg = oa; }
      }
      if (lane == 0) {
        best_label = arg;
        labels[u] = arg;
      }
    }
    __syncthreads();
  }
  // energy of Eq. (1) on the input costs
  double acc = 0.0;
  for (int u = tid; u < n; u += 1024) acc += (double)unaries[(size_t)u * L + labels[u]];
  for (int slot = tid; slot < m; slot += 1024) {
    const SlotInfo si = slots[slot];
    acc += (double)table_at(tables, slot, L, labels[si.u], labels[si.v], potts);
  }
  acc = block_reduce<1024, false>(acc, sh);
  if (tid == 0) *energy = acc;
  (void)best_label;
}

template <typename T>
hipError_t launch_decode(const T* unaries, const T* tables, const T* phi, const SlotInfo* slots, const int* node_ptr,
                         const int* inc, int n, int L, int m, int* labels, double* energy, hipStream_t st,
                         int potts) {
  hipLaunchKernelGGL(k_decode<T>, dim3(1), dim3(1024), 0, st, unaries, tables, phi, slots, node_ptr, inc, n, L, m,
                     potts, labels, energy);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Utilities: finiteness check of device inputs, table packing from a device
// copy in the caller's layout, integer fill (used instead of memset so that
// the same code can sit inside captured graphs).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_check_finite(const T* __restrict__ p, size_t count, int* __restrict__ flag) {
  bool bad = false;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    bad |= sizeof(T) == 4 ? !(__builtin_fabs((double)p[i]) <= MPLPXX_F32_MAX_COST) : !__builtin_isfinite(p[i]);
  if (bad) atomicOr(flag, 1);
}

template <typename T>
hipError_t launch_check_finite(const T* p, size_t count, int* flag, hipStream_t st) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_check_finite<T>, dim3((unsigned)blocks), dim3(256), 0, st, p, count, flag);
  return hipGetLastError();
}

// dst slot i <- src edge slot_edge[i], transposed when slot_flip[i]
template <typename T>
__global__ void k_pack_tables(const T* __restrict__ src, T* __restrict__ dst, const int* __restrict__ slot_edge,
                              const int* __restrict__ slot_flip, int L) {
  const int slot = blockIdx.x;
  const T* s = src + (size_t)slot_edge[slot] * L * L;
  T* d = dst + (size_t)slot * L * L;
  const bool flip = slot_flip[slot] != 0;
  for (int i = threadIdx.x; i < L * L; i += blockDim.x) {
    const int r = i / L, c = i - r * L;
    d[i] = flip ? s[(size_t)c * L + r] : s[i];
  }
}

template <typename T>
hipError_t launch_pack_tables(const T* src, T* dst, const int* slot_edge, const int* slot_flip, int m, int L,
                              hipStream_t st) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_tables<T>, dim3(m), dim3(256), 0, st, src, dst, slot_edge, slot_flip, L);
  return hipGetLastError();
}

__global__ void k_fill_int(int* __restrict__ p, int value, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    p[i] = value;
}

template <typename S, typename D>
__global__ void k_convert(const S* __restrict__ src, D* __restrict__ dst, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (D)src[i];
}

hipError_t launch_convert(const float* src, double* dst, size_t count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL((k_convert<float, double>), dim3((unsigned)blocks), dim3(256), 0, st, src, dst, count);
  return hipGetLastError();
}

hipError_t launch_convert(const double* src, float* dst, size_t count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL((k_convert<double, float>), dim3((unsigned)blocks), dim3(256), 0, st, src, dst, count);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int value, size_t count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_fill_int, dim3((unsigned)blocks), dim3(256), 0, st, p, value, count);
  return hipGetLastError();
}

#define MPLPXX_INST(T)                                                                                              \
  template hipError_t launch_dual<T>(const T*, const T*, const T*, const int*, const int*, int, int, int, double*,  \
                                     double*, double*, hipStream_t, int);                                         \
  template hipError_t launch_trace_nodes<T>(const T*, const T*, int, int, double*, hipStream_t);                             \
  template hipError_t launch_trace_edges<T>(const T*, const T*, int, int, float*, hipStream_t);               \
  template hipError_t launch_trace_sum<T>(double*, const float*, int, int, const T*, const int*, int, int, int,   \
                                          double*, hipStream_t);     \
  template hipError_t launch_decode<T>(const T*, const T*, const T*, const SlotInfo*, const int*, const int*, int, \
                                       int, int, int*, double*, hipStream_t, int);                                 \
  template hipError_t launch_check_finite<T>(const T*, size_t, int*, hipStream_t);                                 \
  template hipError_t launch_pack_tables<T>(const T*, T*, const int*, const int*, int, int, hipStream_t);
MPLPXX_INST(float)
MPLPXX_INST(double)
#undef MPLPXX_INST

}  // namespace mplpxx
