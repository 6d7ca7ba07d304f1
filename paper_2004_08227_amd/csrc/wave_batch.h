// Host interface of the batched launch on the wave engine (batch.hip).
#pragma once
#include "common.h"

namespace mplpxx {

// LDS of one model in LDS mode: the unaries as for the workgroup engine (hi
// FP32, then bf16 lo from lds_lo_offset), then one update counter per node
// from this byte offset
__host__ __device__ inline size_t wv_ver_offset(int n, int L) { return (lds_model_bytes(n, L) + 15) / 16 * 16; }
__host__ __device__ inline size_t wv_lds_bytes(int n, int L) { return wv_ver_offset(n, L) + (size_t)n * 4; }

// kind: the kernel instance for the batch's cost kind (0 dense, MPLPXX_COST_*)
hipError_t launch_wbatch(const BatchArgs& b, int grid, int iters, size_t dyn_lds, int kind, hipStream_t st);
int wbatch_blocks_per_cu(size_t dyn_lds, int kind);
// static LDS of the kernel (out), and the largest dynamic LDS it can have
size_t wbatch_lds_limit(size_t* static_bytes, int kind);
int wbatch_waves();           // waves (workers) per workgroup
size_t wbatch_sink_words();   // scratch words per workgroup

}  // namespace mplpxx
