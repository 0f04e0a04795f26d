// Block-level helpers shared by the kernels of the step (header-only, since
// the kernels are built without relocatable device code).
#pragma once
#include "common.h"

namespace rfk {

__device__ __forceinline__ int pow2ceil(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Block-wide deterministic sum of per-block partials:
//   out[s] = sum_{b < nb} src[b * stride + s]   for s < S,
// with a fixed team of threads per slot and a fixed LDS tree.  `scratch`
// holds blockDim.x doubles; out may alias nothing that src uses.
__device__ inline void team_reduce(const double* __restrict__ src, int stride, int S, int nb,
                            double* scratch, double* out) {
  const int NT = blockDim.x, tid = threadIdx.x;
  int ts = 1;
  while (ts * 2 * S <= NT) ts *= 2;
  for (int s0 = 0; s0 < S; s0 += NT / ts) {
    const int s = s0 + tid / ts, m = tid % ts;
    double acc = 0.0;
    if (tid / ts < NT / ts && s < S)
      for (int b = m; b < nb; b += ts) acc += src[(int64_t)b * stride + s];
    scratch[tid] = acc;
    __syncthreads();
    for (int h = ts / 2; h >= 1; h /= 2) {
      if (m < h) scratch[tid] += scratch[tid + h];
      __syncthreads();
    }
    if (m == 0 && s < S && tid / ts < NT / ts) out[s] = scratch[tid];
    __syncthreads();
  }
}

// Arrival counter of the last-block pattern: returns true in exactly one block
// (the last to arrive) once all nb blocks of the problem have published their
// partials; that block resets the counter for the next launch.
__device__ inline bool last_block_arrival(int32_t* counter, int nb, int* flag) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const int t = atomicAdd(counter, 1);
    *flag = (t == nb - 1);
  }
  __syncthreads();
  const bool last = *flag;
  if (last) __threadfence();
  return last;
}

}  // namespace rfk
