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
//   out[s] = sum_{b < nb} src[b * stride + s]   for s < S <= 2 blockDim.x,
// with ts (a power of two) teams of SP threads: thread m*SP + q sums the
// blocks b = m, m + ts, ... of its slots, sixteen loads in flight per round
// trip (consecutive threads read consecutive slots of one block row), then a
// fixed LDS tree across the teams.  When S and stride are even and src is
// 16-byte aligned a thread takes the slot pair (2q, 2q + 1) with 16-byte
// loads (SP = S / 2: twice the teams, half the round trips per thread);
// otherwise the slot q (SP = S).  `scratch` holds blockDim.x doubles.  All
// threads of the block must call it.
__device__ inline void team_reduce(const double* __restrict__ src, int stride, int S, int nb,
                                   double* scratch, double* out) {
  typedef double v2d __attribute__((ext_vector_type(2)));
  const int NT = blockDim.x, tid = threadIdx.x;
  const bool pairs = (S & 1) == 0 && (stride & 1) == 0 && (((uintptr_t)src) & 15) == 0;
  const int SP = pairs ? S / 2 : S;
  int ts = 1;
  while (ts * 2 * SP <= NT) ts *= 2;
  const int q = tid % SP, m = tid / SP;
  double a0 = 0.0, a1 = 0.0;
  if (m < ts) {
    if (pairs) {
      for (int b0 = m; b0 < nb; b0 += 16 * ts) {
        v2d v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int b = b0 + u * ts;
          v[u] = b < nb ? *gld(reinterpret_cast<const v2d*>(src + (int64_t)b * stride + 2 * q))
                        : v2d{0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          a0 += v[u].x;
          a1 += v[u].y;
        }
      }
    } else {
      for (int b0 = m; b0 < nb; b0 += 16 * ts) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int b = b0 + u * ts;
          v[u] = b < nb ? *gld(src + (int64_t)b * stride + q) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) a0 += v[u];
      }
    }
  }
  // the teams' sums of the first (then the second) slot of each pair
  for (int pass = 0; pass < (pairs ? 2 : 1); ++pass) {
    scratch[tid] = pass == 0 ? a0 : a1;
    __syncthreads();
    for (int h = ts / 2; h >= 1; h /= 2) {
      if (m < h) scratch[tid] += scratch[tid + h * SP];
      __syncthreads();
    }
    if (m == 0) out[pairs ? 2 * q + pass : q] = scratch[tid];
    __syncthreads();
  }
}

// Per-column block sums for the Rayleigh quotients (eq. Rayleigh).  Threads
// are laid out as [NT/KP rows][KP columns], KP = pow2ceil(k): thread
// (trow, col) holds sums of x*w and x*x over its rows of column col.  The
// block's column sums are written as partial `blk` of Prob::dpart; a
// separate kernel forms d.
// red holds 2*NT doubles.  Block-uniform call.
template <int NT>
__device__ void rayleigh_block_partial(const Prob& P, int blk, double sxw, double sxx,
                                       double* red) {
  const int tid = threadIdx.x;
  const int k = P.k, kp = pow2ceil(k), tr = NT / kp;
  const int col = tid % kp, trow = tid / kp;
  red[tid] = sxw;
  red[NT + tid] = sxx;
  __syncthreads();
  for (int h = tr / 2; h >= 1; h /= 2) {
    if (trow < h) {
      red[tid] += red[tid + h * kp];
      red[NT + tid] += red[NT + tid + h * kp];
    }
    __syncthreads();
  }
  if (trow == 0 && col < k) {
    P.dpart[(int64_t)blk * 2 * k + col] = red[tid];
    P.dpart[(int64_t)blk * 2 * k + k + col] = red[NT + tid];
  }
  __syncthreads();
}

}  // namespace rfk
