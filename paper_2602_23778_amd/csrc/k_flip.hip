// One-time column sign flip X <- X Sigma of Sec. 3.1.1, for an X whose leading
// block X1 - I is singular (or too ill-conditioned) for the compact WY form of
// Algorithm 1.  Sigma = diag(sigma) comes from the modified LU factorisation of
// Algorithm 2: at column j the sign sigma_j = -sign(q_jj) of the current
// diagonal entry is taken off it before the elimination (sign(0) = +1), so
// every pivot has magnitude |q_jj| + 1 >= 1.
//
// The pivot of column j after j eliminations depends on rows 1..j only, so
// the k x k leading block determines Sigma: one workgroup eliminates that
// block in LDS (FP64, the division and the rank-one update each rounded once,
// as written), then a grid-wide pass scales the columns of X.  A non-finite
// entry or pivot stops the problem with the non-finite status and leaves X
// unchanged.
#include "common.h"

namespace rfk {

constexpr int FL_NT = 256;
constexpr int FL_LD = KMAX + 1;

__global__ __launch_bounds__(FL_NT) void flip_sigma_kernel(const Prob* __restrict__ probs, int nprob) {
  __shared__ double Q[KMAX * FL_LD];
  __shared__ int bad;
  const int tid = threadIdx.x;
  for (int p = blockIdx.x; p < nprob; p += gridDim.x) {
    const Prob& P = probs[p];
    Ctrl* ctrl = P.ctrl;
    __syncthreads();
    if (ctrl->stopped) continue;
    const int k = P.k;
    const double* X = P.x;
    const int64_t ldx = P.ldx;
    double* sigma = P.vec + VEC_SCALE * k;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int e = tid; e < k * k; e += FL_NT) {
      const int i = e / k, j = e - i * k;
      const double v = X[(int64_t)i * ldx + j];
      if (!__builtin_isfinite(v)) bad = 1;
      Q[i * FL_LD + j] = v;
    }
    __syncthreads();
    for (int j = 0; j < k && !bad; ++j) {
      if (tid == 0) {
        const double q = Q[j * FL_LD + j];
        const double s = q >= 0.0 ? -1.0 : 1.0;
        const double piv = q - s;
        if (!__builtin_isfinite(piv)) bad = 1;
        Q[j * FL_LD + j] = piv;
        sigma[j] = s;
      }
      __syncthreads();
      const double piv = Q[j * FL_LD + j];
      for (int l = j + 1 + tid; l < k; l += FL_NT) Q[l * FL_LD + j] = Q[l * FL_LD + j] / piv;
      __syncthreads();
      const int m = k - j - 1;
      for (int e = tid; e < m * m; e += FL_NT) {
        const int l = j + 1 + e / m, h = j + 1 + e % m;
        Q[l * FL_LD + h] = __dsub_rn(Q[l * FL_LD + h], __dmul_rn(Q[l * FL_LD + j], Q[j * FL_LD + h]));
      }
      __syncthreads();
    }
    if (tid == 0 && bad) {
      ctrl->status = -6;
      ctrl->stopped = 1;
    }
  }
}

// X <- X Sigma over (problem, row block) items.
__global__ __launch_bounds__(256) void flip_apply_kernel(const Prob* __restrict__ probs,
                                                        const RowItem* __restrict__ items, int nitems) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem item = items[it];
    const Prob& P = probs[item.prob];
    if (P.ctrl->stopped) continue;
    const int n = P.n, k = P.k;
    const double* sigma = P.vec + VEC_SCALE * k;
    double* X = P.x;
    const int64_t ldx = P.ldx;
    const int r0 = item.blk * P.rbrows, r1 = min(n, r0 + P.rbrows);
    const int64_t cnt = (int64_t)(r1 - r0) * k;
    for (int64_t e = threadIdx.x; e < cnt; e += 256) {
      const int r = r0 + (int)(e / k), c = (int)(e % k);
      if (sigma[c] < 0.0) X[(int64_t)r * ldx + c] = -X[(int64_t)r * ldx + c];
    }
  }
}

hipError_t launch_flip_sigma(const Prob* probs, int nprob, hipStream_t st) {
  hipLaunchKernelGGL(flip_sigma_kernel, dim3(nprob), dim3(FL_NT), 0, st, probs, nprob);
  return hipGetLastError();
}

hipError_t launch_flip_apply(const Prob* probs, const RowItem* items, int nitems, hipStream_t st) {
  hipLaunchKernelGGL(flip_apply_kernel, dim3(nitems), dim3(256), 0, st, probs, items, nitems);
  return hipGetLastError();
}

}  // namespace rfk
