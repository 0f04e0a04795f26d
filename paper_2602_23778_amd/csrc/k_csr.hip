// Line 1 of Algorithm 4 for sparse A in CSR form, fused with the first
// reduction of the step (eq. Rayleigh): W = A X, and per row block the
// column sums of x_j * w_j and x_j * x_j.
//
// Layout: a block of NT threads works on [NT/KP rows] x [KP columns] with KP
// the power of two >= k, so a row's nonzeros (col_idx, val) are broadcast to
// the KP lanes of that row and every X row gather is one contiguous
// 8k-byte read.  The work is bound by HBM bandwidth (12 B per nonzero plus
// the X gathers and the W write); rows of a block are contiguous so that the
// stencil's neighbouring rows of X are reused from cache.
#include "common.h"
#include "dev_util.h"

namespace rfk {

template <int NT>
__global__ __launch_bounds__(NT) void spmm_kernel(const Prob* __restrict__ probs,
                                                 const RowItem* __restrict__ items, int nitems) {
  __shared__ double red[2 * NT];
  const int tid = threadIdx.x;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem item = items[it];
    const Prob& P = probs[item.prob];
    if (P.ctrl->stopped) continue;
    const int n = P.n, k = P.k, kp = pow2ceil(k), tr = NT / kp;
    const int col = tid % kp, trow = tid / kp;
    const int r0 = item.blk * P.rbrows, r1 = min(n, r0 + P.rbrows);
    const int32_t* __restrict__ rp = P.rp;
    const int32_t* __restrict__ ci = P.ci;
    const double* __restrict__ av = P.av;
    const double* __restrict__ X = P.x;
    const int64_t ldx = P.ldx;
    double sxw = 0.0, sxx = 0.0;
    if (col < k) {
      for (int row = r0 + trow; row < r1; row += tr) {
        const int e0 = rp[row], e1 = rp[row + 1];
        double w = 0.0;
        for (int e = e0; e < e1; ++e) w = __builtin_fma(av[e], X[(int64_t)ci[e] * ldx + col], w);
        P.w[(int64_t)row * k + col] = w;
        const double x = X[(int64_t)row * ldx + col];
        sxw = __builtin_fma(x, w, sxw);
        sxx = __builtin_fma(x, x, sxx);
      }
    }
    rayleigh_block_partial<NT>(P, item.blk, sxw, sxx, red);
  }
}

hipError_t launch_spmm(const Prob* probs, const RowItem* items, int nitems, hipStream_t st) {
  hipLaunchKernelGGL((spmm_kernel<1024>), dim3(nitems), dim3(1024), 0, st, probs, items, nitems);
  return hipGetLastError();
}

// Row statistics for ||A||_inf and the Gershgorin bounds (Sec. 5.1 shifts):
// per block the maximum of sum_j |a_ij|, of a_ii + sum_{j!=i} |a_ij| and the
// minimum of a_ii - sum_{j!=i} |a_ij|.  One wavefront per row.
__global__ __launch_bounds__(256) void rowstats_kernel(int kind, int n, const double* __restrict__ a,
                                                       int64_t lda, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci,
                                                       const double* __restrict__ av,
                                                       double* __restrict__ out) {
  __shared__ double s_max[4], s_hi[4], s_lo[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double bmax = 0.0, bhi = -INFINITY, blo = INFINITY;
  for (int row = blockIdx.x * 4 + wave; row < n; row += gridDim.x * 4) {
    double s = 0.0, dg = 0.0;
    if (kind == 0) {
      const double* ar = a + (int64_t)row * lda;
      for (int j = lane; j < n; j += 64) {
        const double v = ar[j];
        s += fabs(v);
        if (j == row) dg = v;
      }
    } else {
      for (int e = rp[row] + lane; e < rp[row + 1]; e += 64) {
        const double v = av[e];
        s += fabs(v);
        if (ci[e] == row) dg = v;
      }
    }
    for (int o = 32; o >= 1; o /= 2) {
      s += __shfl_xor(s, o);
      dg += __shfl_xor(dg, o);
    }
    const double off = s - fabs(dg);
    bmax = fmax(bmax, s);
    bhi = fmax(bhi, dg + off);
    blo = fmin(blo, dg - off);
  }
  if (lane == 0) {
    s_max[wave] = bmax;
    s_hi[wave] = bhi;
    s_lo[wave] = blo;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0, h = -INFINITY, l = INFINITY;
    for (int w = 0; w < 4; ++w) {
      m = fmax(m, s_max[w]);
      h = fmax(h, s_hi[w]);
      l = fmin(l, s_lo[w]);
    }
    out[3 * blockIdx.x] = m;
    out[3 * blockIdx.x + 1] = h;
    out[3 * blockIdx.x + 2] = l;
  }
}

hipError_t launch_rowstats(int kind, int n, const double* a, int64_t lda, const int32_t* rp,
                           const int32_t* ci, const double* av, double* out, int grid,
                           hipStream_t st) {
  hipLaunchKernelGGL(rowstats_kernel, dim3(grid), dim3(256), 0, st, kind, n, a, lda, rp, ci, av,
                     out);
  return hipGetLastError();
}

}  // namespace rfk
