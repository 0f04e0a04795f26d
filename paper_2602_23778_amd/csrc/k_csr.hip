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

// Blocks of the SpMM (each takes every SPMM_GRID-th chunk of SPMM_ROWS rows).
constexpr int SPMM_GRID = 512;
constexpr int SPMM_ROWS = 256;

// Latency: a row costs two dependent round trips (its nonzeros, then the X
// rows they name), so each thread keeps RPT rows in flight at once: the row
// pointers of the next RPT rows are requested while the current ones are
// gathered, and up to eight nonzeros of a row are requested together.  The
// sum over a row's nonzeros runs in CSR order.
//
// Row order: the block takes the row chunks blockIdx.x, blockIdx.x + grid,
// ... (chunks of rbrows rows), so that at any moment the whole GPU works on
// one contiguous window of rows and the far stencil neighbours (N^2 rows
// away on a 3-D grid) are still in the caches.  The block's Rayleigh
// partial covers all of its chunks (partial index = blockIdx.x).
template <int NT, int RPT, int NZB>
__global__ __launch_bounds__(NT) void spmm_kernel(const Prob* __restrict__ probs,
                                                 const RowItem* __restrict__ items, int nitems,
                                                 int chunk_rows) {
  __shared__ double red[2 * NT];
  const int tid = threadIdx.x;
  const Prob& P = probs[0];
  if (P.ctrl->stopped) return;
  double sxw = 0.0, sxx = 0.0;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem item = items[it];
    const int n = P.n, k = P.k, kp = pow2ceil(k), tr = NT / kp;
    const int col = tid % kp, trow = tid / kp;
    const int r0 = item.blk * chunk_rows, r1 = min(n, r0 + chunk_rows);
    const int32_t* __restrict__ rp = P.rp;
    const int32_t* __restrict__ ci = P.ci;
    const double* __restrict__ av = P.av;
    const double* __restrict__ X = P.x;
    const int64_t ldx = P.ldx;
    if (col < k) {
      // rows row0 + u*tr, u < RPT, per round; row pointers one round ahead
      int e0[RPT], e1[RPT];
      const int step = RPT * tr;
      int row0 = r0 + trow;
#pragma unroll
      for (int u = 0; u < RPT; ++u) {
        const int row = row0 + u * tr;
        e0[u] = row < r1 ? *gld(rp + row) : 0;
        e1[u] = row < r1 ? *gld(rp + row + 1) : 0;
      }
      for (; row0 < r1; row0 += step) {
        int ne0[RPT], ne1[RPT];
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          const int row = row0 + step + u * tr;
          ne0[u] = row < r1 ? *gld(rp + row) : 0;
          ne1[u] = row < r1 ? *gld(rp + row + 1) : 0;
        }
        double w[RPT], xs[RPT];
        int len = 0;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          const int row = row0 + u * tr;
          w[u] = 0.0;
          xs[u] = row < r1 ? *gld(X + (int64_t)row * ldx + col) : 0.0;
          len = max(len, e1[u] - e0[u]);
        }
        for (int b = 0; b < len; b += NZB) {
          int c[RPT][NZB];
          double a[RPT][NZB], xv[RPT][NZB];
#pragma unroll
          for (int u = 0; u < RPT; ++u)
#pragma unroll
            for (int z = 0; z < NZB; ++z) {
              const int e = e0[u] + b + z;
              const bool ok = e < e1[u];
              c[u][z] = ok ? *gld(ci + e) : 0;
              a[u][z] = ok ? *gld(av + e) : 0.0;
            }
#pragma unroll
          for (int u = 0; u < RPT; ++u)
#pragma unroll
            for (int z = 0; z < NZB; ++z)
              xv[u][z] = e0[u] + b + z < e1[u] ? *gld(X + (int64_t)c[u][z] * ldx + col) : 0.0;
#pragma unroll
          for (int u = 0; u < RPT; ++u)
#pragma unroll
            for (int z = 0; z < NZB; ++z)
              if (e0[u] + b + z < e1[u]) w[u] = __builtin_fma(a[u][z], xv[u][z], w[u]);
        }
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          const int row = row0 + u * tr;
          if (row < r1) {
            *gst(P.w + (int64_t)row * k + col) = w[u];
            sxw = __builtin_fma(xs[u], w[u], sxw);
            sxx = __builtin_fma(xs[u], xs[u], sxx);
          }
          e0[u] = ne0[u];
          e1[u] = ne1[u];
        }
      }
    }
  }
  rayleigh_block_partial<NT>(P, blockIdx.x, sxw, sxx, red);
}

int spmm_chunk_rows() { return SPMM_ROWS; }
int spmm_grid(int nitems) { return nitems < SPMM_GRID ? nitems : SPMM_GRID; }

hipError_t launch_spmm(const Prob* probs, const RowItem* items, int nitems, hipStream_t st) {
  hipLaunchKernelGGL((spmm_kernel<1024, 1, 8>), dim3(spmm_grid(nitems)), dim3(1024), 0, st, probs,
                     items, nitems, SPMM_ROWS);
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
