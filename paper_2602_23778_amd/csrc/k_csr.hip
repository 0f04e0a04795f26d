// Line 1 of Algorithm 4 for sparse A in CSR form, fused with the first
// reduction of the step (eq. Rayleigh): W = A X, and per block the column
// sums of x_j * w_j and x_j * x_j.
//
// The work is bound by memory: 12 B per nonzero plus the X row gathers (an
// X row is k doubles, reused across the neighbouring rows that name it) and
// the W write.  Rows are taken in chunks of SPMM_ROWS; a block takes the
// chunks blockIdx.x, blockIdx.x + gridDim.x, ..., so that at any moment the
// whole GPU works on one contiguous window of rows and the far stencil
// neighbours (N^2 rows away on a 3-D grid) are still in the caches.
#include <algorithm>

#include "common.h"
#include "dev_util.h"

namespace rfk {

// Rows per chunk of the SpMM (a block takes every gridDim-th chunk).
constexpr int SPMM_ROWS = 256;

// Vector form: G lanes per row, four columns per lane (k <= 4 G), so an X
// row gather is G lanes x 32 bytes (two 16-byte loads per lane when X rows
// are 16-byte aligned) and a wavefront gathers 64 / G rows per instruction.
// Per chunk the block first copies the chunk's row pointers and, when they
// fit (at most NZL), its column indices and values into LDS with coalesced
// loads, so a row round costs one dependent trip to memory (the X gathers)
// instead of three.  A row's G nonzeros of a round are gathered together
// (the lanes past the row's end use a = 0 and the row's own X row, adding
// exact zeros); the sum runs in CSR order.  Chunks are taken block-strided
// as in the scalar form; the block's Rayleigh partial goes to
// dpart[blockIdx.x].
template <int NT, int G>
__global__ __launch_bounds__(NT) void spmm_vec_kernel(const Prob* __restrict__ probs,
                                                     const RowItem* __restrict__ items, int nitems,
                                                     int chunk_rows) {
  typedef double v2d __attribute__((ext_vector_type(2)));
  constexpr int NW = NT / 64, RPB = NT / G, NZL = 2048;
  __shared__ double red[2][NW][4 * G];
  __shared__ double sav[NZL];
  __shared__ int32_t sci[NZL];
  __shared__ int32_t srp[SPMM_ROWS + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int gl = lane % G, c0 = 4 * gl;
  const Prob& P = probs[0];
  if (P.ctrl->stopped) return;
  const int n = P.n, k = P.k;
  const int32_t* __restrict__ rp = P.rp;
  const int32_t* __restrict__ ci = P.ci;
  const double* __restrict__ av = P.av;
  const double* __restrict__ X = P.x;
  const int64_t ldx = P.ldx;
  double* __restrict__ W = P.w;
  // this lane's valid columns; the paired loads need 16-byte aligned rows
  const int vc = max(0, min(4, k - c0));
  const bool vec = vc == 4 && (ldx & 1) == 0 && (((uintptr_t)X) & 15) == 0 && (k & 1) == 0;
  auto load4 = [&](int64_t row, double (&v)[4]) {
    const double* p = X + row * ldx + c0;
    if (vec) {
      const v2d a = *gld(reinterpret_cast<const v2d*>(p));
      const v2d b = *gld(reinterpret_cast<const v2d*>(p + 2));
      v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = q < vc ? *gld(p + q) : 0.0;
    }
  };
  double sxw[4] = {0.0, 0.0, 0.0, 0.0}, sxx[4] = {0.0, 0.0, 0.0, 0.0};
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem item = items[it];
    const int r0 = item.blk * chunk_rows, r1 = min(n, r0 + chunk_rows);
    __syncthreads();  // the previous chunk's LDS copies are no longer read
    for (int i = tid; i <= r1 - r0; i += NT) srp[i] = *gld(rp + r0 + i);
    __syncthreads();
    const int E0 = srp[0], nz = srp[r1 - r0] - E0;
    const bool staged = nz <= NZL;
    if (staged) {
      for (int i = tid; i < nz; i += NT) {
        sci[i] = *gld(ci + E0 + i);
        sav[i] = *gld(av + E0 + i);
      }
    }
    __syncthreads();
    for (int rb = r0; rb < r1; rb += RPB) {
      const int row = rb + tid / G;
      const bool rok = row < r1;
      const int rr = rok ? row : r0;
      const int e0 = srp[rr - r0], e1 = rok ? srp[rr - r0 + 1] : e0;
      double xs[4];
      load4(rr, xs);
      double w[4] = {0.0, 0.0, 0.0, 0.0};
      for (int eb = e0; eb < e1; eb += G) {
        int cz[G];
        double az[G];
#pragma unroll
        for (int z = 0; z < G; ++z) {
          const int e = eb + z;
          const bool ok = e < e1;
          cz[z] = !ok ? rr : staged ? sci[e - E0] : *gld(ci + e);
          az[z] = !ok ? 0.0 : staged ? sav[e - E0] : *gld(av + e);
        }
        double xv[G][4];
#pragma unroll
        for (int z = 0; z < G; ++z) load4(cz[z], xv[z]);
#pragma unroll
        for (int z = 0; z < G; ++z)
#pragma unroll
          for (int q = 0; q < 4; ++q) w[q] = __builtin_fma(az[z], xv[z][q], w[q]);
      }
      if (rok) {
        double* wp = W + (int64_t)row * k + c0;
        if (vec) {
          *gst(reinterpret_cast<v2d*>(wp)) = v2d{w[0], w[1]};
          *gst(reinterpret_cast<v2d*>(wp + 2)) = v2d{w[2], w[3]};
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (q < vc) *gst(wp + q) = w[q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          sxw[q] = __builtin_fma(xs[q], w[q], sxw[q]);
          sxx[q] = __builtin_fma(xs[q], xs[q], sxx[q]);
        }
      }
    }
  }
  // Rayleigh partial of the block: lanes with equal gl hold the same columns
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int o = G; o < 64; o *= 2) {
      sxw[q] += __shfl_xor(sxw[q], o);
      sxx[q] += __shfl_xor(sxx[q], o);
    }
  }
  if (lane < G) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      red[0][wave][c0 + q] = sxw[q];
      red[1][wave][c0 + q] = sxx[q];
    }
  }
  __syncthreads();
  if (tid < k) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < NW; ++w) {
      a += red[0][w][tid];
      b += red[1][w][tid];
    }
    *gst(P.dpart + (int64_t)blockIdx.x * 2 * k + tid) = a;
    *gst(P.dpart + (int64_t)blockIdx.x * 2 * k + k + tid) = b;
  }
}

// Grid: three resident 256-thread blocks on each of the 256 CUs.
constexpr int SPMM_GRID = 768;

int spmm_chunk_rows() { return SPMM_ROWS; }
int spmm_grid(int nitems) { return nitems < SPMM_GRID ? nitems : SPMM_GRID; }

// k picks the lanes per row: G = pow2ceil(k) / 4, at least 1.
hipError_t launch_spmm(const Prob* probs, const RowItem* items, int nitems, int k, hipStream_t st) {
  const int grid = spmm_grid(nitems);
  int kp = 1;
  while (kp < k) kp *= 2;
  const int g = std::max(1, kp / 4);
  switch (g) {
#define RFK_SPMM(GV)                                                                            \
  case GV:                                                                                      \
    hipLaunchKernelGGL((spmm_vec_kernel<256, GV>), dim3(grid), dim3(256), 0, st, probs, items, \
                       nitems, SPMM_ROWS);                                                      \
    break;
    RFK_SPMM(1) RFK_SPMM(2) RFK_SPMM(4) RFK_SPMM(8) RFK_SPMM(16) RFK_SPMM(32)
#undef RFK_SPMM
    default:
      return hipErrorInvalidValue;
  }
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
