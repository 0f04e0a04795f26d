// The product step of Algorithm 4 for sparse A in CSR form, fused with the first
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
#include <cstdlib>

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

// Row form for narrow X (k <= KC <= 8) and wide rows: L lanes share a row
// and stride over its nonzeros, two at a time per lane, so a row's column
// indices and values are read by coalesced loads and a row of tens of
// nonzeros spreads over the lanes.  The next pair's index and value are
// requested before the current pair's X gathers are used, so a round waits
// on one memory trip, not two.  Each lane accumulates all k columns of its
// nonzeros (lanes past the row's end use a = 0 and the row's own X row,
// adding exact zeros); the row's sum is then a butterfly over its L lanes
// (the terms are associated differently from CSR order, within the rounding
// of any FP64 order).  Lane j < k of the row owns column j: it writes w_rj
// and keeps column j's Rayleigh terms.  Chunks of ROW_CHUNK rows, taken
// block-strided as in the vector form, over a grid sized to the occupancy.
// 32 rows: a 149k-row matrix gives 4.7k chunks, two or three per block of
// the grid, so the last round of chunks leaves few CUs idle (64-row chunks,
// one or two per block, measured 4.6 % slower on that shape).
constexpr int ROW_CHUNK = 32;
constexpr int ROW_GRID = 2048;

template <int NT, int L, int KC>
__global__ __launch_bounds__(NT) void spmm_row_kernel(const Prob* __restrict__ probs,
                                                     const RowItem* __restrict__ items, int nitems,
                                                     int chunk_rows) {
  static_assert(64 % L == 0 && KC <= L, "row groups must tile a wavefront");
  constexpr int NW = NT / 64, RPB = NT / L;
  __shared__ double red[2][NW][KC];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = lane % L;
  const Prob& P = probs[0];
  if (P.ctrl->stopped) return;
  const int n = P.n, k = P.k;
  const int32_t* __restrict__ rp = P.rp;
  const int32_t* __restrict__ ci = P.ci;
  const double* __restrict__ av = P.av;
  const double* __restrict__ X = P.x;
  const int64_t ldx = P.ldx;
  double* __restrict__ W = P.w;
  double sxw = 0.0, sxx = 0.0;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem item = items[it];
    const int r0 = item.blk * chunk_rows, r1 = min(n, r0 + chunk_rows);
    for (int rb = r0; rb < r1; rb += RPB) {
      const int row = rb + tid / L;
      const bool rok = row < r1;
      const int rr = rok ? row : r0;
      const int e0 = *gld(rp + rr), e1 = rok ? *gld(rp + rr + 1) : e0;
      auto fetch = [&](int e, int& c0, double& a0, int& c1, double& a1) {
        const bool ok0 = e < e1, ok1 = e + L < e1;
        c0 = ok0 ? *gld(ci + e) : rr;
        a0 = ok0 ? *gld(av + e) : 0.0;
        c1 = ok1 ? *gld(ci + e + L) : rr;
        a1 = ok1 ? *gld(av + e + L) : 0.0;
      };
      double acc[KC];
#pragma unroll
      for (int q = 0; q < KC; ++q) acc[q] = 0.0;
      int ca, cb;
      double aa, ab;
      fetch(e0 + j, ca, aa, cb, ab);
      for (int e = e0 + j; e < e1; e += 2 * L) {
        double xa[KC], xb[KC];
#pragma unroll
        for (int q = 0; q < KC; ++q) {
          xa[q] = q < k ? *gld(X + (int64_t)ca * ldx + q) : 0.0;
          xb[q] = q < k ? *gld(X + (int64_t)cb * ldx + q) : 0.0;
        }
        int nca, ncb;
        double naa, nab;
        fetch(e + 2 * L, nca, naa, ncb, nab);
#pragma unroll
        for (int q = 0; q < KC; ++q) acc[q] = __builtin_fma(ab, xb[q], __builtin_fma(aa, xa[q], acc[q]));
        ca = nca;
        cb = ncb;
        aa = naa;
        ab = nab;
      }
#pragma unroll
      for (int q = 0; q < KC; ++q)
#pragma unroll
        for (int o = L / 2; o >= 1; o /= 2) acc[q] += __shfl_xor(acc[q], o);
      if (rok && j < k) {
        double wv = 0.0;
#pragma unroll
        for (int q = 0; q < KC; ++q)
          if (q == j) wv = acc[q];
        *gst(W + (int64_t)row * k + j) = wv;
        const double xv = *gld(X + (int64_t)row * ldx + j);
        sxw = __builtin_fma(xv, wv, sxw);
        sxx = __builtin_fma(xv, xv, sxx);
      }
    }
  }
  // column j's partial over the wavefront's row groups, then over waves
#pragma unroll
  for (int o = L; o < 64; o *= 2) {
    sxw += __shfl_xor(sxw, o);
    sxx += __shfl_xor(sxx, o);
  }
  if (lane < KC) {
    red[0][wave][lane] = sxw;
    red[1][wave][lane] = sxx;
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

// Rows per chunk and grid of either form; REFINE_SPMM_CHUNK and
// REFINE_SPMM_GRID override them (tuning hooks, read once per process; the
// vector form's chunk stays within its LDS copy of SPMM_ROWS + 1 row
// pointers).
static int env_int(const char* name) {
  const char* env = getenv(name);
  return env ? atoi(env) : 0;
}
static int chunk_rows_for(bool row_form) {
  static const int c = env_int("REFINE_SPMM_CHUNK");
  if (row_form) return (c >= 8 && c <= 1024) ? c : ROW_CHUNK;
  return (c >= 8 && c <= SPMM_ROWS) ? c : SPMM_ROWS;
}
static int grid_for(bool row_form) {
  static const int g = env_int("REFINE_SPMM_GRID");
  if (g >= 64 && g <= 65536) return g;
  return row_form ? ROW_GRID : SPMM_GRID;
}

int spmm_chunk_rows(int lanes) { return chunk_rows_for(lanes != 0); }
int spmm_grid(int nitems, int lanes) {
  const int g = grid_for(lanes != 0);
  return nitems < g ? nitems : g;
}

// k picks the lanes per row: G = pow2ceil(k) / 4, at least 1.
// Lanes per row of the row form for k <= 8 (0: the vector form): rows of 16
// or more nonzeros on average take the row form, with 8 lanes (two nonzeros
// per lane and round) up to 160 and 16 beyond.  REFINE_SPMM_L overrides it
// (0, 8, 16 or 32; a tuning hook).
int spmm_row_lanes(int k, int64_t n, int64_t nnz) {
  if (const char* env = getenv("REFINE_SPMM_L")) {
    const int l = atoi(env);
    if (l == 0) return 0;
    if ((l == 8 || l == 16 || l == 32) && k <= 8) return l;
  }
  if (k > 8 || n <= 0) return 0;
  const double mean = (double)nnz / (double)n;
  return mean < 16.0 ? 0 : mean < 160.0 ? 8 : 16;
}

template <int L>
hipError_t launch_spmm_row(const Prob* probs, const RowItem* items, int nitems, int k, int grid,
                           hipStream_t st) {
  switch (k) {
#define RFK_SPMM_ROW(KV)                                                                         \
  case KV:                                                                                       \
    hipLaunchKernelGGL((spmm_row_kernel<256, L, KV>), dim3(grid), dim3(256), 0, st, probs, items, \
                       nitems, chunk_rows_for(true));                                            \
    break;
    RFK_SPMM_ROW(1) RFK_SPMM_ROW(2) RFK_SPMM_ROW(3) RFK_SPMM_ROW(4)
    RFK_SPMM_ROW(5) RFK_SPMM_ROW(6) RFK_SPMM_ROW(7) RFK_SPMM_ROW(8)
#undef RFK_SPMM_ROW
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_spmm(const Prob* probs, const RowItem* items, int nitems, int k, int lanes,
                       hipStream_t st) {
  const int grid = spmm_grid(nitems, lanes);
  if (lanes == 8) return launch_spmm_row<8>(probs, items, nitems, k, grid, st);
  if (lanes == 16) return launch_spmm_row<16>(probs, items, nitems, k, grid, st);
  if (lanes == 32) return launch_spmm_row<32>(probs, items, nitems, k, grid, st);
  if (lanes) return hipErrorInvalidValue;
  int kp = 1;
  while (kp < k) kp *= 2;
  const int g = std::max(1, kp / 4);
  switch (g) {
#define RFK_SPMM(GV)                                                                            \
  case GV:                                                                                      \
    hipLaunchKernelGGL((spmm_vec_kernel<256, GV>), dim3(grid), dim3(256), 0, st, probs, items, \
                       nitems, chunk_rows_for(false));                                          \
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
