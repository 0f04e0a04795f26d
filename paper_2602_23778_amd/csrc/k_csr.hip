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

// Vector form: G lanes per row, four columns per lane (k <= 4 G) as two
// pairs, columns 2 gl, 2 gl + 1 and 2 G + 2 gl, 2 G + 2 gl + 1 of lane gl,
// so that one 16-byte load instruction takes whole 128-byte lines of G x 16
// bytes from each of the 64 / G rows it touches (four consecutive columns per
// lane would touch twice the lines, each half used: 5 % slower at 128^3,
// k = 32).  Per chunk the block first copies the chunk's row pointers and,
// when they fit (at most NZL), its column indices and values into LDS with
// coalesced loads, so a row round costs one dependent trip to memory (the X
// gathers) instead of three.  A row's G nonzeros of a round are gathered
// together; slots past the row's end load nothing (on the 7-point stencil,
// one slot in eight), and the sum runs in CSR order.  Chunks are taken
// block-strided as in the scalar form; the block's Rayleigh partial goes to
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
  const int gl = lane % G;
  const Prob& P = probs[0];
  if (P.ctrl->stopped) return;
  const int n = P.n, k = P.k;
  const int32_t* __restrict__ rp = P.rp;
  const int32_t* __restrict__ ci = P.ci;
  const double* __restrict__ av = P.av;
  const double* __restrict__ X = P.x;
  const int64_t ldx = P.ldx;
  double* __restrict__ W = P.w;
  // this lane's columns: pair h starts at column 2 G h + 2 gl; whole pairs
  // move as 16-byte loads (stores) when the rows of X (W) are 16-byte aligned
  int col[2];
  bool px[2], pw[2];
  const bool xal = (ldx & 1) == 0 && (((uintptr_t)X) & 15) == 0;
  const bool wal = (k & 1) == 0 && (((uintptr_t)W) & 15) == 0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    col[h] = 2 * G * h + 2 * gl;
    px[h] = xal && col[h] + 1 < k;
    pw[h] = wal && col[h] + 1 < k;
  }
  auto load4 = [&](int64_t row, double (&v)[4]) {
    const double* p = X + row * ldx;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (px[h]) {
        const v2d a = *gld(reinterpret_cast<const v2d*>(p + col[h]));
        v[2 * h] = a.x;
        v[2 * h + 1] = a.y;
      } else {
        v[2 * h] = col[h] < k ? *gld(p + col[h]) : 0.0;
        v[2 * h + 1] = col[h] + 1 < k ? *gld(p + col[h] + 1) : 0.0;
      }
    }
  };
  double sxw[4] = {0.0, 0.0, 0.0, 0.0}, sxx[4] = {0.0, 0.0, 0.0, 0.0};
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem item = items[it];
    const int r0 = item.blk * chunk_rows, r1 = min(n, r0 + chunk_rows);
    __syncthreads();  // the previous chunk's LDS copies are no longer read
    // the copies into LDS request all their entries before storing any
    // (indices clamped into the chunk): a loop of load-then-store would wait
    // one round trip per pass
    {
      constexpr int RU = (SPMM_ROWS + NT) / NT;  // passes over rows 0..chunk
      int v[RU];
#pragma unroll
      for (int u = 0; u < RU; ++u) v[u] = *gld(rp + r0 + min(tid + u * NT, r1 - r0));
#pragma unroll
      for (int u = 0; u < RU; ++u)
        if (tid + u * NT <= r1 - r0) srp[tid + u * NT] = v[u];
    }
    __syncthreads();
    const int E0 = srp[0], nz = srp[r1 - r0] - E0;
    const bool staged = nz <= NZL;
    if (staged && nz > 0) {
      constexpr int ZU = NZL / NT;
      int cv[ZU];
      double avv[ZU];
#pragma unroll
      for (int u = 0; u < ZU; ++u) {
        const int i = min(tid + u * NT, nz - 1);
        cv[u] = *gld(ci + E0 + i);
        avv[u] = *gld(av + E0 + i);
      }
#pragma unroll
      for (int u = 0; u < ZU; ++u)
        if (tid + u * NT < nz) {
          sci[tid + u * NT] = cv[u];
          sav[tid + u * NT] = avv[u];
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
        for (int z = 0; z < G; ++z) {
          if (eb + z < e1) {
            load4(cz[z], xv[z]);
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) xv[z][q] = 0.0;
          }
        }
#pragma unroll
        for (int z = 0; z < G; ++z)
#pragma unroll
          for (int q = 0; q < 4; ++q) w[q] = __builtin_fma(az[z], xv[z][q], w[q]);
      }
      if (rok) {
        double* wp = W + (int64_t)row * k;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (pw[h]) {
            *gst(reinterpret_cast<v2d*>(wp + col[h])) = v2d{w[2 * h], w[2 * h + 1]};
          } else {
            if (col[h] < k) *gst(wp + col[h]) = w[2 * h];
            if (col[h] + 1 < k) *gst(wp + col[h] + 1) = w[2 * h + 1];
          }
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
      red[0][wave][col[q / 2] + q % 2] = sxw[q];
      red[1][wave][col[q / 2] + q % 2] = sxx[q];
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
// block-strided as in the vector form, over a grid of as many blocks as are
// resident at once.  16 rows: a 149k-row matrix gives 9.3k chunks, about
// five per block, so the last round leaves few CUs idle (32-row chunks
// measured 7 % slower on that shape, 8-row chunks 43 %).
constexpr int ROW_CHUNK = 16;

template <int NT, int L, int KC>
__global__ __launch_bounds__(NT) void spmm_row_kernel(const Prob* __restrict__ probs,
                                                     const RowItem* __restrict__ items, int nitems,
                                                     int chunk_rows) {
  static_assert(64 % L == 0 && KC <= L, "row groups must tile a wavefront");
  typedef double v2d __attribute__((ext_vector_type(2)));
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
  // an X row of k = KC doubles as 16-byte pairs (8-byte aligned, which
  // global loads accept) and one last double for odd k: 3 loads instead of
  // 5 at k = 5
  auto xrow = [&](int c, double (&v)[KC]) {
    const double* p = X + (int64_t)c * ldx;
    if (k == KC) {
#pragma unroll
      for (int q = 0; q + 1 < KC; q += 2) {
        const v2d a = *gld(reinterpret_cast<const v2d*>(p + q));
        v[q] = a.x;
        v[q + 1] = a.y;
      }
      if (KC & 1) v[KC - 1] = *gld(p + KC - 1);
    } else {
#pragma unroll
      for (int q = 0; q < KC; ++q) v[q] = q < k ? *gld(p + q) : 0.0;
    }
  };
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
        xrow(ca, xa);
        xrow(cb, xb);
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

// Rows per chunk of either form; REFINE_SPMM_CHUNK overrides it (a tuning
// hook, read once per process; the vector form's chunk stays within its LDS
// copy of SPMM_ROWS + 1 row pointers).
static int env_int(const char* name) {
  const char* env = getenv(name);
  return env ? atoi(env) : 0;
}
static int chunk_rows_for(bool row_form) {
  static const int c = env_int("REFINE_SPMM_CHUNK");
  if (row_form) return (c >= 8 && c <= 1024) ? c : ROW_CHUNK;
  return (c >= 8 && c <= SPMM_ROWS) ? c : SPMM_ROWS;
}

int spmm_chunk_rows(int lanes) { return chunk_rows_for(lanes != 0); }

typedef void (*SpmmKernel)(const Prob*, const RowItem*, int, int);

template <int L>
static SpmmKernel row_kernel_for(int k) {
  switch (k) {
    case 1: return spmm_row_kernel<256, L, 1>;
    case 2: return spmm_row_kernel<256, L, 2>;
    case 3: return spmm_row_kernel<256, L, 3>;
    case 4: return spmm_row_kernel<256, L, 4>;
    case 5: return spmm_row_kernel<256, L, 5>;
    case 6: return spmm_row_kernel<256, L, 6>;
    case 7: return spmm_row_kernel<256, L, 7>;
    case 8: return spmm_row_kernel<256, L, 8>;
    default: return nullptr;
  }
}

// The kernel of the product for k columns and `lanes` lanes per row (0: the
// vector form with G = pow2ceil(k) / 4 lanes per row, at least 1).
static SpmmKernel spmm_kernel_for(int k, int lanes) {
  if (lanes == 8) return row_kernel_for<8>(k);
  if (lanes == 16) return row_kernel_for<16>(k);
  if (lanes == 32) return row_kernel_for<32>(k);
  if (lanes) return nullptr;
  int kp = 1;
  while (kp < k) kp *= 2;
  switch (std::max(1, kp / 4)) {
    case 1: return spmm_vec_kernel<256, 1>;
    case 2: return spmm_vec_kernel<256, 2>;
    case 4: return spmm_vec_kernel<256, 4>;
    case 8: return spmm_vec_kernel<256, 8>;
    case 16: return spmm_vec_kernel<256, 16>;
    case 32: return spmm_vec_kernel<256, 32>;
    default: return nullptr;
  }
}

// Grid of the product over nitems chunks on the current device: as many
// 256-thread blocks as are resident at once (the occupancy of the kernel's
// registers and LDS times the CU count: 3 x 256 for the vector form at
// k = 32, 7 x 256 for the row form at k = 5), at most one per chunk.
// REFINE_SPMM_GRID overrides it (a tuning hook).  0 if k or lanes has no
// kernel.
int spmm_grid(int nitems, int k, int lanes) {
  const SpmmKernel fn = spmm_kernel_for(k, lanes);
  if (!fn || nitems <= 0) return 0;
  static const int genv = env_int("REFINE_SPMM_GRID");
  int g = 0;
  if (genv >= 64 && genv <= 65536) {
    g = genv;
  } else {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn), 256, 0) !=
            hipSuccess ||
        per_cu <= 0)
      per_cu = 1;
    g = per_cu * cus;
  }
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

hipError_t launch_spmm(const Prob* probs, const RowItem* items, int nitems, int k, int lanes, int grid,
                       hipStream_t st) {
  const SpmmKernel fn = spmm_kernel_for(k, lanes);
  if (!fn || grid <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, st, probs, items, nitems, chunk_rows_for(lanes != 0));
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
