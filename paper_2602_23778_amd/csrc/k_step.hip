// Lines 3-7 of Algorithm 4 (and the column normalisation of Sec. 3.3) for one
// or many problems.  The step is written so that no n x n matrix and no
// explicit H is formed (Sec. 3.2, after Table 1) and so that every pass over
// the n x k arrays streams them once:
//
//   pass 1  (wreduce)  W = sum of split-K partials; alpha_j = x_j^T x_j and
//                      x_j^T w_j per row block; the last block forms
//                      d_j = x_j^T w_j / alpha_j (eq. Rayleigh).
//   pass 2  (gram)     R = W - X D on the fly; X2^T R2, X2^T X2 (rows >= k) as
//                      per-block partials on the FP64 matrix cores, and
//                      X1^T R1, X1^T X1, R1 for the leading k rows.
//   reduce             sums the Gram partials in a fixed order.
//   kxk     (1 WG)     Y1 = X1 - I and T = -Y1^{-T} (Algorithm 1, by
//                      Gauss-Jordan with partial pivoting); with
//                      C = Y^T R = X^T R - R1 the bottom rows of V = H^T R are
//                      V2 = R2 - X2 M, M = T^T C; the top rows are X^T R.
//                      E11 (line 6), F = Y^T E_L from k x k identities, N = T F,
//                      and the updated top rows X1 + E11 - Y1 N.
//   pass 3  (update)   bottom rows: E21 = (R2 - X2 M) diag(1/(d - mu)) and
//                      X2 + E21 - X2 N, with [X2 M | X2 N] on the matrix cores;
//                      the last block forms the normalisation factors and
//                      the statistics, and accepts or rejects the step.
//   pass 4  (normalize) X = scaled update, only when the step was accepted.
#include "common.h"
#include "dev_util.h"

namespace rfk {

// ---------------------------------------------------------------------------
// pass 1
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(NT) void wreduce_kernel(const Prob* __restrict__ probs,
                                                    const RowItem* __restrict__ items, int nitems) {
  __shared__ double red[2][NT];
  __shared__ double tot[2 * KMAX];
  __shared__ int flag;
  const int tid = threadIdx.x;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem item = items[it];
    const Prob& P = probs[item.prob];
    if (P.ctrl->stopped) continue;
    const int n = P.n, k = P.k, kp = pow2ceil(k), tr = NT / kp;
    const int col = tid % kp, trow = tid / kp;
    const int r0 = item.blk * P.rbrows, r1 = min(n, r0 + P.rbrows);
    double sxw = 0.0, sxx = 0.0;
    if (col < k) {
      const int S = P.ksplit;
      const int64_t nk = (int64_t)n * k;
      for (int row = r0 + trow; row < r1; row += tr) {
        const int64_t o = (int64_t)row * k + col;
        double w;
        if (S > 1) {
          w = P.wp[o];
          for (int s = 1; s < S; ++s) w += P.wp[o + s * nk];
          P.w[o] = w;
        } else {
          w = P.w[o];
        }
        if (P.wlo) w += P.wlo[o];
        const double x = P.x[(int64_t)row * P.ldx + col];
        sxw = __builtin_fma(x, w, sxw);
        sxx = __builtin_fma(x, x, sxx);
      }
    }
    red[0][tid] = sxw;
    red[1][tid] = sxx;
    __syncthreads();
    for (int h = tr / 2; h >= 1; h /= 2) {
      if (trow < h) {
        red[0][tid] += red[0][tid + h * kp];
        red[1][tid] += red[1][tid + h * kp];
      }
      __syncthreads();
    }
    const int stride = 5 * k;
    if (trow == 0 && col < k) {
      P.part[(int64_t)item.blk * stride + col] = red[0][tid];
      P.part[(int64_t)item.blk * stride + k + col] = red[1][tid];
    }
    if (last_block_arrival(&P.ctrl->ticket_a, P.nrb, &flag)) {
      team_reduce(P.part, stride, 2 * k, P.nrb, &red[0][0], tot);
      bool bad = false;
      for (int j = tid; j < k; j += NT) {
        const double a = tot[k + j];
        const double d = tot[j] / a;
        P.vec[VEC_D * k + j] = d;
        P.vec[VEC_ALPHA * k + j] = a;
        P.vec[VEC_DINV * k + j] = 1.0 / (d - P.mu);
        if (!__builtin_isfinite(d) || !(a > 0.0)) bad = true;
      }
      if (bad) {
        P.ctrl->status = -6;
        P.ctrl->stopped = 1;
      }
      if (tid == 0) P.ctrl->ticket_a = 0;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// pass 2: Gram partials on the matrix cores.  One wavefront per 16-column
// tile ti of the left factor; it accumulates the tiles (ti, tj) of X^T R for
// all tj and of X^T X for tj >= ti (X^T X is symmetric; the reduction mirrors
// the rest).  Lane l reads row (r + l/16) at column (t*16 + l%16): the MFMA
// operand layouts of both X^T and R are plain row-major reads.
// ---------------------------------------------------------------------------
template <int CT>
__global__ __launch_bounds__(CT * 64) void gram_kernel(const Prob* __restrict__ probs,
                                                      const RowItem* __restrict__ items,
                                                      int nitems) {
  __shared__ double rsq_s[CT][64];
  const int lane = threadIdx.x & 63, ti = threadIdx.x >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem item = items[it];
    const Prob& P = probs[item.prob];
    if (P.ctrl->stopped) continue;
    const int n = P.n, k = P.k;
    const int ct_used = (k + 15) / 16;
    const bool has_lo = P.wlo != nullptr;
    const double* __restrict__ X = P.x;
    const int64_t ldx = P.ldx;
    const int r0 = item.blk * P.gbrows, r1 = min(n, r0 + P.gbrows);
    const int kk2 = k * k;
    double dv[CT];
    bool cok[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int c = t * 16 + r16;
      cok[t] = c < k;
      dv[t] = cok[t] ? P.vec[VEC_D * k + c] : 0.0;
    }
    const int ca = ti * 16 + r16;
    const bool aok = ca < k;
    double rsq[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) rsq[t] = 0.0;

    // phase 0: rows < k (leading block, only in block 0); phase 1: rows >= k
    for (int phase = 0; phase < 2; ++phase) {
      const int lo = phase == 0 ? r0 : max(r0, k);
      const int hi = phase == 0 ? min(r1, k) : r1;
      if (lo >= hi) continue;
      v4d accP[CT], accG[CT];
#pragma unroll
      for (int t = 0; t < CT; ++t) {
        accP[t] = v4d{0.0, 0.0, 0.0, 0.0};
        accG[t] = v4d{0.0, 0.0, 0.0, 0.0};
      }
      if (ti < ct_used) {
        for (int rb = lo; rb < hi; rb += 4) {
          const int row = rb + g;
          const bool rok = row < hi;
          const double* xr = X + (int64_t)(rok ? row : lo) * ldx;
          const double* wr = P.w + (int64_t)(rok ? row : lo) * k;
          const double* wl = has_lo ? P.wlo + (int64_t)(rok ? row : lo) * k : nullptr;
          const double xa = (rok && aok) ? xr[ca] : 0.0;
          double xv[CT], rv[CT];
#pragma unroll
          for (int t = 0; t < CT; ++t) {
            const int c = t * 16 + r16;
            if (rok && cok[t]) {
              const double x = xr[c];
              xv[t] = x;
              rv[t] = residual(wr[c], has_lo ? wl[c] : 0.0, x, dv[t], has_lo);
            } else {
              xv[t] = 0.0;
              rv[t] = 0.0;
            }
          }
#pragma unroll
          for (int t = 0; t < CT; ++t) {
            if (t < ct_used) {
              accP[t] = mfma_f64(xa, rv[t], accP[t]);
              if (t >= ti) accG[t] = mfma_f64(xa, xv[t], accG[t]);
            }
          }
          if (ti == 0) {
#pragma unroll
            for (int t = 0; t < CT; ++t) rsq[t] = __builtin_fma(rv[t], rv[t], rsq[t]);
            if (phase == 0 && rok) {
#pragma unroll
              for (int t = 0; t < CT; ++t)
                if (cok[t]) P.kk[KK_R1 * kk2 + row * k + t * 16 + r16] = rv[t];
            }
          }
        }
        // store the tiles: register r holds entry (ti*16 + mfma_row(g, r), t*16 + r16)
        double* dstP;
        double* dstG;
        if (phase == 0) {
          dstP = P.kk + KK_PT * kk2;
          dstG = P.kk + KK_GT * kk2;
        } else {
          dstP = P.gpart + (int64_t)item.blk * (2 * kk2 + k);
          dstG = dstP + kk2;
        }
#pragma unroll
        for (int t = 0; t < CT; ++t) {
          const int c = t * 16 + r16;
          if (t < ct_used && c < k) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = ti * 16 + mfma_row(g, r);
              if (i < k) {
                dstP[i * k + c] = accP[t][r];
                if (t >= ti) dstG[i * k + c] = accG[t][r];
              }
            }
          }
        }
      }
    }
    // blocks without rows >= k still publish zero partials
    if (max(r0, k) >= r1) {
      double* dst = P.gpart + (int64_t)item.blk * (2 * kk2 + k);
      for (int e = threadIdx.x; e < 2 * kk2; e += blockDim.x) dst[e] = 0.0;
    }
    // column sums of r^2 (wave 0 holds them, one partial per lane group)
    if (ti == 0) {
#pragma unroll
      for (int t = 0; t < CT; ++t) rsq_s[t][lane] = rsq[t];
    }
    __syncthreads();
    if (threadIdx.x < CT * 16) {
      const int t = threadIdx.x / 16, c16 = threadIdx.x % 16, c = t * 16 + c16;
      if (c < k) {
        const double s = rsq_s[t][c16] + rsq_s[t][16 + c16] + rsq_s[t][32 + c16] + rsq_s[t][48 + c16];
        P.gpart[(int64_t)item.blk * (2 * kk2 + k) + 2 * kk2 + c] = s;
      }
    }
    __syncthreads();
  }
}

// Sums the Gram partials of every problem (fixed order over blocks).  Slots
// [0, k^2) are X2^T R2, [k^2, 2k^2) X2^T X2 (lower tiles mirrored from the
// upper ones), [2k^2, 2k^2 + k) the column sums of r^2.
struct GramRedItem {
  int32_t prob, s0;
};
__global__ __launch_bounds__(256) void gram_reduce_kernel(const Prob* __restrict__ probs,
                                                          const GramRedItem* __restrict__ items,
                                                          int nitems) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const GramRedItem item = items[it];
    const Prob& P = probs[item.prob];
    if (P.ctrl->stopped) continue;
    const int k = P.k, kk2 = k * k, S = 2 * kk2 + k;
    const int s = item.s0 + threadIdx.x;
    if (s >= S) continue;
    int src = s;
    if (s >= kk2 && s < 2 * kk2) {
      const int e = s - kk2, i = e / k, j = e % k;
      if (i / 16 > j / 16) src = kk2 + j * k + i;
    }
    const int stride = S;
    double acc = 0.0;
    for (int b = 0; b < P.ngb; ++b) acc += P.gpart[(int64_t)b * stride + src];
    if (s < kk2)
      P.kk[KK_P2 * kk2 + s] = acc;
    else if (s < 2 * kk2)
      P.kk[KK_G2 * kk2 + (s - kk2)] = acc;
    else
      P.vec[VEC_RSQ * k + (s - 2 * kk2)] = acc;
  }
}

// ---------------------------------------------------------------------------
// k-by-k work, one workgroup per problem.
// ---------------------------------------------------------------------------
constexpr int KXK_NT = 1024;

// out(i, j) = sum_l a(i, l) b(l, j) for i, j < k; each thread owns 4x4 tiles.
template <class FA, class FB, class FO>
__device__ __forceinline__ void kk_gemm(int k, FA a, FB b, FO store) {
  const int nt = (k + 3) / 4;
  for (int t = threadIdx.x; t < nt * nt; t += blockDim.x) {
    const int i0 = (t / nt) * 4, j0 = (t % nt) * 4;
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    for (int l = 0; l < k; ++l) {
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) av[u] = (i0 + u < k) ? a(i0 + u, l) : 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) bv[v] = (j0 + v < k) ? b(l, j0 + v) : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = __builtin_fma(av[u], bv[v], acc[u][v]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (i0 + u < k && j0 + v < k) store(i0 + u, j0 + v, acc[u][v]);
  }
}

__global__ __launch_bounds__(KXK_NT) void kxk_kernel(const Prob* __restrict__ probs, int nprob,
                                                     int lds_doubles) {
  extern __shared__ double smem[];
  __shared__ int piv[KMAX];
  __shared__ double fcol[KMAX];
  __shared__ double redv[KXK_NT / 64];
  __shared__ int sflag;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int p = blockIdx.x; p < nprob; p += gridDim.x) {
    const Prob& P = probs[p];
    Ctrl* ctrl = P.ctrl;
    __syncthreads();
    if (tid == 0) ctrl->apply = 0;
    if (ctrl->stopped) continue;
    const int n = P.n, k = P.k, kk2 = k * k;
    const int64_t ldx = P.ldx;
    const double* __restrict__ X = P.x;
    double* base = (4 * kk2 <= lds_doubles) ? smem : P.kk + KK_S0 * kk2;
    double* Yi = base;
    double* E1 = base + kk2;
    double* F = base + 2 * kk2;
    double* X1 = base + 3 * kk2;
    const double* PT = P.kk + KK_PT * kk2;
    const double* P2 = P.kk + KK_P2 * kk2;
    const double* GT = P.kk + KK_GT * kk2;
    const double* G2 = P.kk + KK_G2 * kk2;
    const double* R1 = P.kk + KK_R1 * kk2;
    double* Cm = P.kk + KK_CM * kk2;  // k x 2k, [M | N]
    double* X1n = P.kk + KK_X1N * kk2;
    const double* d = P.vec + VEC_D * k;
    const double* alpha = P.vec + VEC_ALPHA * k;
    const double* dinv = P.vec + VEC_DINV * k;

    // Y1 = X1 - I_k (Algorithm 1, line 1)
    for (int e = tid; e < kk2; e += KXK_NT) {
      const int i = e / k, j = e % k;
      const double x = X[(int64_t)i * ldx + j];
      X1[e] = x;
      Yi[e] = x - (i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    // ||Y1||_1: maximum column sum
    double cs = 0.0;
    if (tid < k)
      for (int i = 0; i < k; ++i) cs += fabs(Yi[i * k + tid]);
    for (int o = 32; o >= 1; o /= 2) cs = fmax(cs, __shfl_xor(cs, o));
    if (lane == 0) redv[wave] = cs;
    if (tid == 0) sflag = 0;
    __syncthreads();
    double norm1 = 0.0;
    for (int w = 0; w < KXK_NT / 64; ++w) norm1 = fmax(norm1, redv[w]);

    // Y1^{-1} by Gauss-Jordan elimination with partial pivoting, in place.
    for (int c = 0; c < k; ++c) {
      if (wave == 0) {
        // pivot: first row of largest |y_rc|, r >= c
        double best = -1.0;
        int bi = k;
        for (int r = c + lane; r < k; r += 64) {
          const double v = fabs(Yi[r * k + c]);
          if (v > best) {
            best = v;
            bi = r;
          }
        }
        for (int o = 32; o >= 1; o /= 2) {
          const double ob = __shfl_xor(best, o);
          const int oi = __shfl_xor(bi, o);
          if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
          }
        }
        if (best <= 0.0) {
          if (lane == 0) sflag = 1;
        } else {
          if (lane == 0) piv[c] = bi;
          if (bi != c)
            for (int j = lane; j < k; j += 64) {
              const double t = Yi[c * k + j];
              Yi[c * k + j] = Yi[bi * k + j];
              Yi[bi * k + j] = t;
            }
          const double pv = Yi[c * k + c];
          const double ipv = 1.0 / pv;
          for (int j = lane; j < k; j += 64) Yi[c * k + j] = (j == c ? 1.0 : Yi[c * k + j]) * ipv;
          for (int r = lane; r < k; r += 64) fcol[r] = (r == c) ? 0.0 : Yi[r * k + c];
        }
      }
      __syncthreads();
      if (sflag) break;
      for (int e = tid; e < kk2; e += KXK_NT) {
        const int r = e / k, j = e % k;
        if (r != c) {
          const double y = (j == c) ? 0.0 : Yi[e];
          Yi[e] = y - fcol[r] * Yi[c * k + j];
        }
      }
      __syncthreads();
    }
    if (sflag) {
      if (tid == 0) {
        ctrl->status = -4;
        ctrl->stopped = 1;
      }
      continue;
    }
    for (int c = k - 1; c >= 0; --c) {
      const int pc = piv[c];
      if (pc != c && tid < k) {
        const double t = Yi[tid * k + c];
        Yi[tid * k + c] = Yi[tid * k + pc];
        Yi[tid * k + pc] = t;
      }
      __syncthreads();
    }
    // ||Y1^{-1}||_1 and the condition test of Algorithm 1
    cs = 0.0;
    if (tid < k)
      for (int i = 0; i < k; ++i) cs += fabs(Yi[i * k + tid]);
    for (int o = 32; o >= 1; o /= 2) cs = fmax(cs, __shfl_xor(cs, o));
    if (lane == 0) redv[wave] = cs;
    __syncthreads();
    double ninv = 0.0;
    for (int w = 0; w < KXK_NT / 64; ++w) ninv = fmax(ninv, redv[w]);
    const double cond = norm1 * ninv;
    bool bad_in = false;
    for (int j = 0; j < k; ++j)
      if (!__builtin_isfinite(d[j]) || !__builtin_isfinite(alpha[j])) bad_in = true;
    if (!(cond <= 1.0 / ((double)n * UNIT_ROUNDOFF)) || bad_in) {
      __syncthreads();
      if (tid == 0) {
        ctrl->status = bad_in || !__builtin_isfinite(cond) ? (bad_in ? -6 : -4) : -4;
        ctrl->stopped = 1;
      }
      continue;
    }

    // C = Y^T R = (X1^T R1 + X2^T R2) - R1, stored in F; M = T^T C = -Y1^{-1} C
    for (int e = tid; e < kk2; e += KXK_NT) F[e] = (PT[e] + P2[e]) - R1[e];
    __syncthreads();
    kk_gemm(
        k, [&](int i, int l) { return Yi[i * k + l]; }, [&](int l, int j) { return F[l * k + j]; },
        [&](int i, int j, double v) { Cm[i * 2 * k + j] = -v; });
    // E11 (line 6 of Algorithm 4)
    double e1sq = 0.0;
    const double delta = P.delta;
    for (int e = tid; e < kk2; e += KXK_NT) {
      const int i = e / k, j = e % k;
      double v;
      if (i == j) {
        v = (1.0 - alpha[i]) * 0.5;
      } else if (fabs(d[j] - d[i]) <= delta) {
        v = P.beta_zero ? 0.0 : -(GT[e] + G2[e]) * 0.5;
      } else {
        v = (PT[e] + P2[e]) / (d[j] - d[i]);
      }
      E1[e] = v;
      e1sq = __builtin_fma(v, v, e1sq);
    }
    for (int o = 32; o >= 1; o /= 2) e1sq += __shfl_xor(e1sq, o);
    __syncthreads();
    if (lane == 0) redv[wave] = e1sq;
    __syncthreads();
    // F = Y^T E_L = X1^T E11 + (X2^T R2 - X2^T X2 M) diag(1/(d - mu)) - E11
    kk_gemm(
        k, [&](int i, int l) { return X1[l * k + i]; }, [&](int l, int j) { return E1[l * k + j]; },
        [&](int i, int j, double v) { F[i * k + j] = v; });
    kk_gemm(
        k, [&](int i, int l) { return G2[i * k + l]; },
        [&](int l, int j) { return Cm[l * 2 * k + j]; },
        [&](int i, int j, double v) {
          F[i * k + j] = F[i * k + j] + (P2[i * k + j] - v) * dinv[j] - E1[i * k + j];
        });
    __syncthreads();
    // N = T F = -Y1^{-T} F, into the right half of Cm
    kk_gemm(
        k, [&](int i, int l) { return Yi[l * k + i]; }, [&](int l, int j) { return F[l * k + j]; },
        [&](int i, int j, double v) { Cm[i * 2 * k + k + j] = -v; });
    __syncthreads();
    // top rows of the update: X1 + E11 - Y1 N
    kk_gemm(
        k, [&](int i, int l) { return X1[i * k + l] - (i == l ? 1.0 : 0.0); },
        [&](int l, int j) { return Cm[l * 2 * k + k + j]; },
        [&](int i, int j, double v) { X1n[i * k + j] = X1[i * k + j] + E1[i * k + j] - v; });
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < KXK_NT / 64; ++w) s += redv[w];
      P.vec[VEC_E1SQ * k] = s;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// pass 3: update of the bottom rows on the matrix cores, statistics and the
// accept/reject decision.  Each wavefront owns 16 rows; B = [M | N] (k x 2k)
// is staged through LDS in chunks of 16 rows.
// ---------------------------------------------------------------------------
template <int CT>
__global__ __launch_bounds__(512) void update_kernel(const Prob* __restrict__ probs,
                                                    const RowItem* __restrict__ items, int nitems) {
  constexpr int NT = 512, WAVES = 8, KCU = 16, LDC = 2 * CT * 16 + 2;
  __shared__ double Cs[KCU * LDC];
  __shared__ double colred[2][WAVES][CT * 16];
  __shared__ double tot[2 * KMAX + 8];
  __shared__ double scr[NT];
  __shared__ int flag;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem item = items[it];
    const Prob& P = probs[item.prob];
    if (P.ctrl->stopped) continue;
    const int n = P.n, k = P.k, kk2 = k * k;
    const bool has_lo = P.wlo != nullptr;
    const double* __restrict__ X = P.x;
    const int64_t ldx = P.ldx;
    const double* __restrict__ Cm = P.kk + KK_CM * kk2;
    const double* __restrict__ X1n = P.kk + KK_X1N * kk2;
    const int r0 = item.blk * P.rbrows, r1 = min(n, r0 + P.rbrows);
    double dv[CT], di[CT], xsq[CT], esq[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int c = t * 16 + r16;
      dv[t] = c < k ? P.vec[VEC_D * k + c] : 0.0;
      di[t] = c < k ? P.vec[VEC_DINV * k + c] : 0.0;
      xsq[t] = 0.0;
      esq[t] = 0.0;
    }
    const int nkc = (k + KCU - 1) / KCU;
    for (int rc = r0; rc < r1; rc += WAVES * 16) {
      v4d accM[CT], accN[CT];
#pragma unroll
      for (int t = 0; t < CT; ++t) {
        accM[t] = v4d{0.0, 0.0, 0.0, 0.0};
        accN[t] = v4d{0.0, 0.0, 0.0, 0.0};
      }
      const int arow = rc + wave * 16 + r16;
      const bool arok = arow < r1;
      const double* xr = X + (int64_t)(arok ? arow : r0) * ldx;
      for (int kc = 0; kc < nkc; ++kc) {
        __syncthreads();
        for (int e = tid; e < KCU * 2 * CT * 16; e += NT) {
          const int rr = e / (2 * CT * 16), cc = e % (2 * CT * 16);
          const int half = cc / (CT * 16), cj = cc % (CT * 16);
          const int kr = kc * KCU + rr;
          double v = 0.0;
          if (kr < k && cj < k) v = Cm[kr * 2 * k + half * k + cj];
          Cs[rr * LDC + cc] = v;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int kk = kc * KCU + 4 * g + s;
          const double a = (arok && kk < k) ? xr[kk] : 0.0;
          const double* brow = Cs + (4 * g + s) * LDC + r16;
#pragma unroll
          for (int t = 0; t < CT; ++t) {
            accM[t] = mfma_f64(a, brow[t * 16], accM[t]);
            accN[t] = mfma_f64(a, brow[CT * 16 + t * 16], accN[t]);
          }
        }
      }
      // epilogue: register r holds row rc + wave*16 + mfma_row(g, r), column t*16 + r16
#pragma unroll
      for (int t = 0; t < CT; ++t) {
        const int c = t * 16 + r16;
        if (c < k) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = rc + wave * 16 + mfma_row(g, r);
            if (row < r1) {
              double xt;
              if (row < k) {
                xt = X1n[row * k + c];
              } else {
                const int64_t o = (int64_t)row * k + c;
                const double x = X[(int64_t)row * ldx + c];
                const double rr = residual(P.w[o], has_lo ? P.wlo[o] : 0.0, x, dv[t], has_lo);
                const double e = (rr - accM[t][r]) * di[t];
                xt = (x + e) - accN[t][r];
                esq[t] = __builtin_fma(e, e, esq[t]);
              }
              P.xn[(int64_t)row * k + c] = xt;
              xsq[t] = __builtin_fma(xt, xt, xsq[t]);
            }
          }
        }
      }
    }
    // block partials of sum x~^2 and sum e^2 per column
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      double a = xsq[t], b = esq[t];
      a += __shfl_xor(a, 16);
      a += __shfl_xor(a, 32);
      b += __shfl_xor(b, 16);
      b += __shfl_xor(b, 32);
      if (g == 0) {
        colred[0][wave][t * 16 + r16] = a;
        colred[1][wave][t * 16 + r16] = b;
      }
    }
    __syncthreads();
    const int stride = 5 * k;
    if (tid < k) {
      double a = 0.0, b = 0.0;
      for (int w = 0; w < WAVES; ++w) {
        a += colred[0][w][tid];
        b += colred[1][w][tid];
      }
      P.part[(int64_t)item.blk * stride + 2 * k + tid] = a;
      P.part[(int64_t)item.blk * stride + 3 * k + tid] = b;
    }
    if (last_block_arrival(&P.ctrl->ticket_b, P.nrb, &flag)) {
      team_reduce(P.part + 2 * k, stride, 2 * k, P.nrb, scr, tot);
      for (int j = tid; j < k; j += NT)
        P.vec[VEC_SCALE * k + j] = P.normalize ? 1.0 / sqrt(tot[j]) : 1.0;
      if (tid == 0) {
        Ctrl* C = P.ctrl;
        double e2 = P.vec[VEC_E1SQ * k], r2 = 0.0;
        for (int j = 0; j < k; ++j) {
          e2 += tot[k + j];
          r2 += P.vec[VEC_RSQ * k + j];
        }
        const double corr = sqrt(e2);
        const double resid = sqrt(r2) / P.norm_a;
        C->corr_fro = corr;
        C->resid_rel = resid;
        bool finite = __builtin_isfinite(corr) && __builtin_isfinite(resid);
        for (int j = 0; j < k; ++j) finite = finite && __builtin_isfinite(tot[j]) && tot[j] > 0.0;
        const int h = C->iters;
        const bool grew = h >= 3 && corr > 10.0 * C->hist[(h - 3) & 3];
        if (!finite) {
          C->status = -6;
          C->stopped = 1;
        } else if (corr >= 1.0 || grew) {
          C->status = -5;
          C->stopped = 1;
        } else {
          C->apply = 1;
          C->hist[h & 3] = corr;
          C->iters = h + 1;
          if ((C->stop_mode == 1 && corr <= C->tol) || (C->stop_mode == 2 && resid <= C->tol)) {
            C->converged = 1;
            C->stopped = 1;
          }
        }
        C->ticket_b = 0;
      }
    }
    __syncthreads();
  }
}

// pass 4: X = update * scale, only for accepted steps.
template <int NT>
__global__ __launch_bounds__(NT) void normalize_kernel(const Prob* __restrict__ probs,
                                                      const RowItem* __restrict__ items,
                                                      int nitems) {
  const int tid = threadIdx.x;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem item = items[it];
    const Prob& P = probs[item.prob];
    if (!P.ctrl->apply) continue;
    const int n = P.n, k = P.k, kp = pow2ceil(k), tr = NT / kp;
    const int col = tid % kp, trow = tid / kp;
    if (col >= k) continue;
    const double s = P.vec[VEC_SCALE * k + col];
    const int r0 = item.blk * P.rbrows, r1 = min(n, r0 + P.rbrows);
    for (int row = r0 + trow; row < r1; row += tr)
      P.x[(int64_t)row * P.ldx + col] = P.xn[(int64_t)row * k + col] * s;
  }
}

// Control-word helpers issued outside the step graph.
__global__ void ctrl_reset_kernel(const Prob* __restrict__ probs, int nprob, int stop_mode,
                                  double tol) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nprob) {
    Ctrl* C = probs[p].ctrl;
    C->stopped = 0;
    C->apply = 0;
    C->status = 0;
    C->iters = 0;
    C->stop_mode = stop_mode;
    C->converged = 0;
    C->ticket_a = 0;
    C->ticket_b = 0;
    C->tol = tol;
    C->corr_fro = 0.0;
    C->resid_rel = 0.0;
    for (int i = 0; i < 4; ++i) C->hist[i] = 0.0;
  }
}

__global__ void set_x_kernel(Prob* __restrict__ probs, int p, double* x, int64_t ldx) {
  if (threadIdx.x == 0) {
    probs[p].x = x;
    probs[p].ldx = ldx;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
constexpr int ROW_NT = 1024;

hipError_t launch_wreduce(const Prob* probs, const RowItem* items, int nitems, hipStream_t st) {
  hipLaunchKernelGGL((wreduce_kernel<ROW_NT>), dim3(nitems), dim3(ROW_NT), 0, st, probs, items,
                     nitems);
  return hipGetLastError();
}

hipError_t launch_gram(const Prob* probs, const RowItem* items, int nitems, int kmax,
                       hipStream_t st) {
  const int ct = (kmax + 15) / 16;
#define RFK_CASE(CTV)                                                                         \
  case CTV:                                                                                   \
    hipLaunchKernelGGL((gram_kernel<CTV>), dim3(nitems), dim3(CTV * 64), 0, st, probs, items, \
                       nitems);                                                               \
    break;
  switch (ct) {
    RFK_CASE(1) RFK_CASE(2) RFK_CASE(3) RFK_CASE(4) RFK_CASE(5) RFK_CASE(6) RFK_CASE(7) RFK_CASE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef RFK_CASE
  return hipGetLastError();
}

hipError_t launch_gram_reduce(const Prob* probs, const GramRedItem* items, int nitems,
                              hipStream_t st) {
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(nitems), dim3(256), 0, st, probs, items, nitems);
  return hipGetLastError();
}

int kxk_lds_doubles(int kmax) {
  const int need = 4 * kmax * kmax;
  return need <= 16384 ? need : 0;  // 128 KiB of LDS at most
}

hipError_t launch_kxk(const Prob* probs, int nprob, int kmax, hipStream_t st) {
  const int ld = kxk_lds_doubles(kmax);
  hipLaunchKernelGGL(kxk_kernel, dim3(nprob), dim3(KXK_NT), (size_t)ld * sizeof(double), st, probs,
                     nprob, ld);
  return hipGetLastError();
}

hipError_t launch_update(const Prob* probs, const RowItem* items, int nitems, int kmax,
                         hipStream_t st) {
  const int ct = (kmax + 15) / 16;
#define RFK_CASE(CTV)                                                                   \
  case CTV:                                                                             \
    hipLaunchKernelGGL((update_kernel<CTV>), dim3(nitems), dim3(512), 0, st, probs, items, \
                       nitems);                                                         \
    break;
  switch (ct) {
    RFK_CASE(1) RFK_CASE(2) RFK_CASE(3) RFK_CASE(4) RFK_CASE(5) RFK_CASE(6) RFK_CASE(7) RFK_CASE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef RFK_CASE
  return hipGetLastError();
}

hipError_t launch_normalize(const Prob* probs, const RowItem* items, int nitems, hipStream_t st) {
  hipLaunchKernelGGL((normalize_kernel<ROW_NT>), dim3(nitems), dim3(ROW_NT), 0, st, probs, items,
                     nitems);
  return hipGetLastError();
}

hipError_t launch_ctrl_reset(const Prob* probs, int nprob, int stop_mode, double tol,
                             hipStream_t st) {
  hipLaunchKernelGGL(ctrl_reset_kernel, dim3((nprob + 255) / 256), dim3(256), 0, st, probs, nprob,
                     stop_mode, tol);
  return hipGetLastError();
}

hipError_t launch_set_x(Prob* probs, int p, double* x, int64_t ldx, hipStream_t st) {
  hipLaunchKernelGGL(set_x_kernel, dim3(1), dim3(64), 0, st, probs, p, x, ldx);
  return hipGetLastError();
}

}  // namespace rfk

namespace rfk {
hipError_t kxk_set_attributes() {
  return hipFuncSetAttribute((const void*)kxk_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             16384 * (int)sizeof(double));
}
}  // namespace rfk
