// Rayleigh-Ritz preprocessing for clustered targets (Sec. 3.4, handling
// clustered eigenvalues): on span(X) solve (X^T A X) S = (X^T X) S Theta, set
// X <- X S (then X^T X = I and X^T A X = Theta), and arm the next step to take
// the leading k x k block of E_L as zero, so that no d_j - d_i denominator
// is formed for the clustered pairs.
//
// W = A X comes from the step's own product kernels; the Gram pass with d = 0
// then yields X^T W and X^T X (leading rows and the rest, as in the step).
// One workgroup per problem solves the k x k problem in FP64:
//   G = X^T X = L L^T (Cholesky), C = L^{-1} H L^{-T} with H = sym(X^T W),
//   C = Q Theta Q^T by cyclic Jacobi rotations in parallel rounds (a round
//   rotates k/2 disjoint index pairs of the round-robin schedule, so every
//   pair is visited once per sweep), S = L^{-T} Q with the columns ordered by
//   |theta - mu| descending (ties in ascending theta), each column signed so
//   that z_jj = (X S)_jj <= 0 (the leading block X1 - I of the compact-WY
//   factor then keeps its diagonal at or below -1).
// The tall product X S is formed in place, 16 rows at a time through LDS.
#include "common.h"
#include "dev_util.h"

namespace rfk {

// d = 0 for the Gram pass, which then forms X^T W instead of X^T R.
__global__ void rr_prep_kernel(const Prob* __restrict__ probs, int nprob) {
  for (int p = blockIdx.x; p < nprob; p += gridDim.x) {
    const Prob& P = probs[p];
    for (int j = threadIdx.x; j < P.k; j += blockDim.x) P.vec[VEC_D * P.k + j] = 0.0;
  }
}

constexpr int RR_NT = 256;
constexpr int RR_LD = KMAX + 1;
constexpr int RR_SWEEPS = 40;

__global__ __launch_bounds__(RR_NT) void rr_solve_kernel(const Prob* __restrict__ probs, int nprob) {
  __shared__ double C[KMAX * RR_LD];  // C (stride k + 1), then Q when it fits
  __shared__ double rc[KMAX / 2 + 1], rs[KMAX / 2 + 1];
  __shared__ int ra[KMAX / 2 + 1], rb[KMAX / 2 + 1];
  __shared__ double red[2][RR_NT];
  __shared__ int perm[KMAX];
  __shared__ double gdiag[KMAX];
  __shared__ int fail;
  const int tid = threadIdx.x;
  for (int p = blockIdx.x; p < nprob; p += gridDim.x) {
    const Prob& P = probs[p];
    Ctrl* ctrl = P.ctrl;
    __syncthreads();
    if (ctrl->stopped) continue;
    const int k = P.k, kk2 = k * k;
    // C at stride k + 1; the Jacobi eigenvectors Q and the Cholesky factor L
    // (row-major, lower) follow it in LDS while they fit (Q for k <= 90, L for
    // k <= 74): the triangular solves read L once per multiply-add, and from
    // memory each read would be a round trip
    const int ld = k + 1;
    const bool q_lds = 2 * k * ld <= KMAX * RR_LD, l_lds = 2 * k * ld + kk2 <= KMAX * RR_LD;
    const int qd = q_lds ? ld : k;  // Q's row stride (padded in LDS: no bank conflicts by column)
    double* Q = q_lds ? C + k * ld : P.kk + (KK_S0 + 1) * kk2;
    double* L = l_lds ? C + 2 * k * ld : P.kk + KK_S0 * kk2;
    double* S = P.kk + (KK_S0 + 2) * kk2;  // result
    const double* PT = P.kk + KK_PT * kk2;
    const double* P2 = P.kk + KK_P2 * kk2;
    const double* GT = P.kk + KK_GT * kk2;
    const double* G2 = P.kk + KK_G2 * kk2;
    if (tid == 0) fail = 0;
    // G = X^T X (the leading-row part holds only the tiles on or above the
    // diagonal of 16 x 16 tiles; the rest is mirrored)
    for (int e = tid; e < kk2; e += RR_NT) {
      const int i = e / k, j = e - i * k;
      const double gt = (i / 16 <= j / 16) ? GT[i * k + j] : GT[j * k + i];
      C[i * ld + j] = gt + G2[i * k + j];
      if (i == j) gdiag[i] = gt + G2[i * k + j];
    }
    __syncthreads();
    // Cholesky in place (right-looking, lower); a pivot below 64 k u of its
    // column's norm means numerically dependent columns
    for (int c = 0; c < k; ++c) {
      if (tid == 0) {
        const double v = C[c * ld + c];
        if (!(v > 64.0 * k * UNIT_ROUNDOFF * gdiag[c]) || !__builtin_isfinite(v)) fail = 1;
        C[c * ld + c] = sqrt(fmax(v, 0.0));
      }
      __syncthreads();
      if (fail) break;
      const double piv = C[c * ld + c];
      for (int r = c + 1 + tid; r < k; r += RR_NT) C[r * ld + c] /= piv;
      __syncthreads();
      const int m = k - c - 1;
      const float invm = 1.0f / (float)max(m, 1);
      for (int e = tid; e < m * m; e += RR_NT) {
        const int qe = __float2int_rz((e + 0.5f) * invm);
        const int r = c + 1 + qe, j = c + 1 + (e - qe * m);
        if (j <= r) C[r * ld + j] -= C[r * ld + c] * C[j * ld + c];
      }
      __syncthreads();
    }
    if (fail) {
      if (tid == 0) {
        ctrl->status = -7;
        ctrl->stopped = 1;
      }
      continue;
    }
    for (int e = tid; e < kk2; e += RR_NT) {
      const int i = e / k, j = e - i * k;
      L[e] = j <= i ? C[i * ld + j] : 0.0;
    }
    __syncthreads();
    // H = sym(X^T W) into C
    for (int e = tid; e < kk2; e += RR_NT) {
      const int i = e / k, j = e - i * k;
      const double hij = PT[i * k + j] + P2[i * k + j], hji = PT[j * k + i] + P2[j * k + i];
      C[i * ld + j] = 0.5 * (hij + hji);
    }
    __syncthreads();
    // B = L^{-1} H, one column per thread (forward substitution)
    for (int c = tid; c < k; c += RR_NT) {
      for (int r = 0; r < k; ++r) {
        double b = C[r * ld + c];
        for (int l = 0; l < r; ++l) b -= L[r * k + l] * C[l * ld + c];
        C[r * ld + c] = b / L[r * k + r];
      }
    }
    __syncthreads();
    // C = B L^{-T}, one row per thread
    for (int r = tid; r < k; r += RR_NT) {
      for (int j = 0; j < k; ++j) {
        double v = C[r * ld + j];
        for (int l = 0; l < j; ++l) v -= C[r * ld + l] * L[j * k + l];
        C[r * ld + j] = v / L[j * k + j];
      }
    }
    __syncthreads();
    for (int e = tid; e < kk2; e += RR_NT) {
      const int i = e / k, j = e - i * k;
      if (i < j) {
        const double v = 0.5 * (C[i * ld + j] + C[j * ld + i]);
        C[i * ld + j] = v;
        C[j * ld + i] = v;
      }
      Q[i * qd + j] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();
    // cyclic Jacobi in parallel rounds (element index / k by a float
    // reciprocal: exact for indices below 2^13)
    const float invk = 1.0f / (float)k;
    const int m = k + (k & 1), npair = m / 2;
    for (int sweep = 0; sweep < RR_SWEEPS; ++sweep) {
      double off = 0.0, dia = 0.0;
      for (int e = tid; e < kk2; e += RR_NT) {
        const int i = e / k, j = e - i * k;
        const double v = C[i * ld + j];
        if (i == j)
          dia += v * v;
        else
          off += v * v;
      }
      red[0][tid] = off;
      red[1][tid] = dia;
      __syncthreads();
      for (int h = RR_NT / 2; h >= 1; h /= 2) {
        if (tid < h) {
          red[0][tid] += red[0][tid + h];
          red[1][tid] += red[1][tid + h];
        }
        __syncthreads();
      }
      // converged once the off-diagonal mass is at the rounding floor: every
      // rotation leaves entries of about u ||C||, so off^2 settles near
      // k u^2 dia^2 and further sweeps change nothing (a fixed 1e-32 sat below
      // that floor and always ran every sweep)
      const bool done = !(red[0][0] > 16.0 * k * UNIT_ROUNDOFF * UNIT_ROUNDOFF * red[1][0]);
      __syncthreads();
      if (done) break;
      for (int r = 0; r < m - 1; ++r) {
        if (tid < npair) {
          auto at = [&](int i) { return i == 0 ? 0 : ((i - 1 + r) % (m - 1)) + 1; };
          int a = at(tid), b = at(m - 1 - tid);
          if (a > b) {
            const int t = a;
            a = b;
            b = t;
          }
          double c = 1.0, s = 0.0;
          const bool valid = b < k;
          if (valid) {
            const double apq = C[a * ld + b];
            if (apq != 0.0) {
              const double th = (C[b * ld + b] - C[a * ld + a]) / (2.0 * apq);
              const double t = fabs(th) > 1e150 ? 0.5 / th
                                                : (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
              c = 1.0 / sqrt(1.0 + t * t);
              s = t * c;
            }
          }
          ra[tid] = valid ? a : -1;
          rb[tid] = b;
          rc[tid] = c;
          rs[tid] = s;
        }
        __syncthreads();
        // rows a, b of C: C <- J^T C
        for (int e = tid; e < npair * k; e += RR_NT) {
          const int q = __float2int_rz((e + 0.5f) * invk), j = e - q * k, a = ra[q];
          if (a >= 0) {
            const int b = rb[q];
            const double c = rc[q], s = rs[q];
            const double x = C[a * ld + j], y = C[b * ld + j];
            C[a * ld + j] = c * x - s * y;
            C[b * ld + j] = s * x + c * y;
          }
        }
        __syncthreads();
        // columns a, b of C and of Q: C <- C J, Q <- Q J
        for (int e = tid; e < npair * k; e += RR_NT) {
          const int q = __float2int_rz((e + 0.5f) * invk), j = e - q * k, a = ra[q];
          if (a >= 0) {
            const int b = rb[q];
            const double c = rc[q], s = rs[q];
            const double x = C[j * ld + a], y = C[j * ld + b];
            C[j * ld + a] = c * x - s * y;
            C[j * ld + b] = s * x + c * y;
            const double u = Q[j * qd + a], v = Q[j * qd + b];
            Q[j * qd + a] = c * u - s * v;
            Q[j * qd + b] = s * u + c * v;
          }
        }
        __syncthreads();
      }
    }
    // order: |theta - mu| descending, ties in ascending theta, then index
    for (int j = tid; j < k; j += RR_NT) {
      const double tj = C[j * ld + j], kj = fabs(tj - P.mu);
      int rank = 0;
      for (int i = 0; i < k; ++i) {
        const double ti = C[i * ld + i], ki = fabs(ti - P.mu);
        if (ki > kj || (ki == kj && (ti < tj || (ti == tj && i < j)))) ++rank;
      }
      perm[rank] = j;
    }
    __syncthreads();
    // the Ritz values, before C's storage takes S (when L is in LDS)
    for (int j = tid; j < k; j += RR_NT) gdiag[j] = C[j * ld + j];
    __syncthreads();
    double* Sw = l_lds ? C : S;  // S is formed in LDS and written out once
    // S = L^{-T} Q(:, perm), one column per thread (back substitution), then
    // the sign that makes z_cc = (X S)_cc <= 0; the Ritz values go to d
    for (int c = tid; c < k; c += RR_NT) {
      const int src = perm[c];
      for (int r = k - 1; r >= 0; --r) {
        double v = Q[r * qd + src];
        for (int l = r + 1; l < k; ++l) v -= L[l * k + r] * Sw[l * k + c];
        Sw[r * k + c] = v / L[r * k + r];
      }
      double z = 0.0;
      for (int l = 0; l < k; ++l) z += P.x[(int64_t)c * P.ldx + l] * Sw[l * k + c];
      if (z > 0.0)
        for (int l = 0; l < k; ++l) Sw[l * k + c] = -Sw[l * k + c];
      P.vec[VEC_D * k + c] = gdiag[src];
    }
    __syncthreads();
    if (l_lds)
      for (int e = tid; e < kk2; e += RR_NT) S[e] = Sw[e];
    __syncthreads();
    if (tid == 0) ctrl->rr_top = 1;
  }
}

// X <- X S in place, 16 rows at a time: a chunk's rows are copied to LDS
// before any of them is overwritten, and the next chunk's rows are requested
// (into registers) before the current chunk is multiplied, so the block waits
// on memory once per chunk rather than twice.  S sits in LDS for k <= 64
// (read from L2 otherwise); for k <= 32 each thread keeps its column of S in
// registers, so the product reads LDS once per multiply-add, by broadcast.
constexpr int RA_ROWS = 16;
constexpr int RA_SMAX = 64;
__global__ __launch_bounds__(256) void rr_apply_kernel(const Prob* __restrict__ probs,
                                                      const RowItem* __restrict__ items, int nitems) {
  constexpr int NT = 256, PF = RA_ROWS * KMAX / NT;
  __shared__ double xs[2][RA_ROWS * KMAX];
  __shared__ double ss[RA_SMAX * RA_SMAX];
  const int tid = threadIdx.x;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem item = items[it];
    const Prob& P = probs[item.prob];
    __syncthreads();  // the previous item's reads of xs and ss are done
    if (P.ctrl->stopped) continue;
    const int n = P.n, k = P.k, kk2 = k * k, rk = RA_ROWS * k;
    const double* S = P.kk + (KK_S0 + 2) * kk2;
    const bool s_lds = k <= RA_SMAX;
    if (s_lds)
      for (int e = tid; e < kk2; e += NT) ss[e] = *gld(S + e);
    const double* Sv = s_lds ? ss : S;
    // k <= 32: this thread's column of S (tid % 32) in registers
    double scol[32];
    {
      const int c = tid % 32;
#pragma unroll
      for (int l = 0; l < 32; ++l) scol[l] = (l < k && c < k) ? *gld(S + l * k + c) : 0.0;
    }
    double* X = P.x;
    const int64_t ldx = P.ldx;
    const int r0 = item.blk * P.rbrows, r1 = min(n, r0 + P.rbrows);
    double pf[PF];
    auto fetch = [&](int rb) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int e = tid + u * NT;
        const int r = e / k, j = e - r * k;
        pf[u] = (e < rk && rb + r < r1) ? *gld(X + (int64_t)(rb + r) * ldx + j) : 0.0;
      }
    };
    fetch(r0);
    int b = 0;
    for (int rb = r0; rb < r1; rb += RA_ROWS) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int e = tid + u * NT;
        if (e < rk) xs[b][e] = pf[u];
      }
      __syncthreads();
      if (rb + RA_ROWS < r1) fetch(rb + RA_ROWS);
      if (k <= 32) {
        // lane c of a 32-lane row slot owns column c with S(:, c) in
        // registers; the slot's rows r and r + 8 come from LDS by broadcast
        const int c = tid % 32, r = tid / 32;
        if (c < k) {
          double v0 = 0.0, v1 = 0.0;
#pragma unroll
          for (int l = 0; l < 32; ++l) {
            if (l < k) {
              v0 = __builtin_fma(xs[b][r * k + l], scol[l], v0);
              v1 = __builtin_fma(xs[b][(r + 8) * k + l], scol[l], v1);
            }
          }
          if (rb + r < r1) X[(int64_t)(rb + r) * ldx + c] = v0;
          if (rb + r + 8 < r1) X[(int64_t)(rb + r + 8) * ldx + c] = v1;
        }
      } else {
        for (int e = tid; e < rk; e += NT) {
          const int r = e / k, c = e - r * k;
          if (rb + r < r1) {
            double v = 0.0;
            for (int l = 0; l < k; ++l) v = __builtin_fma(xs[b][r * k + l], Sv[l * k + c], v);
            X[(int64_t)(rb + r) * ldx + c] = v;
          }
        }
      }
      b ^= 1;
    }
  }
}

hipError_t launch_rr_prep(const Prob* probs, int nprob, hipStream_t st) {
  hipLaunchKernelGGL(rr_prep_kernel, dim3(nprob), dim3(128), 0, st, probs, nprob);
  return hipGetLastError();
}

hipError_t launch_rr_solve(const Prob* probs, int nprob, hipStream_t st) {
  hipLaunchKernelGGL(rr_solve_kernel, dim3(nprob), dim3(RR_NT), 0, st, probs, nprob);
  return hipGetLastError();
}

hipError_t launch_rr_apply(const Prob* probs, const RowItem* items, int nitems, hipStream_t st) {
  hipLaunchKernelGGL(rr_apply_kernel, dim3(nitems), dim3(256), 0, st, probs, items, nitems);
  return hipGetLastError();
}

}  // namespace rfk
