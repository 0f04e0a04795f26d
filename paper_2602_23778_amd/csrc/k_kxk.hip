// The k-by-k part of one refinement step (one workgroup per problem).
//
// Inputs (from the Gram pass): X2^T R2, X2^T X2, X1^T R1, X1^T X1, R1, and the
// Rayleigh quotients d, alpha = diag(X^T X).  With Y1 = X1 - I_k:
//   * Algorithm 1: T = -Y1^{-T}.  Z = Y1^{-1} is obtained by Newton-Schulz
//     iteration Z <- Z + Z (I - Y1 Z), started from the previous step's Z
//     (X1 moves by about the eigenvector error per step, so one or two
//     products suffice) or from Z = -I (valid while ||X1|| < 1, which holds
//     for the O(1/sqrt(n)) leading rows of a subspace basis).  When neither
//     start converges, Gauss-Jordan elimination with partial pivoting
//     computes Z instead.  Both yield Y1^{-1} up to rounding; the 1-norm
//     condition number of Y1 decides singularity (cond > 1/(n u)).
//   * C = Y^T R = X^T R - R1 and M = T^T C = -Z C, so that the bottom rows of
//     V = H^T R are V2 = R2 - X2 M (line 5 of Algorithm 4; the top rows of V
//     are X^T R).
//   * E11 per line 6 of Algorithm 4 (eqs. Ediag, Eoffdiag; beta for
//     |d_j - d_i| <= delta).
//   * F = Y^T E_L = X1^T E11 + (X2^T R2 - X2^T X2 M) diag(1/(d - mu)) - E11,
//     using E21 = V2 diag(1/(d - mu)) without forming it, and N = T F = -Z^T F.
//   * The new leading rows X1 + E11 - Y1 N (line 7).
// [M | N] and the new leading rows go to the workspace for the update pass.
//
// All k-by-k products run on the FP64 matrix cores, 16x16 tiles dealt to the
// wavefronts.  For k <= 64 the four working matrices live in LDS (128 KiB);
// beyond that in a global scratch area that stays in L2.
#include "common.h"
#include "dev_util.h"

namespace rfk {

constexpr int KXK_NT = 512;
constexpr int KXK_NW = KXK_NT / 64;

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o >= 1; o /= 2) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < KXK_NW; ++w) s += red[w];
  return s;
}

__device__ __forceinline__ double block_max(double v, double* red) {
  for (int o = 32; o >= 1; o /= 2) v = fmax(v, __shfl_xor(v, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < KXK_NW; ++w) s = fmax(s, red[w]);
  return s;
}

// out(i, j) = sum_{l < k} a(i, l) b(l, j) for i, j < k, with k <= 4*KQ.  Each
// wavefront takes 16x16 output tiles in turn; for a tile, all its operand
// values along K are loaded first (one round trip to LDS or L2), then the
// k/4 MFMAs run on two accumulators.
template <int KQ, class FA, class FB, class FS>
__device__ __forceinline__ void kk_mm(int k, FA a, FB b, FS store) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  const int nt = (k + 15) / 16;
  const int kq = (k + 3) / 4;
  for (int t = wave; t < nt * nt; t += KXK_NW) {
    const int ti = t / nt, tj = t - ti * nt;
    const int i = ti * 16 + r16, j = tj * 16 + r16;
    const bool iok = i < k, jok = j < k;
    double av[KQ], bv[KQ];
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      const int l = 4 * q + g;
      const bool lok = q < kq && l < k;
      av[q] = (iok && lok) ? a(i, l) : 0.0;
      bv[q] = (jok && lok) ? b(l, j) : 0.0;
    }
    v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < KQ; q += 2) {
      if (q < kq) acc0 = mfma_f64(av[q], bv[q], acc0);
      if (q + 1 < kq) acc1 = mfma_f64(av[q + 1], bv[q + 1], acc1);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = ti * 16 + mfma_row(g, r);
      if (row < k && jok) store(row, j, acc0[r] + acc1[r]);
    }
  }
}

// In-place inverse of the k x k matrix in Yi by Gauss-Jordan elimination with
// partial pivoting.  Returns false when a pivot is exactly zero.
__device__ bool gauss_jordan_inverse(double* Yi, int k, int* piv, double* fcol, int* sflag) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kk2 = k * k;
  if (tid == 0) *sflag = 0;
  __syncthreads();
  for (int c = 0; c < k; ++c) {
    if (wave == 0) {
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
        if (lane == 0) *sflag = 1;
      } else {
        if (lane == 0) piv[c] = bi;
        if (bi != c)
          for (int j = lane; j < k; j += 64) {
            const double t = Yi[c * k + j];
            Yi[c * k + j] = Yi[bi * k + j];
            Yi[bi * k + j] = t;
          }
        const double ipv = 1.0 / Yi[c * k + c];
        for (int j = lane; j < k; j += 64) Yi[c * k + j] = (j == c ? 1.0 : Yi[c * k + j]) * ipv;
        for (int r = lane; r < k; r += 64) fcol[r] = (r == c) ? 0.0 : Yi[r * k + c];
      }
    }
    __syncthreads();
    if (*sflag) return false;
    for (int e = tid; e < kk2; e += KXK_NT) {
      const int r = e / k, j = e - r * k;
      if (r != c) {
        const double y = (j == c) ? 0.0 : Yi[e];
        Yi[e] = y - fcol[r] * Yi[c * k + j];
      }
    }
    __syncthreads();
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
  return true;
}

template <bool LDS>
__global__ __launch_bounds__(KXK_NT) void kxk_kernel(const Prob* __restrict__ probs, int nprob) {
  constexpr int KQ = LDS ? 16 : 32;  // k <= 64 in LDS, k <= 128 otherwise
  extern __shared__ double smem[];
  __shared__ double red[KXK_NW];
  __shared__ int piv[KMAX];
  __shared__ double fcol[KMAX];
  __shared__ int sflag;
  const int tid = threadIdx.x;
  for (int p = blockIdx.x; p < nprob; p += gridDim.x) {
    const Prob& P = probs[p];
    Ctrl* ctrl = P.ctrl;
    __syncthreads();
    if (tid == 0) ctrl->apply = 0;
    if (ctrl->stopped) continue;
    const int n = P.n, k = P.k, kk2 = k * k;
    const int64_t ldx = P.ldx;
    const double* __restrict__ X = P.x;
    double* S = LDS ? smem : P.kk + KK_S0 * kk2;
    double* X1 = S;
    double* Zb = S + kk2;
    double* Eb = S + 2 * kk2;
    double* Fb = S + 3 * kk2;
    double* Zg = P.kk + KK_Z * kk2;
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
    const double tol_ns = 16.0 * k * UNIT_ROUNDOFF;

    double sx = 0.0;
    for (int e = tid; e < kk2; e += KXK_NT) {
      const int i = e / k, j = e - i * k;
      const double x = X[(int64_t)i * ldx + j];
      X1[e] = x;
      Zb[e] = Zg[e];
      sx = __builtin_fma(x, x, sx);
    }
    const double nx1 = sqrt(block_sum(sx, red));
    auto y1 = [&](int i, int l) { return X1[i * k + l] - (i == l ? 1.0 : 0.0); };

    // ---- Z = Y1^{-1}: Newton-Schulz with warm start, else Gauss-Jordan ----
    double* Z = Zb;
    double* Zt = Fb;
    double es = 0.0;
    kk_mm<KQ>(
        k, y1, [&](int l, int j) { return Z[l * k + j]; },
        [&](int i, int j, double v) {
          const double e = (i == j ? 1.0 : 0.0) - v;
          Eb[i * k + j] = e;
          es = __builtin_fma(e, e, es);
        });
    double eres = sqrt(block_sum(es, red));
    bool ok = false;
    bool try_ns = true;
    // Newton-Schulz contracts in the Frobenius norm once ||I - Y1 Z||_F < 1.
    if (!(eres < 0.9)) {
      if (nx1 < 0.9) {
        // Z = -I, hence I - Y1 Z = I + Y1 = X1
        for (int e = tid; e < kk2; e += KXK_NT) {
          const int i = e / k, j = e - i * k;
          Z[e] = (i == j) ? -1.0 : 0.0;
          Eb[e] = X1[e];
        }
        eres = nx1;
        __syncthreads();
      } else {
        try_ns = false;
      }
    }
    if (try_ns) {
      for (int it = 0; it < 16; ++it) {
        if (eres <= tol_ns) {
          ok = true;
          break;
        }
        if (!(eres < 0.9)) break;
        kk_mm<KQ>(
            k, [&](int i, int l) { return Z[i * k + l]; },
            [&](int l, int j) { return Eb[l * k + j]; },
            [&](int i, int j, double v) { Zt[i * k + j] = Z[i * k + j] + v; });
        __syncthreads();
        double* sw = Z;
        Z = Zt;
        Zt = sw;
        if (eres * eres <= 0.25 * tol_ns) {
          // the residual after this update is at most eres^2
          ok = true;
          break;
        }
        es = 0.0;
        kk_mm<KQ>(
            k, y1, [&](int l, int j) { return Z[l * k + j]; },
            [&](int i, int j, double v) {
              const double e = (i == j ? 1.0 : 0.0) - v;
              Eb[i * k + j] = e;
              es = __builtin_fma(e, e, es);
            });
        eres = sqrt(block_sum(es, red));
      }
    }
    if (!ok) {
      Z = Zb;
      for (int e = tid; e < kk2; e += KXK_NT) {
        const int i = e / k, j = e - i * k;
        Z[e] = X1[e] - (i == j ? 1.0 : 0.0);
      }
      __syncthreads();
      ok = gauss_jordan_inverse(Z, k, piv, fcol, &sflag);
    }
    // Y1 and Z = Y1^{-1} column sums: cond_1(Y1) = ||Y1||_1 ||Z||_1
    double cy = 0.0, cz = 0.0;
    if (ok && tid < k)
      for (int i = 0; i < k; ++i) {
        cy += fabs(y1(i, tid));
        cz += fabs(Z[i * k + tid]);
      }
    const double ny = block_max(cy, red);
    const double nz = block_max(cz, red);
    const double cond = ny * nz;
    const bool bad_in = __syncthreads_or(
        tid < k && (!__builtin_isfinite(d[tid]) || !__builtin_isfinite(alpha[tid])));
    if (!ok || bad_in || !(cond <= 1.0 / ((double)n * UNIT_ROUNDOFF))) {
      __syncthreads();
      if (tid == 0) {
        ctrl->status = bad_in ? -6 : -4;
        ctrl->stopped = 1;
      }
      continue;
    }
    for (int e = tid; e < kk2; e += KXK_NT) Zg[e] = Z[e];  // warm start of the next step

    // ---- M = T^T C = -Z C with C = X^T R - R1 ----
    kk_mm<KQ>(
        k, [&](int i, int l) { return Z[i * k + l]; },
        [&](int l, int j) { return (PT[l * k + j] + P2[l * k + j]) - R1[l * k + j]; },
        [&](int i, int j, double v) { Cm[i * 2 * k + j] = -v; });
    // ---- E11 (line 6 of Algorithm 4) into the E buffer ----
    // free buffers: Eb, and whichever of Zb / Fb does not hold Z
    double* E1 = Eb;
    double* Fm = (Z == Fb) ? Zb : Fb;
    double e1sq = 0.0;
    const double delta = P.delta;
    for (int e = tid; e < kk2; e += KXK_NT) {
      const int i = e / k, j = e - i * k;
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
    e1sq = block_sum(e1sq, red);
    // ---- F = X1^T E11 + (X2^T R2 - X2^T X2 M) diag(1/(d - mu)) - E11 ----
    kk_mm<KQ>(
        k, [&](int i, int l) { return X1[l * k + i]; }, [&](int l, int j) { return E1[l * k + j]; },
        [&](int i, int j, double v) { Fm[i * k + j] = v; });
    kk_mm<KQ>(
        k, [&](int i, int l) { return G2[i * k + l]; },
        [&](int l, int j) { return Cm[l * 2 * k + j]; },
        [&](int i, int j, double v) {
          Fm[i * k + j] = Fm[i * k + j] + (P2[i * k + j] - v) * dinv[j] - E1[i * k + j];
        });
    __syncthreads();
    // ---- N = T F = -Z^T F into the right half of Cm ----
    kk_mm<KQ>(
        k, [&](int i, int l) { return Z[l * k + i]; }, [&](int l, int j) { return Fm[l * k + j]; },
        [&](int i, int j, double v) { Cm[i * 2 * k + k + j] = -v; });
    __syncthreads();
    // ---- leading rows of the update: X1 + E11 - Y1 N ----
    kk_mm<KQ>(
        k, y1, [&](int l, int j) { return Cm[l * 2 * k + k + j]; },
        [&](int i, int j, double v) { X1n[i * k + j] = X1[i * k + j] + E1[i * k + j] - v; });
    if (tid == 0) P.vec[VEC_E1SQ * k] = e1sq;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// k <= 64: everything in LDS, one workgroup of four wavefronts per problem.
// Every phase first issues all of its loads (compile-time bounded, unrolled)
// and then computes, so each phase costs one memory round trip.  Four k x k
// LDS buffers suffice: B0 = X1; B1 = Z (and later N); B2 = the Newton-Schulz
// residual, then C, then E11; B3 = the Newton-Schulz temporary, then M, then F.
// F and N are held in registers (tile slots) until every wavefront has read
// the buffer they replace.
// ---------------------------------------------------------------------------
constexpr int KS_NT = 512;
constexpr int KS_NW = KS_NT / 64;
constexpr int KS_K = 64;
constexpr int KS_EPT = KS_K * KS_K / KS_NT;  // elements per thread of a k x k sweep
constexpr int KS_SLOTS = (KS_K / 16) * (KS_K / 16) / KS_NW;  // 16x16 tiles per wavefront

__device__ __forceinline__ double ks_sum(double v, double* red) {
  for (int o = 32; o >= 1; o /= 2) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < KS_NW; ++w) t += red[w];
  return t;
}

// res[slot] += sum_l a(i, l) b(l, j) for the wavefront's tiles (slot s is
// tile wave + s*KS_NW of the row-major tile grid).
template <class FA, class FB>
__device__ __forceinline__ void ks_mm(int k, FA a, FB b, v4d (&res)[KS_SLOTS]) {
  constexpr int QC = 8;  // K steps of 4 loaded per round trip
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  const int nt = (k + 15) / 16, kq = (k + 3) / 4;
#pragma unroll
  for (int sl = 0; sl < KS_SLOTS; ++sl) {
    const int t = wave + sl * KS_NW;
    if (t < nt * nt) {
      const int ti = t / nt, tj = t - ti * nt;
      const int i = ti * 16 + r16, j = tj * 16 + r16;
      const bool iok = i < k, jok = j < k;
      v4d acc1 = {0.0, 0.0, 0.0, 0.0};
      for (int q0 = 0; q0 < kq; q0 += QC) {
        double av[QC], bv[QC];
#pragma unroll
        for (int q = 0; q < QC; ++q) {
          const int l = 4 * (q0 + q) + g;
          const bool lok = q0 + q < kq && l < k;
          av[q] = (iok && lok) ? a(i, l) : 0.0;
          bv[q] = (jok && lok) ? b(l, j) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < QC; q += 2) {
          res[sl] = mfma_f64(av[q], bv[q], res[sl]);
          acc1 = mfma_f64(av[q + 1], bv[q + 1], acc1);
        }
      }
      res[sl] += acc1;
    }
  }
}

// store(i, j, res value) for the wavefront's tiles.
template <class FS>
__device__ __forceinline__ void ks_store(int k, const v4d (&res)[KS_SLOTS], FS store) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  const int nt = (k + 15) / 16;
#pragma unroll
  for (int sl = 0; sl < KS_SLOTS; ++sl) {
    const int t = wave + sl * KS_NW;
    if (t < nt * nt) {
      const int ti = t / nt, tj = t - ti * nt;
      const int j = tj * 16 + r16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = ti * 16 + mfma_row(g, r);
        if (row < k && j < k) store(row, j, res[sl][r]);
      }
    }
  }
}

__device__ __forceinline__ void ks_zero(v4d (&res)[KS_SLOTS]) {
#pragma unroll
  for (int sl = 0; sl < KS_SLOTS; ++sl) res[sl] = v4d{0.0, 0.0, 0.0, 0.0};
}

__global__ __launch_bounds__(KS_NT) void kxk_small_kernel(const Prob* __restrict__ probs, int nprob) {
  __shared__ double B0[KS_K * KS_K], B1[KS_K * KS_K], B2[KS_K * KS_K], B3[KS_K * KS_K];
  __shared__ double red[KS_NW];
  __shared__ int piv[KS_K];
  __shared__ double fcol[KS_K];
  __shared__ int sflag;
  const int tid = threadIdx.x;
  for (int p = blockIdx.x; p < nprob; p += gridDim.x) {
    const Prob& P = probs[p];
    Ctrl* ctrl = P.ctrl;
    __syncthreads();
    if (tid == 0) ctrl->apply = 0;
    if (ctrl->stopped) continue;
    const int n = P.n, k = P.k, kk2 = k * k;
    const int64_t ldx = P.ldx;
    const double* __restrict__ X = P.x;
    double* Zg = P.kk + KK_Z * kk2;
    const double* PT = P.kk + KK_PT * kk2;
    const double* P2 = P.kk + KK_P2 * kk2;
    const double* GT = P.kk + KK_GT * kk2;
    const double* G2 = P.kk + KK_G2 * kk2;
    const double* R1 = P.kk + KK_R1 * kk2;
    double* Cm = P.kk + KK_CM * kk2;
    double* X1n = P.kk + KK_X1N * kk2;
    const double* d = P.vec + VEC_D * k;
    const double* alpha = P.vec + VEC_ALPHA * k;
    const double* dinv = P.vec + VEC_DINV * k;
    const double tol_ns = 16.0 * k * UNIT_ROUNDOFF;
    auto y1 = [&](int i, int l) { return B0[i * k + l] - (i == l ? 1.0 : 0.0); };

    // X1 -> B0, previous Z -> B1
    double sx = 0.0;
    {
      double xv[KS_EPT], zv[KS_EPT];
#pragma unroll
      for (int q = 0; q < KS_EPT; ++q) {
        const int e = tid + q * KS_NT;
        const int i = e / k, j = e - i * k;
        xv[q] = e < kk2 ? X[(int64_t)i * ldx + j] : 0.0;
        zv[q] = e < kk2 ? Zg[e] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < KS_EPT; ++q) {
        const int e = tid + q * KS_NT;
        if (e < kk2) {
          B0[e] = xv[q];
          B1[e] = zv[q];
        }
        sx = __builtin_fma(xv[q], xv[q], sx);
      }
    }
    const double nx1 = sqrt(ks_sum(sx, red));

    // ---- Z = Y1^{-1} by Newton-Schulz (warm start or Z = -I), else Gauss-Jordan
    v4d res[KS_SLOTS];
    auto residual_into_B2 = [&]() {
      ks_zero(res);
      ks_mm(k, y1, [&](int l, int j) { return B1[l * k + j]; }, res);
      double es = 0.0;
      ks_store(k, res, [&](int i, int j, double v) {
        const double e = (i == j ? 1.0 : 0.0) - v;
        B2[i * k + j] = e;
        es = __builtin_fma(e, e, es);
      });
      return sqrt(ks_sum(es, red));
    };
    double eres = residual_into_B2();
    bool ok = false, try_ns = true;
    if (!(eres < 0.9)) {
      if (nx1 < 0.9) {
#pragma unroll
        for (int q = 0; q < KS_EPT; ++q) {
          const int e = tid + q * KS_NT;
          if (e < kk2) {
            const int i = e / k, j = e - i * k;
            B1[e] = (i == j) ? -1.0 : 0.0;
            B2[e] = B0[e];
          }
        }
        eres = nx1;
        __syncthreads();
      } else {
        try_ns = false;
      }
    }
    if (try_ns) {
      for (int it = 0; it < 16; ++it) {
        if (eres <= tol_ns) {
          ok = true;
          break;
        }
        if (!(eres < 0.9)) break;
        // Z <- Z + Z E, through registers
        ks_zero(res);
        ks_mm(k, [&](int i, int l) { return B1[i * k + l]; }, [&](int l, int j) { return B2[l * k + j]; },
              res);
        __syncthreads();
        ks_store(k, res, [&](int i, int j, double v) { B1[i * k + j] += v; });
        __syncthreads();
        if (eres * eres <= 0.25 * tol_ns) {
          ok = true;
          break;
        }
        eres = residual_into_B2();
      }
    }
    if (!ok) {
#pragma unroll
      for (int q = 0; q < KS_EPT; ++q) {
        const int e = tid + q * KS_NT;
        if (e < kk2) {
          const int i = e / k, j = e - i * k;
          B1[e] = B0[e] - (i == j ? 1.0 : 0.0);
        }
      }
      __syncthreads();
      ok = gauss_jordan_inverse(B1, k, piv, fcol, &sflag);
    }
    // cond_1(Y1) = ||Y1||_1 ||Z||_1: eight threads per column
    double cy = 0.0, cz = 0.0;
    {
      const int col = tid >> 3, part = tid & 7;
      if (ok && col < k) {
        for (int i = part; i < k; i += 8) {
          cy += fabs(y1(i, col));
          cz += fabs(B1[i * k + col]);
        }
      }
      for (int o = 1; o < 8; o *= 2) {
        cy += __shfl_xor(cy, o);
        cz += __shfl_xor(cz, o);
      }
      for (int o = 8; o < 64; o *= 2) {
        cy = fmax(cy, __shfl_xor(cy, o));
        cz = fmax(cz, __shfl_xor(cz, o));
      }
    }
    __syncthreads();
    if ((tid & 63) == 0) {
      red[tid >> 6] = cy;
    }
    __syncthreads();
    double ny = 0.0;
    for (int w = 0; w < KS_NW; ++w) ny = fmax(ny, red[w]);
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = cz;
    __syncthreads();
    double nz = 0.0;
    for (int w = 0; w < KS_NW; ++w) nz = fmax(nz, red[w]);
    const double cond = ny * nz;
    const bool bad_in = __syncthreads_or(
        tid < k && (!__builtin_isfinite(d[tid]) || !__builtin_isfinite(alpha[tid])));
    if (!ok || bad_in || !(cond <= 1.0 / ((double)n * UNIT_ROUNDOFF))) {
      if (tid == 0) {
        ctrl->status = bad_in ? -6 : -4;
        ctrl->stopped = 1;
      }
      continue;
    }

    // Z -> global (warm start); C = X^T R - R1 -> B2
    {
      double cv[KS_EPT];
#pragma unroll
      for (int q = 0; q < KS_EPT; ++q) {
        const int e = tid + q * KS_NT;
        cv[q] = e < kk2 ? (PT[e] + P2[e]) - R1[e] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < KS_EPT; ++q) {
        const int e = tid + q * KS_NT;
        if (e < kk2) {
          B2[e] = cv[q];
          Zg[e] = B1[e];
        }
      }
    }
    __syncthreads();
    // M = T^T C = -Z C -> B3 and Cm[:, :k]
    ks_zero(res);
    ks_mm(k, [&](int i, int l) { return B1[i * k + l]; }, [&](int l, int j) { return B2[l * k + j]; }, res);
    ks_store(k, res, [&](int i, int j, double v) {
      B3[i * k + j] = -v;
      Cm[i * 2 * k + j] = -v;
    });
    __syncthreads();
    // E11 (line 6 of Algorithm 4) -> B2
    double e1sq = 0.0;
    {
      double pv[KS_EPT], gv[KS_EPT];
      const double delta = P.delta;
#pragma unroll
      for (int q = 0; q < KS_EPT; ++q) {
        const int e = tid + q * KS_NT;
        pv[q] = e < kk2 ? PT[e] + P2[e] : 0.0;
        gv[q] = (e < kk2 && !P.beta_zero) ? GT[e] + G2[e] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < KS_EPT; ++q) {
        const int e = tid + q * KS_NT;
        if (e < kk2) {
          const int i = e / k, j = e - i * k;
          double v;
          if (i == j)
            v = (1.0 - alpha[i]) * 0.5;
          else if (fabs(d[j] - d[i]) <= delta)
            v = P.beta_zero ? 0.0 : -gv[q] * 0.5;
          else
            v = pv[q] / (d[j] - d[i]);
          B2[e] = v;
          e1sq = __builtin_fma(v, v, e1sq);
        }
      }
    }
    e1sq = ks_sum(e1sq, red);
    // F = X1^T E11 + (X2^T R2 - X2^T X2 M) diag(1/(d - mu)) - E11 -> B3 (replacing M)
    ks_zero(res);
    ks_mm(k, [&](int i, int l) { return G2[i * k + l]; }, [&](int l, int j) { return B3[l * k + j]; },
          res);
    {
      const int lane = tid & 63, wave = tid >> 6, g = lane >> 4, r16 = lane & 15;
      const int nt = (k + 15) / 16;
#pragma unroll
      for (int sl = 0; sl < KS_SLOTS; ++sl) {
        const int t = wave + sl * KS_NW;
        if (t < nt * nt) {
          const int ti = t / nt, tj = t - ti * nt;
          const int j = tj * 16 + r16;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = ti * 16 + mfma_row(g, r);
            if (row < k && j < k)
              res[sl][r] = (P2[row * k + j] - res[sl][r]) * dinv[j] - B2[row * k + j];
          }
        }
      }
    }
    ks_mm(k, [&](int i, int l) { return B0[l * k + i]; }, [&](int l, int j) { return B2[l * k + j]; }, res);
    __syncthreads();
    ks_store(k, res, [&](int i, int j, double v) { B3[i * k + j] = v; });
    __syncthreads();
    // N = T F = -Z^T F -> Cm[:, k:] and B1 (replacing Z)
    ks_zero(res);
    ks_mm(k, [&](int i, int l) { return B1[l * k + i]; }, [&](int l, int j) { return B3[l * k + j]; }, res);
    __syncthreads();
    ks_store(k, res, [&](int i, int j, double v) {
      B1[i * k + j] = -v;
      Cm[i * 2 * k + k + j] = -v;
    });
    __syncthreads();
    // leading rows of the update: X1 + E11 - Y1 N
    ks_zero(res);
    ks_mm(k, y1, [&](int l, int j) { return B1[l * k + j]; }, res);
    ks_store(k, res, [&](int i, int j, double v) { X1n[i * k + j] = B0[i * k + j] + B2[i * k + j] - v; });
    if (tid == 0) P.vec[VEC_E1SQ * k] = e1sq;
  }
}

int kxk_lds_doubles(int kmax) { return 0; }

hipError_t launch_kxk(const Prob* probs, int nprob, int kmax, hipStream_t st) {
  if (kmax <= KS_K)
    hipLaunchKernelGGL(kxk_small_kernel, dim3(nprob), dim3(KS_NT), 0, st, probs, nprob);
  else
    hipLaunchKernelGGL(kxk_kernel<false>, dim3(nprob), dim3(KXK_NT), 0, st, probs, nprob);
  return hipGetLastError();
}

hipError_t kxk_set_attributes() { return hipSuccess; }

}  // namespace rfk
