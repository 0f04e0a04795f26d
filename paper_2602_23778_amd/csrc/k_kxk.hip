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
//     V = H^T R are V2 = R2 - X2 M (the application of H^T in Algorithm 4; the top rows of V
//     are X^T R).
//   * E11 per the correction step of Algorithm 4 (eqs. Ediag, Eoffdiag; beta for
//     |d_j - d_i| <= delta).
//   * F = Y^T E_L = X1^T E11 + (X2^T R2 - X2^T X2 M) diag(1/(d - mu)) - E11,
//     using E21 = V2 diag(1/(d - mu)) without forming it, and N = T F = -Z^T F.
//   * The new leading rows X1 + E11 - Y1 N (the update step).
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
__global__ __launch_bounds__(KXK_NT) void kxk_kernel(const Prob* __restrict__ probs, int nprob,
                                                      int only_fb) {
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
    if (only_fb) {
      if (ctrl->stopped || !ctrl->kxk_fb) continue;
    } else {
      if (tid == 0) ctrl->apply = 0;
      if (ctrl->stopped) continue;
    }
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
    // ---- E11 (correction step of Algorithm 4) into the E buffer ----
    // free buffers: Eb, and whichever of Zb / Fb does not hold Z
    double* E1 = Eb;
    double* Fm = (Z == Fb) ? Zb : Fb;
    double e1sq = 0.0;
    const double delta = P.delta;
    const bool rr_top = ctrl->rr_top != 0;
    for (int e = tid; e < kk2; e += KXK_NT) {
      const int i = e / k, j = e - i * k;
      double v;
      if (rr_top) {
        v = 0.0;  // X is a Rayleigh-Ritz basis (Sec. 3.4, clustered eigenvalues)
      } else if (i == j) {
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
          // unconditional reads at clamped indices, masked afterwards: a
          // guarded read (some operands are in global memory) would wait
          // for each before the next
          const int l = 4 * (q0 + q) + g;
          const bool lok = q0 + q < kq && l < k;
          const int lc = min(l, k - 1);
          const double ta = a(min(i, k - 1), lc), tb = b(lc, min(j, k - 1));
          av[q] = (iok && lok) ? ta : 0.0;
          bv[q] = (jok && lok) ? tb : 0.0;
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

__global__ __launch_bounds__(KS_NT) void kxk_small_kernel(const Prob* __restrict__ probs, int nprob,
                                                           int only_fb) {
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
    if (only_fb) {
      if (ctrl->stopped || !ctrl->kxk_fb) continue;
    } else {
      if (tid == 0) ctrl->apply = 0;
      if (ctrl->stopped) continue;
    }
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
        const int e = tid + q * KS_NT, ec = min(e, kk2 - 1);
        const int i = ec / k, j = ec - i * k;
        const double tx = *gld(X + (int64_t)i * ldx + j), tz = *gld(Zg + ec);
        xv[q] = e < kk2 ? tx : 0.0;
        zv[q] = e < kk2 ? tz : 0.0;
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
        const int e = tid + q * KS_NT, ec = min(e, kk2 - 1);
        const double t = (*gld(PT + ec) + *gld(P2 + ec)) - *gld(R1 + ec);
        cv[q] = e < kk2 ? t : 0.0;
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
    // E11 (correction step of Algorithm 4) -> B2
    double e1sq = 0.0;
    {
      double pv[KS_EPT], gv[KS_EPT], di[KS_EPT], dj[KS_EPT], ai[KS_EPT];
      const double delta = P.delta;
      const bool rr_top = ctrl->rr_top != 0;
      // every operand of the sweep requested together (indices clamped)
#pragma unroll
      for (int q = 0; q < KS_EPT; ++q) {
        const int e = tid + q * KS_NT, ec = min(e, kk2 - 1);
        const int i = ec / k, j = ec - i * k;
        const double tp = *gld(PT + ec) + *gld(P2 + ec), tg = *gld(GT + ec) + *gld(G2 + ec);
        pv[q] = e < kk2 ? tp : 0.0;
        gv[q] = (e < kk2 && !P.beta_zero) ? tg : 0.0;
        di[q] = *gld(d + i);
        dj[q] = *gld(d + j);
        ai[q] = *gld(alpha + i);
      }
#pragma unroll
      for (int q = 0; q < KS_EPT; ++q) {
        const int e = tid + q * KS_NT;
        if (e < kk2) {
          const int i = e / k, j = e - i * k;
          double v;
          if (rr_top)
            v = 0.0;  // X is a Rayleigh-Ritz basis (Sec. 3.4, clustered eigenvalues)
          else if (i == j)
            v = (1.0 - ai[q]) * 0.5;
          else if (fabs(dj[q] - di[q]) <= delta)
            v = P.beta_zero ? 0.0 : -gv[q] * 0.5;
          else
            v = pv[q] / (dj[q] - di[q]);
          B2[e] = v;
          e1sq = __builtin_fma(v, v, e1sq);
        }
      }
    }
    e1sq = ks_sum(e1sq, red);
    // F = X1^T E11 + (X2^T R2 - X2^T X2 M) diag(1/(d - mu)) - E11 -> B3 (replacing M)
    ks_zero(res);
    ks_mm(k, [&](int i, int l) { return *gld(G2 + i * k + l); }, [&](int l, int j) { return B3[l * k + j]; },
          res);
    {
      const int lane = tid & 63, wave = tid >> 6, g = lane >> 4, r16 = lane & 15;
      const int nt = (k + 15) / 16;
#pragma unroll
      for (int sl = 0; sl < KS_SLOTS; ++sl) {
        const int t = wave + sl * KS_NW;
        if (t < nt * nt) {
          const int ti = t / nt, tj = t - ti * nt;
          const int j = tj * 16 + r16, jc = min(j, k - 1);
          // P2 and dinv of the tile requested together (indices clamped)
          double p2[4];
          const double dv = *gld(dinv + jc);
#pragma unroll
          for (int r = 0; r < 4; ++r) p2[r] = *gld(P2 + min(ti * 16 + mfma_row(g, r), k - 1) * k + jc);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = ti * 16 + mfma_row(g, r);
            if (row < k && j < k) res[sl][r] = (p2[r] - res[sl][r]) * dv - B2[row * k + j];
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

// ---------------------------------------------------------------------------
// Panel pipeline (one problem, any k <= 128): the same k-by-k work spread
// over np = ceil(k/16) workgroups, one per 16-row panel, one wavefront per
// 16x16 tile of the panel, in four launches:
//   1. F0 = I - Z0 Y1 with Z0 the previous step's Y1^{-1} (left residual);
//      C = X^T R - R1; E11 (correction step of Algorithm 4).
//   2. Z = (I + F0 + F0^2 + F0^3) Z0, whose left residual is F0^4, so Z is
//      accepted when ||F0||_F^4 <= 16 k u; M = -Z C; column sums of |Z|.
//      Otherwise the step's k-by-k work falls back to the one-workgroup
//      solver (Newton-Schulz from -I or Gauss-Jordan), launched next.
//   3. F = X1^T E11 + (X2^T R2 - X2^T X2 M) diag(1/(d-mu)) - E11;
//      Q = Y1 Z^T; column sums of |Y1|; Z kept as the next warm start.
//   4. cond_1(Y1) check (a failure stops the step before the update applies
//      it); N = -Z^T F and the leading rows X1 + E11 - Y1 N = X1 + E11 + Q F.
// Every product has the panel's rows on the left (a 16 x k panel in LDS) and
// a whole k x k matrix on the right (read from L2), so a panel needs no other
// panel's results within a launch.
// Partial sums (kpp): [0, 8) ||F0||^2 per panel, [8, 16) ||E11||^2 per panel,
// 16 + p k + j column sums of |Y1|, 16 + 8 k + p k + j column sums of |Z|.
// ---------------------------------------------------------------------------
constexpr int PP_LDA = KMAX + 4;  // LDS panel row stride (doubles)

// Loads are never behind a branch, which would make each one wait before
// the next is issued, and carry no masks: an index past k is clamped to
// k - 1 (FULL: k = 4 KQ, 64 or 128, where none is past k).  A right
// operand's rows past k meet the zero-padded columns of the panel in LDS,
// its columns past k and the elementwise operands past k only feed results
// that are not stored, so the clamped entries need only be finite.  The
// k x k offsets are 32-bit from a uniform base, one register per address.
template <bool FULL>
__device__ __forceinline__ int pp_cl(int i, int k) {
  return FULL || i < k ? i : k - 1;
}
// base[i] for p < np (partial sums), zero past np
__device__ __forceinline__ double pp_part(bool ok, const double* base, unsigned i) {
  const double v = *gld(base + (ok ? i : 0u));
  return ok ? v : 0.0;
}

// The right operand b (k x k, read from global memory) of a panel product,
// fetched into registers for the 16x16 result tile tj: lane l holds
// b(4q + l/16, tj*16 + l%16) for q < KQ (KQ >= ceil(k/4)), indices clamped
// to k - 1, so that a kernel can issue every fetch it needs in one round
// before any of them is consumed.
template <int KQ, bool FULL, class FB>
__device__ __forceinline__ void pp_fetch(int k, FB b, int tj, double (&bv)[KQ]) {
  const int lane = threadIdx.x & 63, g = lane >> 4, r16 = lane & 15;
  const int j = tj * 16 + r16;
#pragma unroll
  for (int q = 0; q < KQ; ++q) {
    const int l = 4 * q + g;
    bv[q] = b(pp_cl<FULL>(l, k), pp_cl<FULL>(j, k));
  }
}

// (16 x k panel in LDS, row stride PP_LDA) x (fetched right operand): the
// 16x16 result tile tj; register r of lane l holds row pi*16 + l/16 + 4r and
// column tj*16 + l%16.
template <int KQ, bool FULL>
__device__ __forceinline__ v4d pp_mul(int k, const double* As, const double (&bv)[KQ]) {
  const int lane = threadIdx.x & 63, g = lane >> 4, r16 = lane & 15;
  const int kq = FULL ? KQ : (k + 3) / 4;
  v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < KQ; q += 2) {
    if (q < kq) acc0 = mfma_f64(As[r16 * PP_LDA + 4 * q + g], bv[q], acc0);
    if (q + 1 < kq) acc1 = mfma_f64(As[r16 * PP_LDA + 4 * q + 4 + g], bv[q + 1], acc1);
  }
  return acc0 + acc1;
}

// Loads the 16 x k panel a(i, l) (rows i = pi*16 + r, zero-padded to a
// multiple of 4 columns and beyond k rows) into LDS, four loads per thread at
// most (16 * kp <= 4 * blockDim for kp <= 16 np, blockDim = 64 np), all
// issued before the first LDS store.  No closing barrier: several panels can
// be requested together, and the caller synchronises.
template <int KQ, bool FULL, class FA>
__device__ __forceinline__ void pp_load_nb(int k, int pi, double* As, FA a) {
  const int kp = FULL ? 4 * KQ : (k + 3) / 4 * 4;
  double v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = threadIdx.x + u * blockDim.x;
    const int r = e / kp, l = e - r * kp;
    const int i = pi * 16 + r;
    if constexpr (FULL) {
      v[u] = a(i, l);
    } else {
      const bool ok = e < 16 * kp && i < k && l < k;
      const double t = a(ok ? i : 0, ok ? l : 0);
      v[u] = ok ? t : 0.0;
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = threadIdx.x + u * blockDim.x;
    if (FULL || e < 16 * kp) As[(e / kp) * PP_LDA + e % kp] = v[u];
  }
}

// Calls f(i, j, v) for the valid entries of a tile result.
template <bool FULL, class FS>
__device__ __forceinline__ void pp_each(int k, int pi, int tj, const v4d& acc, FS f) {
  const int lane = threadIdx.x & 63, g = lane >> 4, r16 = lane & 15;
  const int j = tj * 16 + r16;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = pi * 16 + mfma_row(g, r);
    if (FULL || (i < k && j < k)) f(i, j, acc[r]);
  }
}

// Block sum of one value per thread (all threads call it).
__device__ __forceinline__ double pp_sum(double v, double* red) {
  for (int o = 32; o >= 1; o /= 2) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  return t;
}

__device__ __forceinline__ double pp_y1(const Prob& P, int i, int l) {
  return *gld(P.x + (int64_t)i * P.ldx + l) - (i == l ? 1.0 : 0.0);
}

// Every kernel of the pipeline requests all it needs (panels, right
// operands, partial sums) in one round at its start, so that it waits on
// memory once rather than once per product (past k = 64 a third right
// operand comes once the first products are done, within the register file).
template <int KQ, bool FULL>
__global__ __launch_bounds__(512) void pp_res_kernel(const Prob* __restrict__ probs) {
  __shared__ double As[16 * PP_LDA];
  __shared__ double red[8];
  const Prob& P = probs[0];
  Ctrl* ctrl = P.ctrl;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->apply = 0;
  if (ctrl->stopped) return;
  const int k = P.k, kk2 = k * k, pi = blockIdx.x, tj = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63, g = lane >> 4, r16 = lane & 15;
  const double* Zg = P.kk + KK_Z * kk2;
  double* F0 = P.kk + KK_S0 * kk2;
  double* Cb = P.kk + (KK_S0 + 1) * kk2;
  double* E1 = P.kk + (KK_S0 + 2) * kk2;
  const double* PT = P.kk + KK_PT * kk2;
  const double* P2 = P.kk + KK_P2 * kk2;
  const double* GT = P.kk + KK_GT * kk2;
  const double* G2 = P.kk + KK_G2 * kk2;
  const double* R1 = P.kk + KK_R1 * kk2;
  const double* d = P.vec + VEC_D * k;
  const double* alpha = P.vec + VEC_ALPHA * k;
  const bool rr_top = ctrl->rr_top != 0;
  const double delta = P.delta;
  const bool beta_zero = P.beta_zero != 0;
  // this lane's four entries (rows pi*16 + g + 4r, column tj*16 + r16), the
  // right operand Y1 and the panel of Z0
  const int j = tj * 16 + r16;
  double by[KQ];
  pp_fetch<KQ, FULL>(k, [&](int l, int jj) { return pp_y1(P, l, jj); }, tj, by);
  double vpt[4], vp2[4], vr1[4], vg[4], di[4], ai[4];
  const int jc = pp_cl<FULL>(j, k);
  const double dj = *gld(d + jc);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ic = pp_cl<FULL>(pi * 16 + mfma_row(g, r), k);
    const unsigned e = (unsigned)(ic * k + jc);
    vpt[r] = *gld(PT + e);
    vp2[r] = *gld(P2 + e);
    vr1[r] = *gld(R1 + e);
    vg[r] = *gld(GT + e) + *gld(G2 + e);
    di[r] = *gld(d + ic);
    ai[r] = *gld(alpha + ic);
  }
  pp_load_nb<KQ, FULL>(k, pi, As, [&](int i, int l) { return *gld(Zg + (unsigned)(i * k + l)); });
  __syncthreads();
  // F0 = I - Z0 Y1
  const v4d acc = pp_mul<KQ, FULL>(k, As, by);
  double f2 = 0.0, e2 = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = pi * 16 + mfma_row(g, r);
    if (FULL || (i < k && j < k)) {
      const unsigned e = (unsigned)(i * k + j);
      const double f = (i == j ? 1.0 : 0.0) - acc[r];
      *gst(F0 + e) = f;
      f2 = __builtin_fma(f, f, f2);
      const double v1 = vpt[r] + vp2[r];
      *gst(Cb + e) = v1 - vr1[r];
      double ev;
      if (rr_top)
        ev = 0.0;  // X is a Rayleigh-Ritz basis (Sec. 3.4, clustered eigenvalues)
      else if (i == j)
        ev = (1.0 - ai[r]) * 0.5;
      else if (fabs(dj - di[r]) <= delta)
        ev = beta_zero ? 0.0 : -vg[r] * 0.5;
      else
        ev = v1 / (dj - di[r]);
      *gst(E1 + e) = ev;
      e2 = __builtin_fma(ev, ev, e2);
    }
  }
  f2 = pp_sum(f2, red);
  e2 = pp_sum(e2, red);
  if (threadIdx.x == 0) {
    P.kpp[pi] = f2;
    P.kpp[8 + pi] = e2;
  }
}

template <int KQ, bool FULL>
__global__ __launch_bounds__(512) void pp_ns_kernel(const Prob* __restrict__ probs) {
  __shared__ double As[16 * PP_LDA];
  __shared__ double Bs[16 * PP_LDA];
  const Prob& P = probs[0];
  Ctrl* ctrl = P.ctrl;
  if (ctrl->stopped) return;
  const int k = P.k, kk2 = k * k, pi = blockIdx.x;
  const int tj = threadIdx.x >> 6;
  const int np = FULL ? KQ / 4 : (k + 15) / 16;
  const double* Zg = P.kk + KK_Z * kk2;
  const double* F0 = P.kk + KK_S0 * kk2;
  const double* Cb = P.kk + (KK_S0 + 1) * kk2;
  double* Zn = P.kk + (KK_S0 + 3) * kk2;
  double* Cm = P.kk + KK_CM * kk2;
  // one round: F0 and Z0 as right operands, the panel of F0 and the partial
  // norms of F0 (fetched before the acceptance test; unused if the warm
  // start is rejected); C follows past k = 64, once F0^3 is formed
  double bF[KQ], bZ[KQ], bC[KQ];
  auto fetch_c = [&]() {
    pp_fetch<KQ, FULL>(k, [&](int l, int j) { return *gld(Cb + (unsigned)(l * k + j)); }, tj, bC);
  };
  pp_fetch<KQ, FULL>(k, [&](int l, int j) { return *gld(F0 + (unsigned)(l * k + j)); }, tj, bF);
  pp_fetch<KQ, FULL>(k, [&](int l, int j) { return *gld(Zg + (unsigned)(l * k + j)); }, tj, bZ);
  if constexpr (KQ <= 16) fetch_c();
  pp_load_nb<KQ, FULL>(k, pi, As, [&](int i, int l) { return *gld(F0 + (unsigned)(i * k + l)); });
  double f2 = 0.0;
#pragma unroll
  for (int p = 0; p < 8; ++p) f2 += pp_part(p < np, P.kpp, (unsigned)p);  // np <= 8
  const double eres = sqrt(f2);
  const double tol = 16.0 * k * UNIT_ROUNDOFF;
  const bool accept = (eres * eres) * (eres * eres) <= tol;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->kxk_fb = accept ? 0 : 1;
  if (!accept) return;  // the same decision in every thread
  __syncthreads();
  // T = I + F0 + F0^2 + F0^3 on this panel, accumulated in Bs
  {
    const int kp = FULL ? 4 * KQ : (k + 3) / 4 * 4;
    for (int e = threadIdx.x; e < 16 * kp; e += blockDim.x) {
      const int r = e / kp, l = e - r * kp;
      const int i = pi * 16 + r;
      Bs[r * PP_LDA + l] = (FULL || (i < k && l < k)) ? As[r * PP_LDA + l] + (i == l ? 1.0 : 0.0) : 0.0;
    }
  }
  for (int pw = 2; pw <= 3; ++pw) {
    // As <- As F0 (F0^pw on the panel); Bs += As
    const v4d acc = pp_mul<KQ, FULL>(k, As, bF);
    __syncthreads();
    pp_each<FULL>(k, pi, tj, acc, [&](int i, int j, double v) {
      const int r = i - pi * 16;
      As[r * PP_LDA + j] = v;
      Bs[r * PP_LDA + j] += v;
    });
    __syncthreads();
  }
  if constexpr (KQ > 16) fetch_c();
  // Z = T Z0 on this panel -> As and Zn
  {
    const v4d acc = pp_mul<KQ, FULL>(k, Bs, bZ);
    __syncthreads();
    pp_each<FULL>(k, pi, tj, acc, [&](int i, int j, double v) {
      As[(i - pi * 16) * PP_LDA + j] = v;
      *gst(Zn + (unsigned)(i * k + j)) = v;
    });
    __syncthreads();
  }
  // M = -Z C
  {
    const v4d acc = pp_mul<KQ, FULL>(k, As, bC);
    pp_each<FULL>(k, pi, tj, acc, [&](int i, int j, double v) { *gst(Cm + (unsigned)(i * 2 * k + j)) = -v; });
  }
  // column sums of |Z| over the panel's rows
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    double c = 0.0;
    for (int r = 0; r < 16 && pi * 16 + r < k; ++r) c += fabs(As[r * PP_LDA + j]);
    P.kpp[16 + 8 * k + pi * k + j] = c;
  }
}

template <int KQ, bool FULL>
__global__ __launch_bounds__(512) void pp_f_kernel(const Prob* __restrict__ probs) {
  __shared__ double As[3][16 * PP_LDA];
  const Prob& P = probs[0];
  Ctrl* ctrl = P.ctrl;
  if (ctrl->stopped || ctrl->kxk_fb) return;
  const int k = P.k, kk2 = k * k, pi = blockIdx.x, tj = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63, g = lane >> 4, r16 = lane & 15;
  const double* Zn = P.kk + (KK_S0 + 3) * kk2;
  double* Zg = P.kk + KK_Z * kk2;
  double* Fm = P.kk + KK_S0 * kk2;  // F0 is no longer needed
  const double* E1 = P.kk + (KK_S0 + 2) * kk2;
  const double* P2 = P.kk + KK_P2 * kk2;
  const double* G2 = P.kk + KK_G2 * kk2;
  const double* Cm = P.kk + KK_CM * kk2;
  double* Q = P.kk + KK_Q * kk2;
  const int j = tj * 16 + r16;
  // one round: E11, M and Z^T as right operands, the panels of X1^T, G2 and
  // Y1, and the elementwise parts
  // (past k = 64 the third operand is fetched once the first two are used,
  // which keeps the three within the register file)
  double bE[KQ], bM[KQ], bZt[KQ];
  auto fetch_zt = [&]() {
    pp_fetch<KQ, FULL>(k, [&](int l, int jj) { return *gld(Zn + (unsigned)(jj * k + l)); }, tj, bZt);
  };
  pp_fetch<KQ, FULL>(k, [&](int l, int jj) { return *gld(E1 + (unsigned)(l * k + jj)); }, tj, bE);
  pp_fetch<KQ, FULL>(k, [&](int l, int jj) { return *gld(Cm + (unsigned)(l * 2 * k + jj)); }, tj, bM);
  if constexpr (KQ <= 16) fetch_zt();
  double vp2[4], ve1[4], zc[4];
  const int jc = pp_cl<FULL>(j, k);
  const double dj = *gld(P.vec + VEC_DINV * k + jc);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ic = pp_cl<FULL>(pi * 16 + mfma_row(g, r), k);
    const unsigned e = (unsigned)(ic * k + jc);
    vp2[r] = *gld(P2 + e);
    ve1[r] = *gld(E1 + e);
    zc[r] = *gld(Zn + e);
  }
  pp_load_nb<KQ, FULL>(k, pi, As[0], [&](int i, int l) { return *gld(P.x + (int64_t)l * P.ldx + i); });
  pp_load_nb<KQ, FULL>(k, pi, As[1], [&](int i, int l) { return *gld(G2 + (unsigned)(i * k + l)); });
  pp_load_nb<KQ, FULL>(k, pi, As[2], [&](int i, int l) { return pp_y1(P, i, l); });
  __syncthreads();
  // F = X1^T E11 + (P2 - G2 M) diag(dinv) - E11
  const v4d fa = pp_mul<KQ, FULL>(k, As[0], bE);
  const v4d fb = pp_mul<KQ, FULL>(k, As[1], bM);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = pi * 16 + mfma_row(g, r);
    if (FULL || (i < k && j < k)) {
      const unsigned e = (unsigned)(i * k + j);
      *gst(Fm + e) = fa[r] + (vp2[r] - fb[r]) * dj - ve1[r];
      *gst(Zg + e) = zc[r];  // the next step's warm start
    }
  }
  // Q = Y1 Z^T, and the column sums of |Y1| over this panel's rows
  if constexpr (KQ > 16) fetch_zt();
  const v4d qa = pp_mul<KQ, FULL>(k, As[2], bZt);
  pp_each<FULL>(k, pi, tj, qa, [&](int i, int jj, double v) { *gst(Q + (unsigned)(i * k + jj)) = v; });
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    double a = 0.0;
    for (int r = 0; r < 16; ++r) a += fabs(As[2][r * PP_LDA + c]);  // zero rows beyond k
    P.kpp[16 + pi * k + c] = a;
  }
}

template <int KQ, bool FULL>
__global__ __launch_bounds__(512) void pp_n_kernel(const Prob* __restrict__ probs) {
  __shared__ double As[2][16 * PP_LDA];
  __shared__ double red[2][8];
  const Prob& P = probs[0];
  Ctrl* ctrl = P.ctrl;
  if (ctrl->stopped || ctrl->kxk_fb) return;
  const int n = P.n, k = P.k, kk2 = k * k, pi = blockIdx.x, tj = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63, g = lane >> 4, r16 = lane & 15;
  const int np = FULL ? KQ / 4 : (k + 15) / 16;
  const double* Zn = P.kk + (KK_S0 + 3) * kk2;
  const double* Fm = P.kk + KK_S0 * kk2;
  const double* E1 = P.kk + (KK_S0 + 2) * kk2;
  const double* Q = P.kk + KK_Q * kk2;
  double* Cm = P.kk + KK_CM * kk2;
  double* X1n = P.kk + KK_X1N * kk2;
  const int j = tj * 16 + r16;
  // one round: F as the right operand of both products, the panels of Z^T
  // and Q, the elementwise parts and the column sums for cond_1
  double bF[KQ];
  pp_fetch<KQ, FULL>(k, [&](int l, int jj) { return *gld(Fm + (unsigned)(l * k + jj)); }, tj, bF);
  double vx[4], ve1[4];
  const int jc = pp_cl<FULL>(j, k);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ic = pp_cl<FULL>(pi * 16 + mfma_row(g, r), k);
    vx[r] = *gld(P.x + (int64_t)ic * P.ldx + jc);
    ve1[r] = *gld(E1 + (unsigned)(ic * k + jc));
  }
  pp_load_nb<KQ, FULL>(k, pi, As[0], [&](int i, int l) { return *gld(Zn + (unsigned)(l * k + i)); });
  pp_load_nb<KQ, FULL>(k, pi, As[1], [&](int i, int l) { return *gld(Q + (unsigned)(i * k + l)); });
  // cond_1(Y1) = ||Y1||_1 ||Z||_1 from the panel column sums (the same in
  // every block); a failure stops the step before the update applies it
  // (k <= blockDim: one column per thread, its partials requested together)
  double cy = 0.0, cz = 0.0;
  {
    constexpr int NPM = FULL ? KQ / 4 : 8;  // np <= 8
    const int c = (int)threadIdx.x < k ? (int)threadIdx.x : 0;
    double va[NPM], vb[NPM];
#pragma unroll
    for (int p = 0; p < NPM; ++p) {
      va[p] = pp_part(FULL || p < np, P.kpp + 16 + c, (unsigned)(p * k));
      vb[p] = pp_part(FULL || p < np, P.kpp + 16 + 8 * k + c, (unsigned)(p * k));
    }
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int p = 0; p < NPM; ++p) {
      a += va[p];
      b += vb[p];
    }
    if ((int)threadIdx.x < k) {
      cy = a;
      cz = b;
    }
  }
  for (int o = 32; o >= 1; o /= 2) {
    cy = fmax(cy, __shfl_xor(cy, o));
    cz = fmax(cz, __shfl_xor(cz, o));
  }
  if (lane == 0) {
    red[0][tj] = cy;
    red[1][tj] = cz;
  }
  __syncthreads();  // also completes the panels in LDS
  double ny = 0.0, nz = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    ny = fmax(ny, red[0][w]);
    nz = fmax(nz, red[1][w]);
  }
  if (!(ny * nz <= 1.0 / ((double)n * UNIT_ROUNDOFF))) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctrl->status = -4;
      ctrl->stopped = 1;
    }
    return;
  }
  // N = -Z^T F
  const v4d na = pp_mul<KQ, FULL>(k, As[0], bF);
  pp_each<FULL>(k, pi, tj, na, [&](int i, int jj, double v) { *gst(Cm + (unsigned)(i * 2 * k + k + jj)) = -v; });
  // X1 + E11 + Q F
  const v4d xa = pp_mul<KQ, FULL>(k, As[1], bF);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = pi * 16 + mfma_row(g, r);
    if (FULL || (i < k && j < k)) *gst(X1n + (unsigned)(i * k + j)) = vx[r] + ve1[r] + xa[r];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double e2 = 0.0;
#pragma unroll
    for (int p = 0; p < 8; ++p) e2 += pp_part(p < np, P.kpp + 8, (unsigned)p);
    P.vec[VEC_E1SQ * k] = e2;
  }
}

// Statistics of the fused update (one problem through the panel pipeline,
// k > 32), one workgroup per 16-row panel after pp_n (which completes N; on a
// step that took the one-workgroup fallback, that solver wrote M and N).
// With C = M Delta + N and a_j the column j of I - C, the bottom rows update
// as X~2 = X2 + R2 Delta - X2 C, and the column norms of the step are
// quadratic forms in k x k quantities (fin_post_kernel):
//   ||x~_j||^2  = ||x~1_j||^2 + a_j^T G2 a_j + 2 Delta_j a_j^T p_j + Delta_j^2 s_j,
//   ||e21_j||^2 = Delta_j^2 (s_j - 2 m_j^T p_j + m_j^T G2 m_j),
// with G2 = X2^T X2 and p_j, m_j the columns j of X2^T R2 and M.  This
// launch writes C's panel rows (the update's right operand) and, per column,
// the panel rows' parts of a_j^T G2 a_j, m_j^T G2 m_j, a_j^T p_j, m_j^T p_j
// (using (G2 a_j)_i = G2_ij - (G2 C)_ij), ||x~1_j||^2 and ||r1_j||^2.
template <int KQ, bool FULL>
__global__ __launch_bounds__(512) void pp_q_kernel(const Prob* __restrict__ probs) {
  __shared__ double As[16 * PP_LDA];
  const Prob& P = probs[0];
  if (P.ctrl->stopped) return;
  const int k = P.k, kk2 = k * k, k2 = 2 * k, pi = blockIdx.x, tj = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63, g = lane >> 4, r16 = lane & 15;
  const double* G2 = P.kk + KK_G2 * kk2;
  const double* P2 = P.kk + KK_P2 * kk2;
  const double* Cm = P.kk + KK_CM * kk2;
  const double* X1n = P.kk + KK_X1N * kk2;
  const double* R1 = P.kk + KK_R1 * kk2;
  double* Cc = P.kk + KK_FC * kk2;
  double* Qp = P.kk + KK_FQ * kk2;
  const int j = tj * 16 + r16;
  // one round: M and N as right operands, the lane's entries, G2's panel
  double bM[KQ], bC[KQ];
  pp_fetch<KQ, FULL>(k, [&](int l, int jj) { return *gld(Cm + (unsigned)(l * k2 + jj)); }, tj, bM);
  pp_fetch<KQ, FULL>(k, [&](int l, int jj) { return *gld(Cm + (unsigned)(l * k2 + k + jj)); }, tj, bC);
  const int jc = pp_cl<FULL>(j, k);
  const double dj = *gld(P.vec + VEC_DINV * k + jc);
  double vm[4], vn[4], vg[4], vp[4], vx[4], vr[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ic = pp_cl<FULL>(pi * 16 + mfma_row(g, r), k);
    vm[r] = *gld(Cm + (unsigned)(ic * k2 + jc));
    vn[r] = *gld(Cm + (unsigned)(ic * k2 + k + jc));
    vg[r] = *gld(G2 + (unsigned)(ic * k + jc));
    vp[r] = *gld(P2 + (unsigned)(ic * k + jc));
    vx[r] = *gld(X1n + (unsigned)(ic * k + jc));
    vr[r] = *gld(R1 + (unsigned)(ic * k + jc));
  }
  pp_load_nb<KQ, FULL>(k, pi, As, [&](int i, int l) { return *gld(G2 + (unsigned)(i * k + l)); });
  __syncthreads();
#pragma unroll
  for (int q = 0; q < KQ; ++q) bC[q] = __builtin_fma(bM[q], dj, bC[q]);  // C = M Delta + N
  const v4d gc = pp_mul<KQ, FULL>(k, As, bC);
  const v4d gm = pp_mul<KQ, FULL>(k, As, bM);
  double sA = 0.0, sM = 0.0, pA = 0.0, pM = 0.0, top = 0.0, r1 = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = pi * 16 + mfma_row(g, r);
    if (FULL || (i < k && j < k)) {
      const double c = __builtin_fma(vm[r], dj, vn[r]);
      const double a = (i == j ? 1.0 : 0.0) - c;
      *gst(Cc + (unsigned)(i * k + j)) = c;
      sA = __builtin_fma(a, vg[r] - gc[r], sA);
      sM = __builtin_fma(vm[r], gm[r], sM);
      pA = __builtin_fma(a, vp[r], pA);
      pM = __builtin_fma(vm[r], vp[r], pM);
      top = __builtin_fma(vx[r], vx[r], top);
      r1 = __builtin_fma(vr[r], vr[r], r1);
    }
  }
  // the panel's rows of column j sit in the four lane groups
#pragma unroll
  for (int o = 16; o <= 32; o *= 2) {
    sA += __shfl_xor(sA, o);
    sM += __shfl_xor(sM, o);
    pA += __shfl_xor(pA, o);
    pM += __shfl_xor(pM, o);
    top += __shfl_xor(top, o);
    r1 += __shfl_xor(r1, o);
  }
  if (g == 0 && j < k) {
    double* q = Qp + (unsigned)(pi * 6 * k + j);
    *gst(q) = sA;
    *gst(q + k) = sM;
    *gst(q + 2 * k) = pA;
    *gst(q + 3 * k) = pM;
    *gst(q + 4 * k) = top;
    *gst(q + 5 * k) = r1;
  }
}

// One problem: the panel pipeline with the one-workgroup solver as its
// fallback (which runs only when the warm start is not close enough).
// Batches: the one-workgroup solver per problem.
// pipeline: one problem through the four-launch panel pipeline (the
// one-workgroup kernel only as its fallback); otherwise the whole stage runs
// in one workgroup per problem.  fused (with pipeline): a fifth launch forms
// the statistics of the fused update (pp_q_kernel).
hipError_t launch_kxk(const Prob* probs, int nprob, int kmax, bool pipeline, bool fused,
                      hipStream_t st) {
  if (nprob == 1 && pipeline) {
    const int np = (kmax + 15) / 16;
    const dim3 grid(np), block(64 * np);
    const bool q16 = kmax <= 64;  // contraction in groups of four: 16 or 32 groups
    const bool full = kmax == 64 || kmax == 128;  // k = 4 KQ: no entry masked
#define RFK_PP(KERNEL)                                                         \
  do {                                                                         \
    if (q16 && full)                                                           \
      hipLaunchKernelGGL((KERNEL<16, true>), grid, block, 0, st, probs);       \
    else if (q16)                                                              \
      hipLaunchKernelGGL((KERNEL<16, false>), grid, block, 0, st, probs);      \
    else if (full)                                                             \
      hipLaunchKernelGGL((KERNEL<32, true>), grid, block, 0, st, probs);       \
    else                                                                       \
      hipLaunchKernelGGL((KERNEL<32, false>), grid, block, 0, st, probs);      \
  } while (0)
    RFK_PP(pp_res_kernel);
    RFK_PP(pp_ns_kernel);
    if (kmax <= KS_K)
      hipLaunchKernelGGL(kxk_small_kernel, dim3(1), dim3(KS_NT), 0, st, probs, 1, 1);
    else
      hipLaunchKernelGGL(kxk_kernel<false>, dim3(1), dim3(KXK_NT), 0, st, probs, 1, 1);
    RFK_PP(pp_f_kernel);
    RFK_PP(pp_n_kernel);
    if (fused) RFK_PP(pp_q_kernel);
#undef RFK_PP
    return hipGetLastError();
  }
  if (kmax <= KS_K)
    hipLaunchKernelGGL(kxk_small_kernel, dim3(nprob), dim3(KS_NT), 0, st, probs, nprob, 0);
  else
    hipLaunchKernelGGL(kxk_kernel<false>, dim3(nprob), dim3(KXK_NT), 0, st, probs, nprob, 0);
  return hipGetLastError();
}

}  // namespace rfk
