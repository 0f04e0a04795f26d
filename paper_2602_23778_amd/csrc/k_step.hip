// The steps of Algorithm 4 after the product (and the column normalisation of Sec. 3.1.3) for one
// or many problems.  The step is written so that no n x n matrix and no
// explicit H is formed (Sec. 3.1.2, after Table 1) and so that every pass over
// the n x k arrays streams them once:
//
//   pass 1  (products) the product kernels write the column sums of x_j * w_j
//                      and x_j * x_j per block; wsum adds the split-K partials
//                      of the dense product; fin_d forms d_j = x_j^T w_j / alpha_j
//                      (eq. Rayleigh).  Cross-block sums always go through
//                      memory and a later kernel: no in-kernel device-wide
//                      fences, which on this GPU write back the whole L2.
//   pass 2  (gram)     R = W - X D on the fly; X2^T R2, X2^T X2 (rows >= k) as
//                      per-block partials on the FP64 matrix cores, and
//                      X1^T R1, X1^T X1, R1 for the leading k rows.
//   reduce             sums the Gram partials in a fixed order.
//   kxk     (1 WG)     the k-by-k part (k_kxk.hip): T = -Y1^{-T}, M, E11, N and
//                      the updated leading rows.
//   pass 3  (update)   bottom rows: E21 = (R2 - X2 M) diag(1/(d - mu)) and
//                      X2 + E21 - X2 N, with [X2 M | X2 N] on the matrix cores;
//                      fin_stats forms the normalisation factors and the
//                      statistics, and accepts or rejects the step.
//   pass 4  (normalize) X = scaled update, only when the step was accepted.
//
// Fused order (k <= 32, and one problem through the k-by-k panel pipeline):
// the column norms of the update and of E21 come from k x k quadratic forms
// after the k-by-k part (fin_pre, or pp_q + fin_post), so the statistics and
// the decision come first and pass 3 writes the normalised iterate into X
// itself; pass 4 and the n x k copy of the update are not needed.
#include "common.h"
#include "dev_util.h"

namespace rfk {

// ---------------------------------------------------------------------------
// pass 2: Gram partials on the matrix cores (k > 32).  One work item per
// (row block, 16-column tile tj of R): the block's RG wavefronts take
// interleaved 4-row steps of the block's rows.  Each computes r for tile tj
// only, so every W value is read once, and accumulates the tiles (ti, tj) of
// X^T R for every left tile ti and (ti, tj), ti <= tj, of X^T X (the upper
// tiles; the reduction mirrors the rest).  Lane l reads row (r + l/16) at
// column (t*16 + l%16), so both MFMA operands are plain row-major reads.
// Loads never branch: rows past the block repeat its first row and columns
// past k repeat column 0, masked afterwards, so U steps are requested before
// their products.  The wavefronts' tiles are summed in LDS in a fixed order.
// Rows < k (block 0 only) go straight to X1^T R1 and X1^T X1, the latter
// written in full (its lower tiles mirrored), and r itself to R1.
// ---------------------------------------------------------------------------
int gram_groups(int kmax) { return kmax <= 32 ? 1 : (kmax + 15) / 16; }

template <int CT, int RG, int U, bool LO>
__global__ __launch_bounds__(RG * 64) void gram_tile_kernel(const Prob* __restrict__ probs,
                                                           const RowItem* __restrict__ items,
                                                           int nitems) {
  constexpr int QB = 4;  // tiles per LDS exchange round
  __shared__ double xch[RG][QB][256];
  __shared__ double rsq_x[RG][64];
  const int lane = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem item = items[it];
    const Prob& P = probs[item.prob];
    if (P.ctrl->stopped) continue;
    const int n = P.n, k = P.k;
    const int ct_used = (k + 15) / 16;
    const int blk = item.blk / ct_used, tj = item.blk - blk * ct_used;
    const double* __restrict__ X = P.x;
    const double* __restrict__ Wh = P.w;
    const double* __restrict__ Wl = LO ? P.wlo : P.w;
    const int64_t ldx = P.ldx;
    const int r0 = blk * P.gbrows, r1 = min(n, r0 + P.gbrows);
    const int kk2 = k * k;
    const int c = tj * 16 + r16;
    const bool cok = c < k;
    const int cc = cok ? c : 0;
    int ca[CT];
    bool aok[CT];
#pragma unroll
    for (int ti = 0; ti < CT; ++ti) {
      const int a = ti * 16 + r16;
      aok[ti] = a < k;
      ca[ti] = aok[ti] ? a : 0;
    }
    const double dv = *gld(P.vec + VEC_D * k + cc);
    double rsq = 0.0;

    // phase 0: rows < k (only block 0 has them); phase 1: rows >= k, whose
    // partial is written even when the block has none (zeros)
    for (int phase = 0; phase < 2; ++phase) {
      const int lo = phase == 0 ? r0 : max(r0, k);
      const int hi = phase == 0 ? min(r1, k) : r1;
      if (phase == 0 && lo >= hi) continue;
      v4d accP[CT], accG[CT];
#pragma unroll
      for (int t = 0; t < CT; ++t) {
        accP[t] = v4d{0.0, 0.0, 0.0, 0.0};
        accG[t] = v4d{0.0, 0.0, 0.0, 0.0};
      }
      // operands of the U steps from row base on (rows past hi repeat lo)
      auto load = [&](int base, double(&xa)[U][CT], double(&xt)[U], double(&wv)[U], double(&lv)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int row = base + 4 * u + g;
          const int rr = row < hi ? row : lo;
          const double* xr = X + (int64_t)rr * ldx;
#pragma unroll
          for (int ti = 0; ti < CT; ++ti) xa[u][ti] = *gld(xr + ca[ti]);
          xt[u] = *gld(xr + cc);
          wv[u] = *gld(Wh + (int64_t)rr * k + cc);
          lv[u] = LO ? *gld(Wl + (int64_t)rr * k + cc) : 0.0;
        }
      };
      // products of the U steps from row base on (rows past hi add zeros)
      auto step = [&](int base, const double(&xa)[U][CT], const double(&xt)[U], const double(&wv)[U],
                      const double(&lv)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int row = base + 4 * u + g;
          const bool rok = row < hi;
          const bool ok = rok && cok;
          const double xm_t = ok ? xt[u] : 0.0;
          const double rv = ok ? residual(wv[u], lv[u], xt[u], dv, LO) : 0.0;
          rsq = __builtin_fma(rv, rv, rsq);
#pragma unroll
          for (int ti = 0; ti < CT; ++ti) {
            if (ti < ct_used) {
              const double xm = (rok && aok[ti]) ? xa[u][ti] : 0.0;
              accP[ti] = mfma_f64(xm, rv, accP[ti]);
              if (ti <= tj) accG[ti] = mfma_f64(xm, xm_t, accG[ti]);
            }
          }
          if (phase == 0 && ok) *gst(P.kk + KK_R1 * kk2 + row * k + c) = rv;
        }
      };
      // two register sets: the next U steps are requested before the
      // current ones are multiplied
      constexpr int STRIDE = RG * 4 * U;
      double xa0[U][CT], xt0[U], wv0[U], lv0[U], xa1[U][CT], xt1[U], wv1[U], lv1[U];
      int base = lo + rg * 4 * U;
      if (base < hi) load(base, xa0, xt0, wv0, lv0);
      for (; base < hi; base += 2 * STRIDE) {
        load(base + STRIDE, xa1, xt1, wv1, lv1);
        step(base, xa0, xt0, wv0, lv0);
        if (base + STRIDE >= hi) break;
        load(base + 2 * STRIDE, xa0, xt0, wv0, lv0);
        step(base + STRIDE, xa1, xt1, wv1, lv1);
      }
      double* dstP;
      double* dstG;
      if (phase == 0) {
        dstP = P.kk + KK_PT * kk2;
        dstG = P.kk + KK_GT * kk2;
      } else {
        dstP = P.gpart + (int64_t)blk * (2 * kk2 + k);
        dstG = dstP + kk2;
      }
      // tile q < CT is (q, tj) of X^T R, q >= CT is (q - CT, tj) of X^T X;
      // QB tiles a round, each summed over the wavefronts by one of them
#pragma unroll
      for (int q0 = 0; q0 < 2 * CT; q0 += QB) {
#pragma unroll
        for (int qq = 0; qq < QB; ++qq) {
          const int q = q0 + qq;
          if (q < 2 * CT) {
            const v4d& v = q < CT ? accP[q < CT ? q : 0] : accG[q >= CT ? q - CT : 0];
#pragma unroll
            for (int r = 0; r < 4; ++r) xch[rg][qq][lane * 4 + r] = v[r];
          }
        }
        __syncthreads();
        for (int qq = rg; qq < QB; qq += RG) {
          const int q = q0 + qq;
          const bool is_g = q >= CT;
          const int ti = is_g ? q - CT : q;
          if (q < 2 * CT && ti < ct_used && (!is_g || ti <= tj) && cok) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              double a = xch[0][qq][lane * 4 + r];
              for (int w = 1; w < RG; ++w) a += xch[w][qq][lane * 4 + r];
              const int i = ti * 16 + mfma_row(g, r);
              if (i < k) {
                *gst((is_g ? dstG : dstP) + i * k + c) = a;
                if (is_g && phase == 0 && ti < tj) *gst(dstG + c * k + i) = a;
              }
            }
          }
        }
        __syncthreads();
      }
    }
    // column sums of r^2 over the block's rows, tile tj
    rsq_x[rg][lane] = rsq;
    __syncthreads();
    if (threadIdx.x < 16) {
      const int c16 = threadIdx.x, cs = tj * 16 + c16;
      if (cs < k) {
        double s = 0.0;
        for (int q = 0; q < RG; ++q)
          s += (rsq_x[q][c16] + rsq_x[q][16 + c16]) + (rsq_x[q][32 + c16] + rsq_x[q][48 + c16]);
        *gst(P.gpart + (int64_t)blk * (2 * kk2 + k) + 2 * kk2 + cs) = s;
      }
    }
    __syncthreads();
  }
}

// The same pass for k <= 32 (CT <= 2): every wavefront accumulates all
// tiles, so each X and W value is loaded once, and U 4-row steps are
// requested before their products.  Loads never branch (clamped addresses,
// masked values), which keeps the compiler's wait counts exact.  The RG
// wavefronts of a block take interleaved runs of 4U rows; their tiles and
// column sums are added in LDS in a fixed order.  LO (W has a low part) is a
// template argument, so the FP64 form carries no registers for it (166
// registers at CT = 2 in both forms, against 193 with a runtime flag).
template <int CT, int RG, int U, bool LO>
__global__ __launch_bounds__(RG * 64) void gram_all_kernel(const Prob* __restrict__ probs,
                                                          const RowItem* __restrict__ items,
                                                          int nitems) {
  static_assert(CT <= 2, "tile bookkeeping below covers CT <= 2");
  constexpr int NTP = CT * CT, NTG = CT * (CT + 1) / 2;
  __shared__ double xch[RG][256];
  __shared__ double rsq_x[RG][CT * 64];
  const int lane = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem item = items[it];
    const Prob& P = probs[item.prob];
    if (P.ctrl->stopped) continue;
    const int n = P.n, k = P.k;
    const int ct_used = (k + 15) / 16;
    const bool has_lo = LO;  // launched for the form of W (with a low part or not)
    const double* __restrict__ X = P.x;
    const double* __restrict__ Wh = P.w;
    const double* __restrict__ Wl = LO ? P.wlo : P.w;
    const int64_t ldx = P.ldx;
    const int r0 = item.blk * P.gbrows, r1 = min(n, r0 + P.gbrows);
    const int kk2 = k * k;
    double dv[CT];
    bool cok[CT];
    int cc[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int c = t * 16 + r16;
      cok[t] = c < k;
      cc[t] = cok[t] ? c : 0;
      dv[t] = *gld(P.vec + VEC_D * k + cc[t]);
    }
    double rsq[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) rsq[t] = 0.0;

    // phase 0: rows < k (only block 0 has them); phase 1: rows >= k
    for (int phase = 0; phase < 2; ++phase) {
      const int lo = phase == 0 ? r0 : max(r0, k);
      const int hi = phase == 0 ? min(r1, k) : r1;
      if (lo >= hi) continue;
      v4d accP[NTP], accG[NTG];
#pragma unroll
      for (int t = 0; t < NTP; ++t) accP[t] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < NTG; ++t) accG[t] = v4d{0.0, 0.0, 0.0, 0.0};
      for (int base = lo + rg * 4 * U; base < hi; base += RG * 4 * U) {
        double xv[U][CT], wv[U][CT], lv[U][CT];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int row = base + 4 * u + g;
          const int rr = row < hi ? row : lo;
#pragma unroll
          for (int t = 0; t < CT; ++t) {
            xv[u][t] = *gld(X + (int64_t)rr * ldx + cc[t]);
            wv[u][t] = *gld(Wh + (int64_t)rr * k + cc[t]);
            lv[u][t] = LO ? *gld(Wl + (int64_t)rr * k + cc[t]) : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int row = base + 4 * u + g;
          const bool rok = row < hi;
          double xm[CT], rv[CT];
#pragma unroll
          for (int t = 0; t < CT; ++t) {
            const bool ok = rok && cok[t];
            xm[t] = ok ? xv[u][t] : 0.0;
            rv[t] = ok ? residual(wv[u][t], has_lo ? lv[u][t] : 0.0, xv[u][t], dv[t], has_lo) : 0.0;
            rsq[t] = __builtin_fma(rv[t], rv[t], rsq[t]);
          }
#pragma unroll
          for (int ti = 0; ti < CT; ++ti) {
            if (ti < ct_used) {
#pragma unroll
              for (int t = 0; t < CT; ++t) {
                if (t < ct_used) {
                  accP[ti * CT + t] = mfma_f64(xm[ti], rv[t], accP[ti * CT + t]);
                  if (t >= ti) {
                    const int gi = ti * CT - ti * (ti - 1) / 2 + (t - ti);
                    accG[gi] = mfma_f64(xm[ti], xm[t], accG[gi]);
                  }
                }
              }
            }
          }
          if (phase == 0 && rok) {
#pragma unroll
            for (int t = 0; t < CT; ++t)
              if (cok[t]) *gst(P.kk + KK_R1 * kk2 + row * k + t * 16 + r16) = rv[t];
          }
        }
      }
      // sum the wavefronts' tiles into wavefront 0, one tile at a time
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
      for (int q = 0; q < NTP + NTG; ++q) {
        v4d& v = q < NTP ? accP[q] : accG[q - NTP];
        // tile indices of q
        int ti, t;
        if (q < NTP) {
          ti = q / CT;
          t = q % CT;
        } else {
          const int gi = q - NTP;
          ti = gi < CT ? 0 : 1;
          t = ti + (gi - (ti == 0 ? 0 : CT));
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) xch[rg][lane * 4 + r] = v[r];
        __syncthreads();
        if (rg == 0 && ti < ct_used && t < ct_used) {
          double sum[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            double a = xch[0][lane * 4 + r];
            for (int w = 1; w < RG; ++w) a += xch[w][lane * 4 + r];
            sum[r] = a;
          }
          const int c = t * 16 + r16;
          if (c < k) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = ti * 16 + mfma_row(g, r);
              if (i < k) {
                *gst((q < NTP ? dstP : dstG) + i * k + c) = sum[r];
                // X1^T X1 is read in full: its lower tile mirrored
                if (q >= NTP && phase == 0 && ti < t) *gst(dstG + c * k + i) = sum[r];
              }
            }
          }
        }
        __syncthreads();
      }
    }
    // blocks without rows >= k still publish zero partials
    if (max(r0, k) >= r1) {
      double* dst = P.gpart + (int64_t)item.blk * (2 * kk2 + k);
      for (int e = threadIdx.x; e < 2 * kk2; e += blockDim.x) *gst(dst + e) = 0.0;
    }
    // column sums of r^2 over the block's rows
#pragma unroll
    for (int t = 0; t < CT; ++t) rsq_x[rg][t * 64 + lane] = rsq[t];
    __syncthreads();
    if (threadIdx.x < CT * 16) {
      const int t = threadIdx.x / 16, c16 = threadIdx.x % 16, c = t * 16 + c16;
      if (c < k) {
        double s = 0.0;
        for (int q = 0; q < RG; ++q)
          s += (rsq_x[q][t * 64 + c16] + rsq_x[q][t * 64 + 16 + c16]) +
               (rsq_x[q][t * 64 + 32 + c16] + rsq_x[q][t * 64 + 48 + c16]);
        *gst(P.gpart + (int64_t)item.blk * (2 * kk2 + k) + 2 * kk2 + c) = s;
      }
    }
    __syncthreads();
  }
}

// Sums the Gram partials of every problem in a fixed order over blocks:
// 64 slots per workgroup, 16 block groups per slot, then an LDS tree.  Slots
// [0, k^2) are X2^T R2, [k^2, 2k^2) X2^T X2 (lower tiles mirrored from the
// upper ones), [2k^2, 2k^2 + k) the column sums of r^2.
struct GramRedItem {
  int32_t prob, s0;
};
__global__ __launch_bounds__(1024) void gram_reduce_kernel(const Prob* __restrict__ probs,
                                                           const GramRedItem* __restrict__ items,
                                                           int nitems) {
  __shared__ double sh[16][64];
  const int c = threadIdx.x & 63, bg = threadIdx.x >> 6;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const GramRedItem item = items[it];
    const Prob& P = probs[item.prob];
    if (P.ctrl->stopped) continue;
    const int k = P.k, kk2 = k * k, S = 2 * kk2 + k;
    const int s = item.s0 + c;
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    if (s < S) {
      int src = s;
      if (s >= kk2 && s < 2 * kk2) {
        const int e = s - kk2, i = e / k, j = e % k;
        if (i / 16 > j / 16) src = kk2 + j * k + i;
      }
      const int nb = P.ngb;
      int b = bg;
      for (; b + 48 < nb; b += 64) {
        const double v0 = *gld(P.gpart + (int64_t)b * S + src);
        const double v1 = *gld(P.gpart + (int64_t)(b + 16) * S + src);
        const double v2 = *gld(P.gpart + (int64_t)(b + 32) * S + src);
        const double v3 = *gld(P.gpart + (int64_t)(b + 48) * S + src);
        acc0 += v0;
        acc1 += v1;
        acc2 += v2;
        acc3 += v3;
      }
      for (; b < nb; b += 16) acc0 += *gld(P.gpart + (int64_t)b * S + src);
    }
    sh[bg][c] = (acc0 + acc1) + (acc2 + acc3);
    __syncthreads();
    for (int h = 8; h >= 1; h /= 2) {
      if (bg < h) sh[bg][c] += sh[bg + h][c];
      __syncthreads();
    }
    if (bg == 0 && s < S) {
      const double acc = sh[0][c];
      if (s < kk2)
        P.kk[KK_P2 * kk2 + s] = acc;
      else if (s < 2 * kk2)
        P.kk[KK_G2 * kk2 + (s - kk2)] = acc;
      else
        P.vec[VEC_RSQ * k + (s - 2 * kk2)] = acc;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// pass 3: update of the bottom rows on the matrix cores (32 < k <= 64).
// Each wavefront owns 16 rows; the B operand [M | N] (k x 2k) is staged
// whole in LDS and shared by the block's four wavefronts; A is the X row
// block.  The epilogue's X, W and W_lo are requested with the A operand,
// before the products.  The block writes per-column partials of sum x~^2
// and sum e^2; fin_stats finishes them.  (Past k = 64: update_wide_kernel.)
// FUSED (one problem through the panel pipeline, after pp_q_kernel and
// fin_post_kernel): the B operand is C = M Delta + N alone, and an accepted
// step writes the normalised iterate into X, as in update_wide_kernel.
// ---------------------------------------------------------------------------
template <int CT, bool FUSED>
__global__ __launch_bounds__(256) void update_kernel(const Prob* __restrict__ probs,
                                                    const RowItem* __restrict__ items, int nitems) {
  static_assert(CT <= 4, "k <= 64");
  constexpr int NT = 256, WAVES = 4, KCH = 64, BW = (FUSED ? 1 : 2) * CT * 16, LDC = BW + 2;
  __shared__ double Cs[KCH * LDC];
  __shared__ double colred[2][WAVES][CT * 16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem item = items[it];
    const Prob& P = probs[item.prob];
    if (FUSED ? !P.ctrl->apply : P.ctrl->stopped) continue;
    const int n = P.n, k = P.k, kk2 = k * k, k2 = 2 * k;
    const bool has_lo = P.wlo != nullptr;
    const double* __restrict__ X = P.x;
    const int64_t ldx = P.ldx;
    const double* __restrict__ Cm = P.kk + KK_CM * kk2;
    const double* __restrict__ Cf = P.kk + KK_FC * kk2;
    const double* __restrict__ X1n = P.kk + KK_X1N * kk2;
    const int r0 = item.blk * P.rbrows, r1 = min(n, r0 + P.rbrows);
    double dv[CT], di[CT], sc[CT], xsq[CT], esq[CT];
    bool cok[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int c = t * 16 + r16;
      cok[t] = c < k;
      dv[t] = ld_or0(cok[t], P.vec + VEC_D * k, c);
      di[t] = ld_or0(cok[t], P.vec + VEC_DINV * k, c);
      sc[t] = FUSED ? ld_or0(cok[t], P.vec + VEC_SCALE * k, c) : 1.0;
      xsq[t] = 0.0;
      esq[t] = 0.0;
    }
    const double* wlb = has_lo ? P.wlo : P.w;  // a readable base either way
    // stage [M | N] (FUSED: C) (columns padded to 16 CT), sixteen loads per
    // thread issued before their LDS stores
    {
      constexpr int PER = (KCH * BW + NT - 1) / NT, BAT = PER < 16 ? PER : 16;
#pragma unroll 1
      for (int u0 = 0; u0 < PER; u0 += BAT) {
        double v[BAT];
#pragma unroll
        for (int u = 0; u < BAT; ++u) {
          const int e = tid + (u0 + u) * NT;
          const int rr = e / BW, cc = e - rr * BW;
          const int half = cc / (CT * 16), cj = cc - half * (CT * 16);
          // rows past k meet zero A values and columns past k are not
          // written, so those entries need only be finite: they repeat row
          // and column 0 (an unmasked load does not wait on the one before)
          if constexpr (FUSED)
            v[u] = *gld(Cf + (rr < k ? rr : 0) * k + (cj < k ? cj : 0));
          else
            v[u] = *gld(Cm + (rr < k ? rr : 0) * k2 + half * k + (cj < k ? cj : 0));
        }
#pragma unroll
        for (int u = 0; u < BAT; ++u) {
          const int e = tid + (u0 + u) * NT;
          if (e < KCH * BW) Cs[(e / BW) * LDC + e % BW] = v[u];
        }
      }
    }
    __syncthreads();
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
      // the A operand (all of K), then the epilogue's X, W and W_lo
      constexpr int AQ = KCH / 4;
      double a_ch[AQ];
#pragma unroll
      for (int q = 0; q < AQ; ++q) {
        const int kk = 4 * q + g;
        a_ch[q] = ld_or0(arok && kk < k, xr, kk);
      }
      double ex[CT][4], ew[CT][4], el[CT][4];
#pragma unroll
      for (int t = 0; t < CT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rc + wave * 16 + mfma_row(g, r);
          const bool ok = cok[t] && row < r1 && row >= k;
          const int64_t o = (int64_t)row * k + t * 16 + r16;
          ex[t][r] = ld_or0(ok, X, (int64_t)row * ldx + t * 16 + r16);
          ew[t][r] = ld_or0(ok, P.w, o);
          el[t][r] = ld_or0(ok && has_lo, wlb, o);
        }
      for (int kc = 0; kc < k; kc += 16) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const double av = a_ch[kc / 4 + s];
          const double* brow = Cs + (kc + 4 * s + g) * LDC + r16;
#pragma unroll
          for (int t = 0; t < CT; ++t) {
            accM[t] = mfma_f64(av, brow[t * 16], accM[t]);
            if constexpr (!FUSED) accN[t] = mfma_f64(av, brow[CT * 16 + t * 16], accN[t]);
          }
        }
      }
      // epilogue: register r holds row rc + wave*16 + mfma_row(g, r), column t*16 + r16
#pragma unroll
      for (int t = 0; t < CT; ++t) {
        const int c = t * 16 + r16;
        if (cok[t]) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = rc + wave * 16 + mfma_row(g, r);
            if (row < r1) {
              double xt;
              if (row < k) {
                xt = *gld(X1n + row * k + c);
              } else if constexpr (FUSED) {
                const double x = ex[t][r];
                const double rr = residual(ew[t][r], el[t][r], x, dv[t], has_lo);
                xt = __builtin_fma(rr, di[t], x) - accM[t][r];
              } else {
                const double x = ex[t][r];
                const double rr = residual(ew[t][r], el[t][r], x, dv[t], has_lo);
                const double e = (rr - accM[t][r]) * di[t];
                xt = (x + e) - accN[t][r];
                esq[t] = __builtin_fma(e, e, esq[t]);
              }
              if constexpr (FUSED) {
                *gst(P.x + (int64_t)row * ldx + c) = xt * sc[t];
              } else {
                *gst(P.xn + (int64_t)row * k + c) = xt;
                xsq[t] = __builtin_fma(xt, xt, xsq[t]);
              }
            }
          }
        }
      }
    }
    // block partials of sum x~^2 and sum e^2 per column
    if constexpr (FUSED) continue;
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
      *gst(P.part + (int64_t)item.blk * stride + 2 * k + tid) = a;
      *gst(P.part + (int64_t)item.blk * stride + 3 * k + tid) = b;
    }
    __syncthreads();
  }
}

// The same pass for 64 < k <= 128 (CT 5..8): one 64-row tile of X at a time
// in LDS (read once, with consecutive threads on consecutive entries),
// shared by the block's four wavefronts.  Wavefront w owns the column tiles
// w and w + 4 of X~ for all 64 rows, so it needs only the matching columns
// of M and N, which it streams from L2 (the same for every tile) DB K-steps
// ahead of its products; W and W_lo of its entries are requested with the
// tile.  Each wavefront's products are 4 row tiles x 2 column tiles x {M, N},
// the same count for every wavefront at k = 128, against the staging of all
// of [M | N] through LDS in the form above.  Rows past the item's end and
// columns past k are clamped (finite, never stored); the tile's columns from
// k to the next multiple of 4 are zero, which bounds the contraction.
//
// FUSED (after pp_q_kernel and fin_post_kernel, which formed the statistics,
// the scale factors and the decision from k x k quantities): an accepted
// step writes the normalised iterate straight into X (each block reads its
// rows before it overwrites them), from the one product X~2 = X2 + R2 Delta
// - X2 C with C = M Delta + N, so each wavefront streams only its columns of
// C and does half the products, with no partial sums and no normalisation
// pass afterwards.
template <int CT, bool FUSED>
__global__ __launch_bounds__(256) void update_wide_kernel(const Prob* __restrict__ probs,
                                                         const RowItem* __restrict__ items, int nitems) {
  constexpr int WAVES = 4, TW = 2, ROWS = 64, LDX = KMAX + 4, DB = FUSED ? 8 : 4;
  static_assert(CT > 4 && CT <= WAVES * TW, "64 < k <= 128");
  __shared__ double Xs[ROWS * LDX];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem item = items[it];
    const Prob& P = probs[item.prob];
    if (FUSED ? !P.ctrl->apply : P.ctrl->stopped) continue;
    const int n = P.n, k = P.k, kk2 = k * k, k2 = 2 * k;
    const int kq = (k + 3) / 4, kp = 4 * kq;
    const bool has_lo = P.wlo != nullptr;
    const double* __restrict__ X = P.x;
    const int64_t ldx = P.ldx;
    const double* __restrict__ Cm = P.kk + KK_CM * kk2;
    const double* __restrict__ Cf = P.kk + KK_FC * kk2;
    const double* __restrict__ X1n = P.kk + KK_X1N * kk2;
    const double* wlb = has_lo ? P.wlo : P.w;  // a readable base either way
    const int r0 = item.blk * P.rbrows, r1 = min(n, r0 + P.rbrows);
    // this wavefront's columns
    int cc[TW];
    bool cok[TW];
    double dv[TW], di[TW], sc[TW], xsq[TW], esq[TW];
#pragma unroll
    for (int u = 0; u < TW; ++u) {
      const int c = (wave + WAVES * u) * 16 + r16;
      cok[u] = c < k;
      cc[u] = cok[u] ? c : k - 1;
      dv[u] = *gld(P.vec + VEC_D * k + cc[u]);
      di[u] = *gld(P.vec + VEC_DINV * k + cc[u]);
      sc[u] = FUSED ? *gld(P.vec + VEC_SCALE * k + cc[u]) : 1.0;
      xsq[u] = 0.0;
      esq[u] = 0.0;
    }
    const bool busy = wave < (k + 15) / 16;  // owns at least one column tile
    for (int rc = r0; rc < r1; rc += ROWS) {
      __syncthreads();  // the previous tile's LDS reads are done
      // the X tile (rows past r1 repeat row r1 - 1), columns to kp: wavefront
      // w reads rows 16w..16w+15, lane l columns l and l + 64, all at once
      {
        double xv[16][2];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int row = min(rc + wave * 16 + i, r1 - 1);
#pragma unroll
          for (int h = 0; h < 2; ++h) xv[i][h] = *gld(X + (int64_t)row * ldx + min(lane + 64 * h, k - 1));
        }
#pragma unroll
        for (int i = 0; i < 16; ++i)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int col = lane + 64 * h;
            if (col < kp) Xs[(wave * 16 + i) * LDX + col] = col < k ? xv[i][h] : 0.0;
          }
      }
      // W and W_lo of this wavefront's entries
      double wv[4][TW][4], lv[4][TW][4];
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int u = 0; u < TW; ++u)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = min(rc + rt * 16 + mfma_row(g, r), r1 - 1);
            const int64_t o = (int64_t)row * k + cc[u];
            wv[rt][u][r] = *gld(P.w + o);
            lv[rt][u][r] = *gld(wlb + o);
          }
      v4d accM[4][TW], accN[4][TW];
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int u = 0; u < TW; ++u) {
          accM[rt][u] = v4d{0.0, 0.0, 0.0, 0.0};
          accN[rt][u] = v4d{0.0, 0.0, 0.0, 0.0};
        }
      // B fragments of K-step q: lane l holds [M | N](4q + l/16, column)
      // (FUSED: C(4q + l/16, column) in the first array)
      double bM[DB][TW], bN[DB][TW];
      auto load_b = [&](int q, double(&m)[TW], double(&nn)[TW]) {
        const int kr = min(4 * q + g, k - 1);
#pragma unroll
        for (int u = 0; u < TW; ++u) {
          if constexpr (FUSED) {
            m[u] = *gld(Cf + (unsigned)(kr * k + cc[u]));
          } else {
            m[u] = *gld(Cm + (unsigned)(kr * k2 + cc[u]));
            nn[u] = *gld(Cm + (unsigned)(kr * k2 + k + cc[u]));
          }
        }
      };
#pragma unroll
      for (int s = 0; s < DB; ++s) load_b(s, bM[s], bN[s]);
      __syncthreads();  // the tile is in LDS
      if (busy) {
        for (int q0 = 0; q0 < kq; q0 += DB) {
#pragma unroll
          for (int s = 0; s < DB; ++s) {
            const int q = q0 + s;
            if (q < kq) {
              double a[4];
#pragma unroll
              for (int rt = 0; rt < 4; ++rt) a[rt] = Xs[(rt * 16 + r16) * LDX + 4 * q + g];
#pragma unroll
              for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                for (int u = 0; u < TW; ++u) {
                  if (wave + WAVES * u < CT) {
                    accM[rt][u] = mfma_f64(a[rt], bM[s][u], accM[rt][u]);
                    if constexpr (!FUSED) accN[rt][u] = mfma_f64(a[rt], bN[s][u], accN[rt][u]);
                  }
                }
              load_b(q + DB, bM[s], bN[s]);  // clamped past k: harmless
            }
          }
        }
      }
      // epilogue: register r of tile (rt, u) holds row rc + rt*16 + mfma_row(g, r)
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int u = 0; u < TW; ++u) {
          const int c = (wave + WAVES * u) * 16 + r16;
          if (cok[u]) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int lr = rt * 16 + mfma_row(g, r), row = rc + lr;
              if (row < r1) {
                double xt;
                if (row < k) {
                  xt = *gld(X1n + row * k + c);
                } else if constexpr (FUSED) {
                  const double x = Xs[lr * LDX + c];
                  const double rr = residual(wv[rt][u][r], lv[rt][u][r], x, dv[u], has_lo);
                  xt = __builtin_fma(rr, di[u], x) - accM[rt][u][r];
                } else {
                  const double x = Xs[lr * LDX + c];
                  const double rr = residual(wv[rt][u][r], lv[rt][u][r], x, dv[u], has_lo);
                  const double e = (rr - accM[rt][u][r]) * di[u];
                  xt = (x + e) - accN[rt][u][r];
                  esq[u] = __builtin_fma(e, e, esq[u]);
                }
                if constexpr (FUSED) {
                  *gst(P.x + (int64_t)row * ldx + c) = xt * sc[u];
                } else {
                  *gst(P.xn + (int64_t)row * k + c) = xt;
                  xsq[u] = __builtin_fma(xt, xt, xsq[u]);
                }
              }
            }
          }
        }
    }
    // block partials of sum x~^2 and sum e^2 per column (this wavefront's)
    if constexpr (FUSED) continue;
    const int stride = 5 * k;
#pragma unroll
    for (int u = 0; u < TW; ++u) {
      double a = xsq[u], b = esq[u];
      a += __shfl_xor(a, 16);
      a += __shfl_xor(a, 32);
      b += __shfl_xor(b, 16);
      b += __shfl_xor(b, 32);
      const int c = (wave + WAVES * u) * 16 + r16;
      if (g == 0 && c < k) {
        *gst(P.part + (int64_t)item.blk * stride + 2 * k + c) = a;
        *gst(P.part + (int64_t)item.blk * stride + 3 * k + c) = b;
      }
    }
  }
}

// The same pass for k <= 32 (CT <= 2), for long problems: the block's X rows
// come in 64-row tiles read with coalesced 16-byte loads (one tile ahead, in
// registers) into LDS, where the wavefronts take both the MFMA A operand
// (16 rows x 4 columns per step) and the epilogue's x from them, so X is read
// from memory once and in whole rows.  W (and W_lo) are read in the
// epilogue's layout before the products.  [M | N] is staged once per block.
//
// FUSED (with fin_pre_kernel before it): the step's statistics, scale factors
// and acceptance are already known, so an accepted step writes the
// normalised iterate straight into X (each block reads its rows before it
// overwrites them, and no other block reads them), with no partial sums and
// no normalisation pass afterwards.  E21 itself is then not needed, so the
// bottom rows take one product, X~2 = X2 + R2 Delta - X2 (M Delta + N), half
// the matrix-core work of X2 M and X2 N.
template <int CT, bool FUSED>
__global__ __launch_bounds__(256) void update_small_kernel(const Prob* __restrict__ probs,
                                                          const RowItem* __restrict__ items,
                                                          int nitems) {
  typedef double v2d __attribute__((ext_vector_type(2)));
  static_assert(CT <= 2, "tall-skinny form");
  constexpr int NT = 256, WAVES = 4, TR = 64, KP = CT * 16, LDXS = KP + 1;
  // fused: one product X2 C with C = M Delta + N (the form of the statistics
  // formed before the update); otherwise X2 M and X2 N, since E21 is needed
  constexpr int BW = (FUSED ? 1 : 2) * KP, LDC = BW + 2;
  constexpr int UNITS = TR * KP / 2, UPT = (UNITS + NT - 1) / NT;  // 2-double units per tile
  __shared__ double Cs[KP * LDC];
  __shared__ double Xs[TR * LDXS];
  __shared__ double colred[2][WAVES][KP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem item = items[it];
    const Prob& P = probs[item.prob];
    if (FUSED ? !P.ctrl->apply : P.ctrl->stopped) continue;
    const int n = P.n, k = P.k, kk2 = k * k, k2 = 2 * k;
    const bool has_lo = P.wlo != nullptr;
    const double* X = P.x;  // written in place in the fused form
    const int64_t ldx = P.ldx;
    const double* __restrict__ Cm = P.kk + KK_CM * kk2;
    const double* __restrict__ X1n = P.kk + KK_X1N * kk2;
    const int r0 = item.blk * P.rbrows, r1 = min(n, r0 + P.rbrows);
    const bool vec = (ldx & 1) == 0 && (((uintptr_t)X) & 15) == 0 && (k & 1) == 0;
    double dv[CT], di[CT], xsq[CT], esq[CT], sc[CT];
    bool cok[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int c = t * 16 + r16;
      cok[t] = c < k;
      const int cc = cok[t] ? c : 0;
      dv[t] = *gld(P.vec + VEC_D * k + cc);
      di[t] = cok[t] ? *gld(P.vec + VEC_DINV * k + cc) : 0.0;
      sc[t] = FUSED ? *gld(P.vec + VEC_SCALE * k + cc) : 1.0;
      xsq[t] = 0.0;
      esq[t] = 0.0;
    }
    // [M | N] (or C = M Delta + N) rows < KP (zero past k)
    for (int e = tid; e < KP * BW; e += NT) {
      const int rr = e / BW, cc = e - rr * BW;
      const int half = cc / KP, cj = cc - half * KP;
      double v = 0.0;
      if (rr < k && cj < k) {
        if (FUSED)
          v = __builtin_fma(*gld(Cm + rr * k2 + cj), *gld(P.vec + VEC_DINV * k + cj),
                            *gld(Cm + rr * k2 + k + cj));
        else
          v = *gld(Cm + rr * k2 + half * k + cj);
      }
      Cs[rr * LDC + cc] = v;
    }
    // one 64-row tile of X as UPT pairs of doubles per thread (zero past n or k)
    auto load_tile = [&](int rc, v2d (&buf)[UPT]) {
#pragma unroll
      for (int u = 0; u < UPT; ++u) {
        const int e = min(tid + u * NT, UNITS - 1);
        const int rr = e / (KP / 2), c = 2 * (e - rr * (KP / 2));
        const int row = min(rc + rr, r1 - 1);
        const double* p = X + (int64_t)row * ldx;
        if (vec && c + 1 < k) {
          buf[u] = *gld(reinterpret_cast<const v2d*>(p + c));
        } else {
          buf[u].x = *gld(p + min(c, k - 1));
          buf[u].y = *gld(p + min(c + 1, k - 1));
        }
      }
    };
    v2d nxt[UPT];
    load_tile(r0, nxt);
    for (int rc = r0; rc < r1; rc += TR) {
      __syncthreads();  // previous tile's LDS reads (and the [M | N] stores) are done
#pragma unroll
      for (int u = 0; u < UPT; ++u) {
        const int e = tid + u * NT;
        if (e < UNITS) {
          const int rr = e / (KP / 2), c = 2 * (e - rr * (KP / 2));
          const bool rok = rc + rr < r1;
          Xs[rr * LDXS + c] = (rok && c < k) ? nxt[u].x : 0.0;
          Xs[rr * LDXS + c + 1] = (rok && c + 1 < k) ? nxt[u].y : 0.0;
        }
      }
      if (rc + TR < r1) load_tile(rc + TR, nxt);
      // the epilogue's W values of this wavefront's 16 rows
      double ew[CT][4], el[CT][4];
#pragma unroll
      for (int t = 0; t < CT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = min(rc + wave * 16 + mfma_row(g, r), r1 - 1);
          const int64_t o = (int64_t)row * k + (cok[t] ? t * 16 + r16 : 0);
          ew[t][r] = *gld(P.w + o);
          el[t][r] = has_lo ? *gld(P.wlo + o) : 0.0;
        }
      __syncthreads();
      v4d accM[CT], accN[CT];
#pragma unroll
      for (int t = 0; t < CT; ++t) {
        accM[t] = v4d{0.0, 0.0, 0.0, 0.0};
        accN[t] = v4d{0.0, 0.0, 0.0, 0.0};
      }
      const double* xa = Xs + (wave * 16 + r16) * LDXS + g;
#pragma unroll
      for (int s = 0; s < KP / 4; ++s) {
        const double av = xa[4 * s];
        const double* brow = Cs + (4 * s + g) * LDC + r16;
#pragma unroll
        for (int t = 0; t < CT; ++t) {
          accM[t] = mfma_f64(av, brow[t * 16], accM[t]);
          if (!FUSED) accN[t] = mfma_f64(av, brow[KP + t * 16], accN[t]);
        }
      }
      // epilogue: register r holds row rc + wave*16 + mfma_row(g, r), column t*16 + r16
#pragma unroll
      for (int t = 0; t < CT; ++t) {
        const int c = t * 16 + r16;
        if (cok[t]) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int lr = wave * 16 + mfma_row(g, r), row = rc + lr;
            if (row < r1) {
              double xt;
              if (row < k) {
                xt = *gld(X1n + row * k + c);
              } else {
                const double x = Xs[lr * LDXS + c];
                const double rr = residual(ew[t][r], el[t][r], x, dv[t], has_lo);
                if (FUSED) {
                  // x + r / (d - mu) - (x C)_j, the two small terms first
                  xt = x + __builtin_fma(rr, di[t], -accM[t][r]);
                } else {
                  const double e = (rr - accM[t][r]) * di[t];
                  xt = (x + e) - accN[t][r];
                  esq[t] = __builtin_fma(e, e, esq[t]);
                }
              }
              if (FUSED) {
                *gst(P.x + (int64_t)row * ldx + c) = xt * sc[t];
              } else {
                *gst(P.xn + (int64_t)row * k + c) = xt;
                xsq[t] = __builtin_fma(xt, xt, xsq[t]);
              }
            }
          }
        }
      }
    }
    if (FUSED) continue;
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
      *gst(P.part + (int64_t)item.blk * stride + 2 * k + tid) = a;
      *gst(P.part + (int64_t)item.blk * stride + 3 * k + tid) = b;
    }
    __syncthreads();
  }
}

// Statistics and the accept/reject decision of the step, one workgroup per
// problem: sums the update partials (fixed order), forms the normalisation
// factors 1/||x~_j||, ||E_L||_F = sqrt(||E11||_F^2 + sum e^2) and
// ||R||_F / ||A||, and applies the stopping and divergence rules.
__global__ __launch_bounds__(1024) void fin_stats_kernel(const Prob* __restrict__ probs, int nprob) {
  constexpr int NT = 1024, NW = NT / 64;
  __shared__ double tot[2 * KMAX];
  __shared__ double scr[NT];
  __shared__ double fin[2][NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int p = blockIdx.x; p < nprob; p += gridDim.x) {
    const Prob& P = probs[p];
    __syncthreads();
    if (P.ctrl->stopped) continue;
    const int k = P.k, stride = 5 * k;
    team_reduce(P.part + 2 * k, stride, 2 * k, P.nrb, scr, tot);
    double e2 = 0.0, r2 = 0.0;
    int bad = 0;
    for (int j = tid; j < k; j += NT) {
      const double xs = tot[j];
      P.vec[VEC_SCALE * k + j] = P.normalize ? 1.0 / sqrt(xs) : 1.0;
      if (!__builtin_isfinite(xs) || !(xs > 0.0)) bad = 1;
      e2 += tot[k + j];
      r2 += P.vec[VEC_RSQ * k + j];
    }
    for (int o = 32; o >= 1; o /= 2) {
      e2 += __shfl_xor(e2, o);
      r2 += __shfl_xor(r2, o);
    }
    if (lane == 0) {
      fin[0][wave] = e2;
      fin[1][wave] = r2;
    }
    bad = __syncthreads_or(bad);
    if (tid == 0) {
      Ctrl* C = P.ctrl;
      double se = P.vec[VEC_E1SQ * k], sr = 0.0;
      for (int w = 0; w < NW; ++w) {
        se += fin[0][w];
        sr += fin[1][w];
      }
      const double corr = sqrt(se);
      const double resid = sqrt(sr) / P.norm_a;
      C->corr_fro = corr;
      C->resid_rel = resid;
      const bool finite = !bad && __builtin_isfinite(corr) && __builtin_isfinite(resid);
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
        C->rr_top = 0;  // a Rayleigh-Ritz basis serves one step
        C->hist[h & 3] = corr;
        C->iters = h + 1;
        if ((C->stop_mode == 1 && corr <= C->tol) || (C->stop_mode == 2 && resid <= C->tol)) {
          C->converged = 1;
          C->stopped = 1;
        }
      }
    }
  }
}

// The decision of a fused step from its column norms in LDS, colv0[j] =
// ||x~_j||^2 and colv1[j] = ||e21_j||^2 (j < k): the normalisation factors,
// ||E_L||_F, ||R||_F / ||A|| and the rules of fin_stats_kernel.  All threads
// of the block call it; fin holds 2 (blockDim / 64) doubles of LDS.
__device__ void fused_decide(const Prob& P, const double* colv0, const double* colv1, double* fin) {
  const int NT = blockDim.x, NW = NT / 64, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int k = P.k;
  Ctrl* C = P.ctrl;
  const double* rsq = P.vec + VEC_RSQ * k;
  double e2 = 0.0, r2 = 0.0;
  int bad = 0;
  for (int j = tid; j < k; j += NT) {
    const double xs = colv0[j];
    P.vec[VEC_SCALE * k + j] = P.normalize ? 1.0 / sqrt(xs) : 1.0;
    if (!__builtin_isfinite(xs) || !(xs > 0.0)) bad = 1;
    e2 += colv1[j];
    r2 += *gld(rsq + j);
  }
  for (int o = 32; o >= 1; o /= 2) {
    e2 += __shfl_xor(e2, o);
    r2 += __shfl_xor(r2, o);
  }
  if (lane == 0) {
    fin[wave] = e2;
    fin[NW + wave] = r2;
  }
  bad = __syncthreads_or(bad);
  if (tid == 0) {
    double se = P.vec[VEC_E1SQ * k], sr = 0.0;
    for (int w = 0; w < NW; ++w) {
      se += fin[w];
      sr += fin[NW + w];
    }
    const double corr = sqrt(se);
    const double resid = sqrt(sr) / P.norm_a;
    C->corr_fro = corr;
    C->resid_rel = resid;
    const bool finite = !bad && __builtin_isfinite(corr) && __builtin_isfinite(resid);
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
      C->rr_top = 0;  // a Rayleigh-Ritz basis serves one step
      C->hist[h & 3] = corr;
      C->iters = h + 1;
      if ((C->stop_mode == 1 && corr <= C->tol) || (C->stop_mode == 2 && resid <= C->tol)) {
        C->converged = 1;
        C->stopped = 1;
      }
    }
  }
}

// Statistics, normalisation factors and the accept/reject decision before
// the update, for k <= 32, one workgroup per problem.  The bottom rows update
// as X~2 = X2 A + R2 Delta with A = I - N - M Delta and Delta =
// diag(1/(d - mu)), so every column norm the step needs is a quadratic form
// in k x k quantities it already has:
//   ||x~_j||^2  = ||x~1_j||^2 + a_j^T G2 a_j + 2 Delta_j a_j^T p_j + Delta_j^2 s_j,
//   ||e21_j||^2 = Delta_j^2 (s_j - 2 m_j^T p_j + m_j^T G2 m_j),
// with G2 = X2^T X2, p_j and m_j the columns j of X2^T R2 and of M, and
// s_j = ||r2_j||^2 (the column sum of r^2 less the leading rows).  The terms
// are small corrections to a_j^T G2 a_j ~ 1 or sums of squares, so the
// factors are accurate to a few rounding errors.  The rules applied are those
// of fin_stats_kernel; the fused update then writes the normalised iterate.
constexpr int FP_K = 32;
__global__ __launch_bounds__(256) void fin_pre_kernel(const Prob* __restrict__ probs, int nprob) {
  constexpr int NT = 256, NW = NT / 64, LD = FP_K + 1;
  __shared__ double Gs[FP_K * LD], Ps[FP_K * LD], As[FP_K * LD], Ms[FP_K * LD];
  __shared__ double colv[2][FP_K];
  __shared__ double fin[2][NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int p = blockIdx.x; p < nprob; p += gridDim.x) {
    const Prob& P = probs[p];
    Ctrl* C = P.ctrl;
    __syncthreads();
    if (tid == 0) C->apply = 0;
    if (C->stopped) continue;
    const int k = P.k, kk2 = k * k, k2 = 2 * k;
    const double* G2 = P.kk + KK_G2 * kk2;
    const double* P2 = P.kk + KK_P2 * kk2;
    const double* Cm = P.kk + KK_CM * kk2;
    const double* X1n = P.kk + KK_X1N * kk2;
    const double* R1 = P.kk + KK_R1 * kk2;
    const double* dinv = P.vec + VEC_DINV * k;
    const double* rsq = P.vec + VEC_RSQ * k;
    for (int e = tid; e < kk2; e += NT) {
      const int i = e / k, j = e - i * k;
      const double m = *gld(Cm + i * k2 + j), nn = *gld(Cm + i * k2 + k + j);
      Gs[i * LD + j] = *gld(G2 + e);
      Ps[i * LD + j] = *gld(P2 + e);
      Ms[i * LD + j] = m;
      As[i * LD + j] = (i == j ? 1.0 : 0.0) - nn - m * *gld(dinv + j);
    }
    __syncthreads();
    // eight threads per column j, each over the rows l = part, part + 8, ...
    {
      const int j = tid / 8, part = tid % 8;
      double sA = 0.0, sM = 0.0, pA = 0.0, pM = 0.0, top = 0.0, r1 = 0.0;
      if (j < k) {
        for (int l = part; l < k; l += 8) {
          double qa = 0.0, qm = 0.0;
          for (int m = 0; m < k; ++m) {
            const double gv = Gs[l * LD + m];
            qa = __builtin_fma(gv, As[m * LD + j], qa);
            qm = __builtin_fma(gv, Ms[m * LD + j], qm);
          }
          const double al = As[l * LD + j], ml = Ms[l * LD + j], pl = Ps[l * LD + j];
          sA = __builtin_fma(al, qa, sA);
          sM = __builtin_fma(ml, qm, sM);
          pA = __builtin_fma(al, pl, pA);
          pM = __builtin_fma(ml, pl, pM);
          const double xt = *gld(X1n + l * k + j), rt = *gld(R1 + l * k + j);
          top = __builtin_fma(xt, xt, top);
          r1 = __builtin_fma(rt, rt, r1);
        }
      }
#pragma unroll
      for (int o = 1; o < 8; o *= 2) {
        sA += __shfl_xor(sA, o);
        sM += __shfl_xor(sM, o);
        pA += __shfl_xor(pA, o);
        pM += __shfl_xor(pM, o);
        top += __shfl_xor(top, o);
        r1 += __shfl_xor(r1, o);
      }
      if (j < k && part == 0) {
        const double D = *gld(dinv + j);
        const double s2 = fmax(*gld(rsq + j) - r1, 0.0);
        colv[0][j] = top + sA + 2.0 * D * pA + D * D * s2;
        colv[1][j] = fmax(D * D * (s2 - 2.0 * pM + sM), 0.0);
      }
    }
    __syncthreads();
    fused_decide(P, colv[0], colv[1], &fin[0][0]);
  }
}

// The same statistics for one problem through the panel pipeline (k > 32),
// one workgroup after pp_q_kernel: per column j, the panels' parts of the
// quadratic forms, ||x~1_j||^2 and ||r1_j||^2 summed in a fixed order, then
// the norms of fin_pre_kernel and the decision.
__global__ __launch_bounds__(1024) void fin_post_kernel(const Prob* __restrict__ probs) {
  constexpr int NT = 1024, NW = NT / 64, TPC = 8;  // threads per column: one per panel
  __shared__ double colv[2][KMAX];
  __shared__ double fin[2 * NW];
  const Prob& P = probs[0];
  const int tid = threadIdx.x;
  if (P.ctrl->stopped) return;  // set before this launch: the same in every thread
  const int k = P.k, kk2 = k * k, np = (k + 15) / 16;
  const double* Qp = P.kk + KK_FQ * kk2;
  const int j = tid / TPC, part = tid % TPC;
  const int jc = j < k ? j : k - 1;
  double q[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) q[c] = ld_or0(part < np, Qp, (int64_t)(part * 6 + c) * k + jc);
#pragma unroll
  for (int o = 1; o < TPC; o *= 2)
#pragma unroll
    for (int c = 0; c < 6; ++c) q[c] += __shfl_xor(q[c], o);
  if (j < k && part == 0) {
    const double sA = q[0], sM = q[1], pA = q[2], pM = q[3], top = q[4], r1 = q[5];
    const double D = *gld(P.vec + VEC_DINV * k + j);
    const double s2 = fmax(*gld(P.vec + VEC_RSQ * k + j) - r1, 0.0);
    colv[0][j] = top + sA + 2.0 * D * pA + D * D * s2;
    colv[1][j] = fmax(D * D * (s2 - 2.0 * pM + sM), 0.0);
  }
  __syncthreads();
  fused_decide(P, colv[0], colv[1], fin);
}

// Rayleigh quotients, one workgroup per problem: sums the partials of
// x_j^T w_j and x_j^T x_j (fixed order) and forms d_j (eq. Rayleigh),
// alpha_j = x_j^T x_j and 1/(d_j - mu).
__global__ __launch_bounds__(1024) void fin_d_kernel(const Prob* __restrict__ probs, int nprob) {
  constexpr int NT = 1024;
  __shared__ double tot[2 * KMAX];
  __shared__ double totx[2 * KMAX];
  __shared__ double scr[NT];
  const int tid = threadIdx.x;
  for (int p = blockIdx.x; p < nprob; p += gridDim.x) {
    const Prob& P = probs[p];
    __syncthreads();
    if (P.ctrl->stopped) continue;
    const int k = P.k;
    team_reduce(P.dpart, 2 * k, 2 * k, P.ndp, scr, tot);
    // squared variant: x^T A^2 x = ||A x||^2 (A symmetric) is the second
    // product's input norm, x^T x the first product's
    if (P.square) team_reduce(P.dpx, 2 * k, 2 * k, P.ndp, scr, totx);
    int bad = 0;
    for (int j = tid; j < k; j += NT) {
      const double a = P.square ? totx[k + j] : tot[k + j];
      const double d = (P.square ? tot[k + j] : tot[j]) / a;
      P.vec[VEC_D * k + j] = d;
      P.vec[VEC_ALPHA * k + j] = a;
      P.vec[VEC_DINV * k + j] = 1.0 / (d - P.mu);
      if (!__builtin_isfinite(d) || !(a > 0.0)) bad = 1;
    }
    if (__syncthreads_or(bad) && tid == 0) {
      P.ctrl->status = -6;
      P.ctrl->stopped = 1;
    }
  }
}

// Split-K sum for dense A: W = sum of the ksplit partial products in split
// order; each thread sums two adjacent doubles of every partial (n*k even
// keeps the paired loads aligned; an odd tail element is summed alone).
__global__ __launch_bounds__(256) void wsum_kernel(const Prob* __restrict__ probs, int p) {
  typedef double v2d __attribute__((ext_vector_type(2)));
  const Prob& P = probs[p];
  if (P.ctrl->stopped) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nk = (int64_t)P.n * P.k;
  const int S = P.ksplit;
  if (nk % 2 == 0 && 2 * i + 1 < nk) {
    const v2d* src = reinterpret_cast<const v2d*>(P.wp) + i;
    const int64_t st = nk / 2;
    v2d v[16];
#pragma unroll
    for (int s = 0; s < 16; ++s)
      if (s < S) v[s] = src[s * st];
    v2d w = v[0];
#pragma unroll
    for (int s = 1; s < 16; ++s)
      if (s < S) w += v[s];
    reinterpret_cast<v2d*>(P.w)[i] = w;
  } else {
    for (int64_t e = 2 * i; e < 2 * i + 2 && e < nk; ++e) {
      double w = P.wp[e];
      for (int s = 1; s < S; ++s) w += P.wp[e + s * nk];
      P.w[e] = w;
    }
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

// lo: W carries a low part (the split forms).
hipError_t launch_gram(const Prob* probs, const RowItem* items, int nitems, int kmax, bool lo,
                       hipStream_t st) {
  const int ct = (kmax + 15) / 16;
  if (ct <= 2) {
#define RFK_GRAM_ALL(CTV, LOV)                                                                     \
  hipLaunchKernelGGL((gram_all_kernel<CTV, 8, 4, LOV>), dim3(nitems), dim3(512), 0, st, probs, items, \
                     nitems)
    if (ct == 1 && lo)
      RFK_GRAM_ALL(1, true);
    else if (ct == 1)
      RFK_GRAM_ALL(1, false);
    else if (lo)
      RFK_GRAM_ALL(2, true);
    else
      RFK_GRAM_ALL(2, false);
#undef RFK_GRAM_ALL
    return hipGetLastError();
  }
#define RFK_CASE(CTV)                                                                               \
  case CTV:                                                                                         \
    if (lo)                                                                                         \
      hipLaunchKernelGGL((gram_tile_kernel<CTV, 4, 4, true>), dim3(nitems), dim3(256), 0, st, probs, \
                         items, nitems);                                                            \
    else                                                                                            \
      hipLaunchKernelGGL((gram_tile_kernel<CTV, 4, 4, false>), dim3(nitems), dim3(256), 0, st, probs, \
                         items, nitems);                                                            \
    break;
  switch (ct) {
    RFK_CASE(3) RFK_CASE(4) RFK_CASE(5) RFK_CASE(6) RFK_CASE(7) RFK_CASE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef RFK_CASE
  return hipGetLastError();
}

hipError_t launch_gram_reduce(const Prob* probs, const GramRedItem* items, int nitems,
                              hipStream_t st) {
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(nitems), dim3(1024), 0, st, probs, items, nitems);
  return hipGetLastError();
}

// fused: X written in place, normalised, after the statistics were formed
// from k x k quantities: k <= 32 (fin_pre_kernel has run) or k > 32 (one
// problem through the panel pipeline; pp_q_kernel and fin_post_kernel).
hipError_t launch_update(const Prob* probs, const RowItem* items, int nitems, int kmax, bool fused,
                         hipStream_t st) {
  const int ct = (kmax + 15) / 16;
  if (ct <= 2) {
    const dim3 grid(nitems), block(256);
    if (ct == 1 && fused)
      hipLaunchKernelGGL((update_small_kernel<1, true>), grid, block, 0, st, probs, items, nitems);
    else if (ct == 1)
      hipLaunchKernelGGL((update_small_kernel<1, false>), grid, block, 0, st, probs, items, nitems);
    else if (fused)
      hipLaunchKernelGGL((update_small_kernel<2, true>), grid, block, 0, st, probs, items, nitems);
    else
      hipLaunchKernelGGL((update_small_kernel<2, false>), grid, block, 0, st, probs, items, nitems);
    return hipGetLastError();
  }
#define RFK_CASE(CTV)                                                                          \
  case CTV:                                                                                    \
    if (fused)                                                                                 \
      hipLaunchKernelGGL((update_kernel<CTV, true>), dim3(nitems), dim3(256), 0, st, probs, items, \
                         nitems);                                                              \
    else                                                                                       \
      hipLaunchKernelGGL((update_kernel<CTV, false>), dim3(nitems), dim3(256), 0, st, probs,     \
                         items, nitems);                                                       \
    break;
#define RFK_WIDE(CTV)                                                                           \
  case CTV:                                                                                     \
    if (fused)                                                                                  \
      hipLaunchKernelGGL((update_wide_kernel<CTV, true>), dim3(nitems), dim3(256), 0, st, probs,  \
                         items, nitems);                                                        \
    else                                                                                        \
      hipLaunchKernelGGL((update_wide_kernel<CTV, false>), dim3(nitems), dim3(256), 0, st, probs, \
                         items, nitems);                                                        \
    break;
  switch (ct) {
    RFK_CASE(3) RFK_CASE(4) RFK_WIDE(5) RFK_WIDE(6) RFK_WIDE(7) RFK_WIDE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef RFK_CASE
#undef RFK_WIDE
  return hipGetLastError();
}

hipError_t launch_wsum(const Prob* probs, int p, int64_t n, int k, hipStream_t st) {
  const int64_t npairs = (n * k + 1) / 2;
  hipLaunchKernelGGL(wsum_kernel, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, st, probs, p);
  return hipGetLastError();
}

hipError_t launch_fin_d(const Prob* probs, int nprob, hipStream_t st) {
  hipLaunchKernelGGL(fin_d_kernel, dim3(nprob), dim3(1024), 0, st, probs, nprob);
  return hipGetLastError();
}

hipError_t launch_fin_post(const Prob* probs, hipStream_t st) {
  hipLaunchKernelGGL(fin_post_kernel, dim3(1), dim3(1024), 0, st, probs);
  return hipGetLastError();
}

hipError_t launch_fin_pre(const Prob* probs, int nprob, hipStream_t st) {
  hipLaunchKernelGGL(fin_pre_kernel, dim3(nprob), dim3(256), 0, st, probs, nprob);
  return hipGetLastError();
}

hipError_t launch_fin_stats(const Prob* probs, int nprob, hipStream_t st) {
  hipLaunchKernelGGL(fin_stats_kernel, dim3(nprob), dim3(1024), 0, st, probs, nprob);
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

