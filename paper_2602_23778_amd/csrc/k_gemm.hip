// The product step of Algorithm 4 for dense A: W = A X on the FP64 matrix cores.
//
// Shape: A is n x n (streamed once from HBM), X is n x k with k <= 128, so
// the product is a tall-skinny GEMM whose work per byte of A is k/4 flop/B
// (16 flop/B at k = 64, just above the FP64 ridge of about 9.8 flop/B).
// Design for gfx950:
//   * the product is computed as W^T = X^T A (A is symmetric), which puts A
//     in the B operand of v_mfma_f64_16x16x4_f64: lane l supplies
//     b[k = l/16][j = l%16], so each load instruction reads whole 128-byte
//     segments of four A rows (the A-operand form reads 16 rows x 16 bytes and
//     measured 2.3 TB/s against 2.8 TB/s here); A goes straight from HBM to
//     registers, one chunk ahead, with non-temporal loads;
//   * each A value feeds CT = ceil(k/16) MFMAs (one per 16-column tile of X);
//     the X chunk (KC x 16 CT) is shared by the block's wavefronts through a
//     double-buffered LDS tile;
//   * split-K over the work-item table gives enough blocks to fill 256 CUs;
//     items are ordered so that blockIdx % 8 (the XCD that runs the block)
//     fixes the K range, keeping each XCD's X chunk in its L2;
//   * the epilogue transposes each 16x16 result tile through LDS and writes
//     whole W row segments, and adds the block's column sums of x*w (and of
//     x*x for the first K range) for the Rayleigh quotients;
//   * the launch configuration and K split are picked per shape by a
//     measuring tuner in the host runtime.
#include "common.h"
#include "dev_util.h"

namespace rfk {

// Transposed form W^T = X^T A (A is symmetric), which puts A in the MFMA B
// operand: for each 4-row K step, lane group g reads row kk+g of A at columns
// j0 + RT*(l%16) .. + RT-1, i.e. whole 128*RT-byte segments of A rows per
// instruction.  A wavefront owns RT interleaved 16-column tiles of A (RT*16
// rows of W); tile rt holds the columns j0 + RT*c + rt.  The X^T operand (row
// kk of X, 16 consecutive columns per lane group) comes from a double-buffered
// LDS chunk shared by the block.  The epilogue transposes the 16x16 result
// tiles through LDS so that W rows are written contiguously.
template <int CT, int WAVES, int RT, int KC, bool VECA>
__global__ __launch_bounds__(WAVES * 64) void gemm_f64_t_kernel(const Prob* __restrict__ probs,
                                                               const GemmItem* __restrict__ items,
                                                               int nitems) {
  constexpr int BN = CT * 16;      // columns of W (= k, padded)
  constexpr int KS = KC / 4;       // K steps per chunk
  constexpr int LDB = BN + 2;
  constexpr int NT = WAVES * 64;
  constexpr int BPT = (KC * BN + NT - 1) / NT;
  constexpr int WROWS = RT * 16;   // W rows per wavefront
  constexpr int BM = WAVES * WROWS;
  constexpr int TT = 16 * 17;      // epilogue transpose tile per wavefront (doubles)
  constexpr int EPI = WAVES * TT + 2 * WAVES * BN;   // transpose tiles + column sums
  constexpr int BUF = (2 * KC * LDB > EPI) ? 2 * KC * LDB : EPI;
  __shared__ double smem[BUF];
  double* Bs0 = smem;
  double* Bs1 = smem + KC * LDB;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r16 = lane & 15;

  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const GemmItem item = items[it];
    const Prob& P = probs[item.prob];
    if (P.ctrl->stopped) continue;
    const int n = P.n, k = P.k;
    const double* __restrict__ A = P.a;
    const int64_t lda = P.lda;
    const double* __restrict__ X = P.x;
    const int64_t ldx = P.ldx;
    const int k0 = item.k0, k1 = item.k1;
    const int j0 = item.row0 + wave * WROWS;    // first column of A (row of W) of this wave
    const int jl = j0 + RT * r16;                // this lane's first column
    // columns jl .. jl+RT-1 are valid when < n
    v4d acc[RT][CT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[rt][c] = v4d{0.0, 0.0, 0.0, 0.0};

    double a_s0[KS][RT], a_s1[KS][RT], a_s2[KS][RT];
    double bst[BPT];

    // Loads never branch and never write a register before the load itself:
    // rows past the K range are clamped to its last row (their X rows are
    // zero in LDS, so they add nothing) and columns past n to column n - 1
    // (their W rows are never stored).
    auto load_a = [&](double (*dst)[RT], int kb) {
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int kk = min(kb + 4 * s + g, k1 - 1);
        const double* p = A + (int64_t)kk * lda;
        if (VECA && RT == 2) {
          typedef double v2d __attribute__((ext_vector_type(2)));
          // the pair (jl, jl + 1), clamped to the last pair (n - 2, n - 1) of
          // the row; for odd n the lane whose jl is the last column n - 1
          // takes the pair's second entry (its second column, n, is never
          // stored).  Rows of odd leading dimension make every other pair
          // 8-byte aligned only, which gfx9 global loads accept.
          const v2d v = __builtin_nontemporal_load(gld(reinterpret_cast<const v2d*>(p + min(jl, n - 2))));
          dst[s][0] = jl == n - 1 ? v.y : v.x;
          dst[s][RT - 1] = v.y;
        } else {
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) dst[s][rt] = __builtin_nontemporal_load(gld(p + min(jl + rt, n - 1)));
        }
      }
    };
    auto load_b = [&](int kb) {
#pragma unroll
      for (int s = 0; s < BPT; ++s) {
        const int e = min(tid + s * NT, KC * BN - 1);
        const int kr = e / BN, col = e - kr * BN;
        bst[s] = *gld(X + (int64_t)min(kb + kr, k1 - 1) * ldx + min(col, k - 1));
      }
    };
    auto store_b = [&](double* dst, int kb) {
#pragma unroll
      for (int s = 0; s < BPT; ++s) {
        const int e = tid + s * NT;
        if (e < KC * BN) {
          const int kr = e / BN, col = e - kr * BN;
          dst[kr * LDB + col] = (kb + kr < k1 && col < k) ? bst[s] : 0.0;
        }
      }
    };

    // A is prefetched two chunks ahead through three register stages (the
    // chunk loop is unrolled by three so that every stage keeps its
    // registers).  Per chunk the X chunk of the next step is requested
    // before the A chunk two steps ahead, so the wait that precedes its LDS
    // store leaves the A requests in flight.  The loads and the store are
    // unconditional (past the K range they read the clamped last row and
    // store zeros), which keeps the compiler's wait counts exact across the
    // loop.
    const int nchunks = (k1 - k0 + KC - 1) / KC;
    load_b(k0);
    load_a(a_s0, k0);
    store_b(Bs0, k0);
    load_a(a_s1, k0 + KC);
    __syncthreads();
    auto chunk = [&](int c, double (*cur)[RT], double (*ahead)[RT]) {
      const int kb = k0 + c * KC;
      const double* bs = (c & 1) ? Bs1 : Bs0;
      load_b(kb + KC);
      load_a(ahead, kb + 2 * KC);
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const double* xr = bs + (4 * s + g) * LDB + r16;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const double xv = xr[ct * 16];
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) acc[rt][ct] = mfma_f64(xv, cur[s][rt], acc[rt][ct]);
        }
      }
      store_b((c & 1) ? Bs0 : Bs1, kb + KC);
      __syncthreads();
    };
    for (int c = 0; c < nchunks; c += 3) {
      chunk(c, a_s0, a_s2);
      if (c + 1 < nchunks) chunk(c + 1, a_s1, a_s0);
      if (c + 2 < nchunks) chunk(c + 2, a_s2, a_s1);
    }

    // Epilogue: register r of tile (rt, ct) holds W^T[ct*16 + mfma_row(g, r)][column
    // j0 + RT*r16 + rt], i.e. W[j0 + RT*r16 + rt][ct*16 + mfma_row(g, r)].  Each
    // tile is transposed through a per-wavefront 16x17 LDS buffer (the X chunk
    // buffers are free after the last barrier) so that every W row segment of
    // 16 doubles is written by four lanes, 32 contiguous bytes each.
    double* tw = smem + wave * TT;
    double* red = smem + WAVES * TT;  // [WAVES][2][BN]
    double* __restrict__ out = (P.ksplit > 1) ? P.wp + (int64_t)item.split * n * k : P.w;
    const int tc = lane >> 2, tq = lane & 3;
    // One column tile at a time, so that only its 4 + 4 partial sums are live.
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      double sxw[4] = {0.0, 0.0, 0.0, 0.0}, sxx[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int row = j0 + RT * tc + rt;
#pragma unroll
        for (int r = 0; r < 4; ++r) tw[r16 * 17 + mfma_row(g, r)] = acc[rt][ct][r];
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = tw[tc * 17 + 4 * tq + u];
        if (row < n) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int col = ct * 16 + 4 * tq + u;
            if (col < k) {
              *gst(out + (int64_t)row * k + col) = v[u];
              const double x = *gld(X + (int64_t)row * ldx + col);
              sxw[u] = __builtin_fma(x, v[u], sxw[u]);
              sxx[u] = __builtin_fma(x, x, sxx[u]);
            }
          }
        }
      }
      // Rayleigh partials of this item: column sums over its rows of x*w
      // (linear in w, so the K ranges add up) and of x*x (first K range
      // only).  Lanes with equal tq hold the same columns.
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        double a = sxw[u], b = sxx[u];
#pragma unroll
        for (int o = 4; o < 64; o *= 2) {
          a += __shfl_xor(a, o);
          b += __shfl_xor(b, o);
        }
        if (lane < 4) {
          red[(wave * 2) * BN + ct * 16 + 4 * lane + u] = a;
          red[(wave * 2 + 1) * BN + ct * 16 + 4 * lane + u] = b;
        }
      }
    }
    __syncthreads();
    if (tid < k) {
      double a = 0.0, b = 0.0;
      for (int w = 0; w < WAVES; ++w) {
        a += red[(w * 2) * BN + tid];
        b += red[(w * 2 + 1) * BN + tid];
      }
      double* dst = P.dpart + (int64_t)(item.row0 / BM * P.ksplit + item.split) * 2 * k;
      *gst(dst + tid) = a;
      *gst(dst + k + tid) = item.split == 0 ? b : 0.0;
    }
    __syncthreads();
  }
}

// Launch configurations: wavefronts per block, interleaved 16-column A tiles
// per wavefront, K chunk.
struct GemmCfg {
  int waves, rt, kc;
};
static const GemmCfg kGemmCfgs[] = {
    {8, 1, 32}, {8, 2, 32}, {4, 2, 32}, {4, 1, 32}, {8, 2, 16}, {8, 1, 64}, {16, 1, 32}, {4, 1, 64},
};
constexpr int kNumGemmCfgs = sizeof(kGemmCfgs) / sizeof(kGemmCfgs[0]);

int gemm_num_cfgs() { return kNumGemmCfgs; }
int gemm_rows_per_block(int cfg) { return kGemmCfgs[cfg].waves * kGemmCfgs[cfg].rt * 16; }

template <int CT, bool VEC2>
static hipError_t launch_ct(int cfg, const Prob* probs, const GemmItem* items, int nitems,
                            hipStream_t st) {
  switch (cfg) {
#define RFK_T(ID, W, R, K)                                                                   \
  case ID:                                                                                   \
    hipLaunchKernelGGL((gemm_f64_t_kernel<CT, W, R, K, VEC2>), dim3(nitems), dim3(W * 64), 0, \
                       st, probs, items, nitems);                                            \
    break;
    RFK_T(0, 8, 1, 32)
    RFK_T(1, 8, 2, 32)
    RFK_T(2, 4, 2, 32)
    RFK_T(3, 4, 1, 32)
    RFK_T(4, 8, 2, 16)
    RFK_T(5, 8, 1, 64)
    RFK_T(6, 16, 1, 32)
    RFK_T(7, 4, 1, 64)
#undef RFK_T
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Host launcher: the column-tile count comes from the largest k of the
// batch, the vector width from the alignment of every A.
hipError_t launch_gemm_f64(const Prob* probs, const GemmItem* items, int nitems, int kmax,
                           bool vec2, int cfg, hipStream_t stream) {
  const int ct = (kmax + 15) / 16;
#define RFK_CT(CTV)                                                                   \
  case CTV:                                                                           \
    return vec2 ? launch_ct<CTV, true>(cfg, probs, items, nitems, stream)             \
                : launch_ct<CTV, false>(cfg, probs, items, nitems, stream);
  switch (ct) {
    RFK_CT(1) RFK_CT(2) RFK_CT(3) RFK_CT(4) RFK_CT(5) RFK_CT(6) RFK_CT(7) RFK_CT(8)
    default:
      return hipErrorInvalidValue;
  }
#undef RFK_CT
}

}  // namespace rfk
