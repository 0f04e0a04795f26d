// Line 1 of Algorithm 4 for dense A: W = A X on the FP64 matrix cores.
//
// Shape: A is n x n (streamed once from HBM), X is n x k with k <= 128, so
// the product is a tall-skinny GEMM whose work per byte of A is k/4 flop/B.
// Design for gfx950:
//   * one wavefront owns 16 rows of A and all BN = 16*CT columns of W; its
//     A fragments are loaded straight from global memory into registers
//     (16 rows x 64 contiguous bytes per lane group, full 128-byte lines per
//     two chunks), so A never touches LDS and each A element feeds CT MFMAs;
//   * the X chunk (32 x BN) is shared by the WAVES wavefronts of a workgroup
//     through a double-buffered LDS tile (row stride BN+2 doubles to spread
//     the four lane groups over different banks);
//   * v_mfma_f64_16x16x4_f64: each lane holds a[row = l%16][k = l/16] and
//     b[k = l/16][col = l%16] (result layout: see mfma_row in common.h); the
//     K index inside a 32-wide chunk is permuted
//     identically for A and B (lane group g uses k = 8g + m for step m), which
//     leaves the sum unchanged and lets a lane read 8 contiguous doubles;
//   * split-K over the work-item table gives enough workgroups to fill 256
//     CUs; items are ordered on the host so that blockIdx % 8 (the XCD that
//     runs the block) fixes the K range, keeping each XCD's X chunk in its L2.
#include "common.h"

namespace rfk {

template <int CT, int WAVES, int RT, int KC, bool BLDS, bool VEC2>
__global__ __launch_bounds__(WAVES * 64) void gemm_f64_kernel(const Prob* __restrict__ probs,
                                                             const GemmItem* __restrict__ items,
                                                             int nitems) {
  constexpr int BN = CT * 16;
  constexpr int AM = KC / 4;       // K values per lane group per chunk
  constexpr int LDB = BN + 2;
  constexpr int NT = WAVES * 64;
  constexpr int BPT = (KC * BN + NT - 1) / NT;  // X chunk elements per thread
  constexpr int BM = WAVES * RT * 16;
  __shared__ double Bs[BLDS ? 2 : 1][BLDS ? KC * LDB : 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r16 = lane & 15;

  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const GemmItem item = items[it];
    const Prob& P = probs[item.prob];
    if (P.ctrl->stopped) continue;  // uniform over the block
    const int n = P.n, k = P.k;
    const double* __restrict__ A = P.a;
    const int64_t lda = P.lda;
    const double* __restrict__ X = P.x;
    const int64_t ldx = P.ldx;
    const int k0 = item.k0, k1 = item.k1;
    const double* arow[RT];
    bool row_ok[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int row = item.row0 + (wave * RT + rt) * 16 + r16;
      row_ok[rt] = row < n;
      arow[rt] = A + (int64_t)(row_ok[rt] ? row : 0) * lda;
    }

    v4d acc[RT][CT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[rt][c] = v4d{0.0, 0.0, 0.0, 0.0};

    double a_cur[RT][AM], a_nxt[RT][AM];
    double bst[BLDS ? BPT : 1];

    auto load_a = [&](double (*dst)[AM], int kb) {
      const int kk = kb + AM * g;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        if (kb + KC <= k1) {
          if (VEC2) {
            typedef double v2d __attribute__((ext_vector_type(2)));
            const v2d* p = reinterpret_cast<const v2d*>(arow[rt] + kk);
#pragma unroll
            for (int m = 0; m < AM / 2; ++m) {
              v2d v = __builtin_nontemporal_load(p + m);
              dst[rt][2 * m] = v.x;
              dst[rt][2 * m + 1] = v.y;
            }
          } else {
#pragma unroll
            for (int m = 0; m < AM; ++m) dst[rt][m] = arow[rt][kk + m];
          }
        } else {
#pragma unroll
          for (int m = 0; m < AM; ++m) dst[rt][m] = (kk + m < k1) ? arow[rt][kk + m] : 0.0;
        }
        if (!row_ok[rt]) {
#pragma unroll
          for (int m = 0; m < AM; ++m) dst[rt][m] = 0.0;
        }
      }
    };
    auto load_b = [&](int kb) {
#pragma unroll
      for (int s = 0; s < BPT; ++s) {
        const int e = tid + s * NT;
        const int kr = e / BN, col = e - kr * BN;
        double v = 0.0;
        if (e < KC * BN && kb + kr < k1 && col < k) v = X[(int64_t)(kb + kr) * ldx + col];
        bst[s] = v;
      }
    };
    auto store_b = [&](int buf) {
#pragma unroll
      for (int s = 0; s < BPT; ++s) {
        const int e = tid + s * NT;
        if (e < KC * BN) {
          const int kr = e / BN, col = e - kr * BN;
          Bs[buf][kr * LDB + col] = bst[s];
        }
      }
    };

    const int nchunks = (k1 - k0 + KC - 1) / KC;
    load_a(a_cur, k0);
    if (BLDS) {
      load_b(k0);
      store_b(0);
      __syncthreads();
    }
    for (int c = 0; c < nchunks; ++c) {
      const int buf = c & 1;
      const bool more = c + 1 < nchunks;
      const int kb = k0 + c * KC;
      if (more) {
        load_a(a_nxt, kb + KC);
        if (BLDS) load_b(kb + KC);
      }
      if (BLDS) {
        const double* bs = &Bs[buf][0];
#pragma unroll
        for (int m = 0; m < AM; ++m) {
          const double* brow = bs + (AM * g + m) * LDB + r16;
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            const double bv = brow[ct * 16];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) acc[rt][ct] = mfma_f64(a_cur[rt][m], bv, acc[rt][ct]);
          }
        }
        if (more) store_b(buf ^ 1);
        __syncthreads();
      } else {
        // B fragments straight from X (shared by the block's wavefronts in L1)
#pragma unroll
        for (int m = 0; m < AM; ++m) {
          const int kr = kb + AM * g + m;
          const bool kok = kr < k1;
          const double* xr = X + (int64_t)(kok ? kr : k0) * ldx + r16;
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            const double bv = (kok && ct * 16 + r16 < k) ? xr[ct * 16] : 0.0;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) acc[rt][ct] = mfma_f64(a_cur[rt][m], bv, acc[rt][ct]);
          }
        }
      }
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int m = 0; m < AM; ++m) a_cur[rt][m] = a_nxt[rt][m];
    }

    // Epilogue: register r of the lane holds row mfma_row(g, r), column r16
    // of each 16x16 tile.
    double* __restrict__ out = (P.ksplit > 1) ? P.wp + (int64_t)item.split * n * k : P.w;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int orow = item.row0 + (wave * RT + rt) * 16;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int col = ct * 16 + r16;
        if (col < k) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int orr = orow + mfma_row(g, r);
            if (orr < n) out[(int64_t)orr * k + col] = acc[rt][ct][r];
          }
        }
      }
    }
  }
}

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
  constexpr int TT = 16 * 17;      // epilogue transpose tile per wavefront (doubles)
  constexpr int BUF = (2 * KC * LDB > WAVES * TT) ? 2 * KC * LDB : WAVES * TT;
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

    double a_cur[KS][RT], a_nxt[KS][RT];
    double bst[BPT];

    auto load_a = [&](double (*dst)[RT], int kb) {
      const bool full = (kb + KC <= k1) && (jl + RT <= n);
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int kk = kb + 4 * s + g;
        if (full) {
          const double* p = A + (int64_t)kk * lda + jl;
          if (VECA && RT == 2) {
            typedef double v2d __attribute__((ext_vector_type(2)));
            const v2d v = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(p));
            dst[s][0] = v.x;
            dst[s][RT - 1] = v.y;
          } else {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) dst[s][rt] = __builtin_nontemporal_load(p + rt);
          }
        } else {
          const bool kok = kk < k1;
          const double* p = A + (int64_t)(kok ? kk : k0) * lda;
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) dst[s][rt] = (kok && jl + rt < n) ? p[jl + rt] : 0.0;
        }
      }
    };
    auto load_b = [&](int kb) {
#pragma unroll
      for (int s = 0; s < BPT; ++s) {
        const int e = tid + s * NT;
        const int kr = e / BN, col = e - kr * BN;
        double v = 0.0;
        if (e < KC * BN && kb + kr < k1 && col < k) v = X[(int64_t)(kb + kr) * ldx + col];
        bst[s] = v;
      }
    };
    auto store_b = [&](double* dst) {
#pragma unroll
      for (int s = 0; s < BPT; ++s) {
        const int e = tid + s * NT;
        if (e < KC * BN) {
          const int kr = e / BN, col = e - kr * BN;
          dst[kr * LDB + col] = bst[s];
        }
      }
    };

    const int nchunks = (k1 - k0 + KC - 1) / KC;
    load_a(a_cur, k0);
    load_b(k0);
    store_b(Bs0);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
      const bool more = c + 1 < nchunks;
      const int kb = k0 + c * KC;
      const double* bs = (c & 1) ? Bs1 : Bs0;
      if (more) {
        load_a(a_nxt, kb + KC);
        load_b(kb + KC);
      }
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const double* xr = bs + (4 * s + g) * LDB + r16;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const double xv = xr[ct * 16];
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) acc[rt][ct] = mfma_f64(xv, a_cur[s][rt], acc[rt][ct]);
        }
      }
      if (more) store_b((c & 1) ? Bs0 : Bs1);
      __syncthreads();
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) a_cur[s][rt] = a_nxt[s][rt];
    }

    // Epilogue: register r of tile (rt, ct) holds W^T[ct*16 + mfma_row(g, r)][column
    // j0 + RT*r16 + rt], i.e. W[j0 + RT*r16 + rt][ct*16 + mfma_row(g, r)].  Each
    // tile is transposed through a per-wavefront 16x17 LDS buffer (the X chunk
    // buffers are free after the last barrier) so that every W row segment of
    // 16 doubles is written by four lanes, 32 contiguous bytes each.
    double* tw = smem + wave * TT;
    double* __restrict__ out = (P.ksplit > 1) ? P.wp + (int64_t)item.split * n * k : P.w;
    const int tc = lane >> 2, tq = lane & 3;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int row = j0 + RT * tc + rt;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
        for (int r = 0; r < 4; ++r) tw[r16 * 17 + mfma_row(g, r)] = acc[rt][ct][r];
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = tw[tc * 17 + 4 * tq + u];
        if (row < n) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int col = ct * 16 + 4 * tq + u;
            if (col < k) out[(int64_t)row * k + col] = v[u];
          }
        }
      }
    }
    __syncthreads();
  }
}

// Launch configurations: wavefronts per block, row tiles per wavefront,
// K chunk, and whether the X chunk goes through LDS (else through L1).
// Configurations 6.. use the transposed kernel (rt = interleaved A tiles).
struct GemmCfg {
  int waves, rt, kc, blds;
};
static const GemmCfg kGemmCfgs[] = {
    {8, 1, 32, 1}, {8, 1, 32, 0}, {4, 2, 32, 1}, {4, 2, 32, 0}, {8, 1, 64, 1}, {4, 1, 32, 0},
    {8, 1, 32, 1}, {8, 2, 32, 1}, {4, 2, 32, 1}, {4, 1, 32, 1}, {8, 2, 16, 1},
    {8, 1, 64, 1}, {16, 1, 32, 1}, {4, 1, 64, 1},
};
constexpr int kNumGemmCfgs = sizeof(kGemmCfgs) / sizeof(kGemmCfgs[0]);

int gemm_num_cfgs() { return kNumGemmCfgs; }
int gemm_rows_per_block(int cfg) { return kGemmCfgs[cfg].waves * kGemmCfgs[cfg].rt * 16; }

template <int CT, bool VEC2>
static hipError_t launch_ct(int cfg, const Prob* probs, const GemmItem* items, int nitems,
                            hipStream_t st) {
  switch (cfg) {
#define RFK_G(ID, W, R, K, L)                                                                \
  case ID:                                                                                   \
    hipLaunchKernelGGL((gemm_f64_kernel<CT, W, R, K, L, VEC2>), dim3(nitems), dim3(W * 64), 0, \
                       st, probs, items, nitems);                                            \
    break;
    RFK_G(0, 8, 1, 32, true)
    RFK_G(1, 8, 1, 32, false)
    RFK_G(2, 4, 2, 32, true)
    RFK_G(3, 4, 2, 32, false)
    RFK_G(4, 8, 1, 64, true)
    RFK_G(5, 4, 1, 32, false)
#undef RFK_G
#define RFK_T(ID, W, R, K)                                                                   \
  case ID:                                                                                   \
    hipLaunchKernelGGL((gemm_f64_t_kernel<CT, W, R, K, VEC2>), dim3(nitems), dim3(W * 64), 0, \
                       st, probs, items, nitems);                                            \
    break;
    RFK_T(6, 8, 1, 32)
    RFK_T(7, 8, 2, 32)
    RFK_T(8, 4, 2, 32)
    RFK_T(9, 4, 1, 32)
    RFK_T(10, 8, 2, 16)
    RFK_T(11, 8, 1, 64)
    RFK_T(12, 16, 1, 32)
    RFK_T(13, 4, 1, 64)
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
