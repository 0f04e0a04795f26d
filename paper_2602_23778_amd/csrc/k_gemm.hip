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

template <int CT, int WAVES, bool VEC2>
__global__ __launch_bounds__(WAVES * 64) void gemm_f64_kernel(const Prob* __restrict__ probs,
                                                             const GemmItem* __restrict__ items,
                                                             int nitems) {
  constexpr int BN = CT * 16;
  constexpr int KC = 32;
  constexpr int LDB = BN + 2;
  constexpr int NT = WAVES * 64;
  constexpr int BPT = (KC * BN + NT - 1) / NT;  // X chunk elements per thread
  __shared__ double Bs[2][KC * LDB];

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
    const int row = item.row0 + wave * 16 + r16;
    const bool row_ok = row < n;
    const double* __restrict__ arow = A + (int64_t)(row_ok ? row : 0) * lda;

    v4d acc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};

    double a_cur[8], a_nxt[8];
    double bst[BPT];

    auto load_a = [&](double* dst, int kb) {
      const int kk = kb + 8 * g;
      if (kb + KC <= k1) {
        if (VEC2) {
          typedef double v2d __attribute__((ext_vector_type(2)));
          const v2d* p = reinterpret_cast<const v2d*>(arow + kk);
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            v2d v = __builtin_nontemporal_load(p + m);
            dst[2 * m] = v.x;
            dst[2 * m + 1] = v.y;
          }
        } else {
#pragma unroll
          for (int m = 0; m < 8; ++m) dst[m] = arow[kk + m];
        }
      } else {
#pragma unroll
        for (int m = 0; m < 8; ++m) dst[m] = (kk + m < k1) ? arow[kk + m] : 0.0;
      }
      if (!row_ok) {
#pragma unroll
        for (int m = 0; m < 8; ++m) dst[m] = 0.0;
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
    load_b(k0);
    store_b(0);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
      const int buf = c & 1;
      const bool more = c + 1 < nchunks;
      if (more) {
        load_a(a_nxt, k0 + (c + 1) * KC);
        load_b(k0 + (c + 1) * KC);
      }
      const double* bs = &Bs[buf][0];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const double* brow = bs + (8 * g + m) * LDB + r16;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[ct] = mfma_f64(a_cur[m], brow[ct * 16], acc[ct]);
      }
      if (more) store_b(buf ^ 1);
      __syncthreads();
#pragma unroll
      for (int m = 0; m < 8; ++m) a_cur[m] = a_nxt[m];
    }

    // Epilogue: register r of the lane holds row mfma_row(g, r), column r16
    // of each 16x16 tile.
    double* __restrict__ out = (P.ksplit > 1) ? P.wp + (int64_t)item.split * n * k : P.w;
    const int orow = item.row0 + wave * 16;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int col = ct * 16 + r16;
      if (col < k) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int orr = orow + mfma_row(g, r);
          if (orr < n) out[(int64_t)orr * k + col] = acc[ct][r];
        }
      }
    }

  }
}

// Host launcher: picks the column-tile count from the largest k in the
// batch and the vector width from the alignment of every A.
hipError_t launch_gemm_f64(const Prob* probs, const GemmItem* items, int nitems, int grid,
                           int kmax, bool vec2, hipStream_t stream) {
  const int ct = (kmax + 15) / 16;
  constexpr int W = 8;
  dim3 block(W * 64);
#define RFK_GEMM_CASE(CTV)                                                                       \
  case CTV:                                                                                      \
    if (vec2)                                                                                    \
      hipLaunchKernelGGL((gemm_f64_kernel<CTV, W, true>), dim3(grid), block, 0, stream, probs,   \
                         items, nitems);                                                         \
    else                                                                                         \
      hipLaunchKernelGGL((gemm_f64_kernel<CTV, W, false>), dim3(grid), block, 0, stream, probs,  \
                         items, nitems);                                                         \
    break;
  switch (ct) {
    RFK_GEMM_CASE(1)
    RFK_GEMM_CASE(2)
    RFK_GEMM_CASE(3)
    RFK_GEMM_CASE(4)
    RFK_GEMM_CASE(5)
    RFK_GEMM_CASE(6)
    RFK_GEMM_CASE(7)
    RFK_GEMM_CASE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef RFK_GEMM_CASE
  return hipGetLastError();
}

int gemm_rows_per_block() { return 8 * 16; }

}  // namespace rfk
