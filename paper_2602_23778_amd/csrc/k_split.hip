// Split form of the product step of Algorithm 4: W = A X by error-free splitting into
// INT8 digit slices with exact INT32 products on the matrix cores (the
// accelerator direction of Sec. 3.1.3; Ozaki, Ogita, Oishi and Rump 2012, with
// integer slices as in Ootomo, Ozaki and Yokota 2024).
//
// Slicing.  Row i of A gets the scale 2^E_i, column j of X the scale 2^F_j,
// E being the smallest integer with max |entry| < 2^E (0 for a zero line).
// A scaled value v = m 2^(6-E) in (-64, 64) is peeled into s digits by
// rounding to nearest: d = rint(v), v <- (v - d) 2^7, so every digit lies in
// [-64, 64] and m = 2^(E-6) sum_p d_p 2^(-7(p-1)) + r with |r| <= 2^(E-7s).
// Every step is exact in FP64.
//
// Product.  The digit products A_p X_q with p + q <= s + 1 (s(s+1)/2 of them)
// are summed exactly in INT32 into s bins by t = p + q, then
//     W_ij = 2^(E_i + F_j - 12) sum_t B_t 2^(-7(t-2))
// is formed in double-double (Horner in 2^-7 from the smallest bin) and
// stored as (W_hi, W_lo).  |digit products| <= 2^12, so a bin of at most s
// products over a contraction of length L stays below s 2^12 L < 2^31 for
// the K-split lengths the host allows.
//
// Layouts (bytes).  A slice unit = 16 consecutive columns of one row in one
// plane.  A row of a chunk of 32 columns holds the chunk's two halves, each as
// s planes of 16 bytes; the rows of one row block (bm rows, the product's
// block height) and one chunk are stored together, chunks of a row block one
// after another, so that the product reads each A tile as one contiguous
// run (nch = ceil(n/32); row i = bm*b + r, chunk c, half h, plane p at)
//     asl + ((b*nch + c)*bm + r)*32*s + h*16*s + p*16.
// X^T is stored the same way with the column j of X as the "row", the chunks
// outermost so that one chunk of all kpad columns is contiguous:
//     xsl + (c*kpad + j)*32*s + h*16*s + q*16.
// Rows of A are padded to a multiple of 256 and columns to nch*32 with zero
// digits; X^T likewise to kpad columns and nch*32 rows, so the product loop
// needs no bounds checks.
//
// Matrix-core tile: v_mfma_i32_32x32x32_i8 computes C[j][i] = sum_kk
// X^T[j][kk] A[i][kk], i.e. W^T, with the X slice in the A operand and the A
// slice in the B operand.  Both operands of a 32-wide contraction chunk are
// one 16-byte load per lane from the LDS tile.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <vector>

#include "dev_util.h"
#include "split.h"
#include "tune_cache.h"

namespace rfk {

typedef int v16i __attribute__((ext_vector_type(16)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// v_mfma_i32_32x32x32_i8 (gfx950), checked with a lane-layout probe: lane l
// supplies a[m = l%32][kk = 16(l/32) + b] and b[kk = 16(l/32) + b][n = l%32]
// for the bytes b = 0..15 of its 16-byte operand; register r of the result
// holds c[m = 8(r/4) + 4(l/32) + r%4][n = l%32].
__device__ __forceinline__ v16i mfma_i8(v4i a, v4i b, v16i c) {
  return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int mfma32_row(int lane, int r) {
  return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

// The s digits of 16 values sharing the scale 2^e, packed as s 16-byte
// planes (byte b of plane p = digit p of value b).
template <int S>
__device__ __forceinline__ void digits16(const double (&v)[16], int e, u4v (&out)[S]) {
#pragma unroll
  for (int p = 0; p < S; ++p) out[p] = u4v{0u, 0u, 0u, 0u};
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    double t = ldexp(v[b], 6 - e);
#pragma unroll
    for (int p = 0; p < S; ++p) {
      const double d = __builtin_rint(t);
      out[p][b >> 2] |= ((unsigned)(int)d & 0xffu) << (8 * (b & 3));
      t = ldexp(t - d, 7);
    }
  }
}

__device__ __forceinline__ int scale_exponent(double mx) {
  int e = 0;
  if (mx > 0.0) (void)frexp(mx, &e);  // mx = f 2^e, f in [1/2, 1): mx < 2^e
  return e;
}

// ---------------------------------------------------------------------------
// Slicing of A (once, at init)
// ---------------------------------------------------------------------------

// Row scales: one wavefront per row (rows >= n get 0).
__global__ __launch_bounds__(256) void split_aexp_kernel(const double* __restrict__ a, int64_t lda,
                                                         int n, int rows_pad,
                                                         int32_t* __restrict__ aexp) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows_pad) return;
  double m = 0.0;
  if (row < n)
    for (int c = lane; c < n; c += 64) m = fmax(m, fabs(a[(int64_t)row * lda + c]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if (lane == 0) aexp[row] = scale_exponent(m);
}

// Digits: one thread per 16-column unit (row, chunk, half).
template <int S>
__global__ __launch_bounds__(256) void split_aslice_kernel(const double* __restrict__ a,
                                                           int64_t lda, int n, int nch,
                                                           int rows_pad, int bm,
                                                           const int32_t* __restrict__ aexp,
                                                           uint8_t* __restrict__ asl) {
  const int64_t units = (int64_t)rows_pad * nch * 2;
  for (int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x; u < units;
       u += (int64_t)gridDim.x * 256) {
    const int row = (int)(u / (2 * nch));
    const int cu = (int)(u - (int64_t)row * 2 * nch);  // 2 * chunk + half
    const int col0 = cu * 16;
    double v[16];
#pragma unroll
    for (int b = 0; b < 16; ++b)
      v[b] = (row < n && col0 + b < n) ? a[(int64_t)row * lda + col0 + b] : 0.0;
    u4v out[S];
    digits16<S>(v, aexp[row], out);
    const int rb = row / bm, c = cu >> 1;
    u4v* dst = reinterpret_cast<u4v*>(
        asl + (((int64_t)rb * nch + c) * bm + (row - rb * bm)) * (32 * S) + (cu & 1) * 16 * S);
#pragma unroll
    for (int p = 0; p < S; ++p) dst[p] = out[p];
  }
}

// ---------------------------------------------------------------------------
// Slicing of X (every step)
// ---------------------------------------------------------------------------

// Column maxima of |X|: work item (problem, block of xrows rows); each block
// merges its maxima into the problem's xmaxp[j] with an atomic maximum on
// the bit patterns (for non-negative doubles the unsigned order of the bits
// is the numeric order, and a maximum does not depend on the order of the
// merges).  xmaxp is zeroed by the product kernel after use.
__global__ __launch_bounds__(256) void split_xmax_kernel(const Prob* __restrict__ probs,
                                                         const RowItem* __restrict__ items,
                                                         int nitems) {
  __shared__ double red[256];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem item = items[it];
    const Prob& P = probs[item.prob];
    if (P.ctrl->stopped) continue;
    const int k = P.k, kp = pow2ceil(k), rl = 256 / kp;
    const int tid = threadIdx.x, j = tid % kp, r = tid / kp;
    const int r0 = item.blk * P.xrows, r1 = min(P.n, r0 + P.xrows);
    double m = 0.0;
    if (j < k) {
      // eight independent loads in flight per thread
#pragma unroll 8
      for (int i = r0 + r; i < r1; i += rl) m = fmax(m, fabs(*gld(P.x + (int64_t)i * P.ldx + j)));
    }
    red[tid] = m;
    __syncthreads();
    for (int s = rl / 2; s > 0; s >>= 1) {
      if (r < s) red[tid] = fmax(red[tid], red[tid + s * kp]);
      __syncthreads();
    }
    if (tid < k)
      atomicMax(reinterpret_cast<unsigned long long*>(P.xmaxp) + tid,
                (unsigned long long)__double_as_longlong(red[tid]));
    __syncthreads();
  }
}

// Digits of X^T: work item (problem, 256 consecutive 16-row units), one
// thread per unit (chunk, column, half).
template <int S>
__global__ __launch_bounds__(256) void split_xslice_kernel(const Prob* __restrict__ probs,
                                                           const RowItem* __restrict__ items,
                                                           int nitems) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const RowItem item = items[it];
    const Prob& P = probs[item.prob];
    if (P.ctrl->stopped) continue;
    const int kpad = P.kpad, k = P.k, n = P.n;
    const int64_t units = (int64_t)P.nch * kpad * 2;
    const int64_t u = (int64_t)item.blk * 256 + threadIdx.x;
    if (u >= units) continue;
    const unsigned long long* mx = reinterpret_cast<const unsigned long long*>(P.xmaxp);
    const int h = (int)(u & 1);
    const int64_t cj = u >> 1;
    const int c = (int)(cj / kpad);
    const int j = (int)(cj - (int64_t)c * kpad);
    // the column maximum and the 16 entries are requested together (indices
    // clamped into X, entries past it masked to zero afterwards)
    const bool jok = j < k;
    const int jc = jok ? j : k - 1;
    const int r0 = c * 32 + h * 16;
    const unsigned long long mxj = *gld(mx + jc);
    double v[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) v[b] = *gld(P.x + (int64_t)min(r0 + b, n - 1) * P.ldx + jc);
#pragma unroll
    for (int b = 0; b < 16; ++b) v[b] = (jok && r0 + b < n) ? v[b] : 0.0;
    const int e = jok ? scale_exponent(__longlong_as_double((long long)mxj)) : 0;
    if (c == 0 && h == 0) P.xexp[j] = e;
    u4v out[S];
    digits16<S>(v, e, out);
    u4v* dst = reinterpret_cast<u4v*>(P.xsl + u * 16 * S);
#pragma unroll
    for (int p = 0; p < S; ++p) dst[p] = out[p];
  }
}

// ---------------------------------------------------------------------------
// The product
// ---------------------------------------------------------------------------

// Epilogue of one work item.  Register r of bin t holds B_t[j][i] for the
// column j = 32 wj + mfma32_row(lane, r) of W and the row i = row0 + 32 wi +
// l32.  Each (hi, lo) goes straight to the wavefront's two LDS transpose
// tiles, so that 32 lanes then write 32 consecutive columns of a row.  The
// LDS tiles must be idle on entry (every wave past the last barrier, no
// direct-to-LDS load in flight).
template <int S, int WM, int WN>
__device__ __forceinline__ void split_epilogue(const Prob& P, const GemmItem& item, v16i (&acc)[S],
                                               uint8_t* smem) {
  constexpr int NW = WM * WN, BM = 32 * WM, BN = 32 * WN;
  constexpr int TT = 32 * 33;  // transpose tile (doubles)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave / WN, wj = wave % WN;
  const int l32 = lane & 31, hh = lane >> 5;
  const int n = P.n, k = P.k, row0 = item.row0;
  const int ea = *gld(P.aexp + row0 + wi * 32 + l32);
  double* Th = reinterpret_cast<double*>(smem) + wave * 2 * TT;
  double* Tl = Th + TT;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    double h = (double)acc[S - 1][r], l = 0.0;
#pragma unroll
    for (int t = S - 2; t >= 0; --t) {
      double s, e;
      two_sum((double)acc[t][r], h * 0x1p-7, s, e);
      l = __builtin_fma(l, 0x1p-7, e);
      two_sum(s, l, h, l);
    }
    const int jr = mfma32_row(lane, r);
    const int sc = ea + *gld(P.xexp + wj * 32 + jr) - 12;
    Th[l32 * 33 + jr] = ldexp(h, sc);
    Tl[l32 * 33 + jr] = ldexp(l, sc);
  }
  __builtin_amdgcn_wave_barrier();
  const bool part = P.ksplit > 1;
  double* __restrict__ out_hi = part ? P.swp + (int64_t)item.split * 2 * n * k : P.w;
  double* __restrict__ out_lo = part ? out_hi + (int64_t)n * k : P.wlo;
  double* red = reinterpret_cast<double*>(smem) + NW * 2 * TT;  // [WM][2][BN]
  const int col = wj * 32 + l32;
  double sxw = 0.0, sxx = 0.0;
#pragma unroll 4
  for (int v = 0; v < 16; ++v) {
    const int il = 2 * v + hh;
    const int row = row0 + wi * 32 + il;
    if (row < n && col < k) {
      const double w = Th[il * 33 + l32];
      *gst(out_hi + (int64_t)row * k + col) = w;
      *gst(out_lo + (int64_t)row * k + col) = Tl[il * 33 + l32];
      const double x = *gld(P.x + (int64_t)row * P.ldx + col);
      sxw = __builtin_fma(x, w, sxw);
      sxx = __builtin_fma(x, x, sxx);
    }
  }
  // Rayleigh partials (x*w_hi over the block's rows; x*x for the first K range)
  sxw += __shfl_xor(sxw, 32);
  sxx += __shfl_xor(sxx, 32);
  if (lane < 32) {
    red[(wi * 2) * BN + col] = sxw;
    red[(wi * 2 + 1) * BN + col] = sxx;
  }
  __syncthreads();
  if (tid < k) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < WM; ++w) {
      a += red[(w * 2) * BN + tid];
      b += red[(w * 2 + 1) * BN + tid];
    }
    double* dst = P.dpart + (int64_t)(row0 / BM * P.ksplit + item.split) * 2 * k;
    *gst(dst + tid) = a;
    *gst(dst + k + tid) = item.split == 0 ? b : 0.0;
  }
}

// Block = WM x WN wavefronts; wavefront (wi, wj) owns rows row0 + 32 wi ..
// +31 of W and columns 32 wj .. +31 (BN = 32 WN = kpad).  Per 32-wide
// contraction chunk the block stages the A tile (BM rows) and the X^T tile
// (BN columns) of all s planes through a double-buffered LDS tile (rows padded
// by 16 bytes, which keeps the 16-byte fragment reads of 16 lanes on distinct
// banks), and each wavefront issues the s(s+1)/2 products of its 32 x 32 tile.
template <int S, int WM, int WN, bool DMA>
__global__ __launch_bounds__(WM* WN * 64) void gemm_split_kernel(const Prob* __restrict__ probs,
                                                                 const GemmItem* __restrict__ items,
                                                                 int nitems) {
  constexpr int NW = WM * WN, NT = NW * 64;
  constexpr int BM = 32 * WM, BN = 32 * WN;
  constexpr int UB = 32 * S;  // bytes of one row (or column) of a chunk
  constexpr int LS = UB + 16;
  constexpr int TILE = (BM + BN) * LS;
  constexpr int UA = BM * 2 * S, UX = BN * 2 * S;  // 16-byte units per chunk
  constexpr int UPT = DMA ? 1 : (UA + UX + NT - 1) / NT;
  // direct-to-LDS form: 16-byte slots of the tile (one padding slot per row),
  // 64 consecutive slots per wavefront instruction
  constexpr int SROW = 2 * S + 1;
  constexpr int TSLOTS = (BM + BN) * SROW;
  constexpr int NINS = (TSLOTS + 63) / 64;
  constexpr int IPW = (NINS + NW - 1) / NW;
  constexpr int TT = 32 * 33;                      // epilogue transpose tile (doubles)
  constexpr int EPI = (NW * 2 * TT + 2 * WM * BN) * 8;
  constexpr int SMEM = 2 * TILE > EPI ? 2 * TILE : EPI;
  __shared__ __attribute__((aligned(16))) uint8_t smem[SMEM];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave / WN, wj = wave % WN;
  const int l32 = lane & 31, hh = lane >> 5;

  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const GemmItem item = items[it];
    const Prob& P = probs[item.prob];
    // the column maxima of this step have been consumed by the slicing pass
    if (item.row0 == 0 && item.split == 0 && tid < P.kpad)
      reinterpret_cast<unsigned long long*>(P.xmaxp)[tid] = 0ull;
    if (P.ctrl->stopped) continue;
    const int n = P.n, k = P.k;
    const int row0 = item.row0;
    const int c0 = item.k0 >> 5, c1 = item.k1 >> 5;
    const int64_t rs = P.asl_rs;
    const uint8_t* __restrict__ Ab = P.asl + (int64_t)row0 * rs;
    const uint8_t* __restrict__ Xb = P.xsl;

    v16i acc[S];
#pragma unroll
    for (int t = 0; t < S; ++t) acc[t] = v16i{};

    u4v stg[UPT];
    auto gload = [&](int c) {
#pragma unroll
      for (int u = 0; u < UPT; ++u) {
        const int e = tid + u * NT;
        if (e < UA) {
          const int row = e / (2 * S), part = e - row * (2 * S);
          stg[u] = __builtin_nontemporal_load(
              gld(reinterpret_cast<const u4v*>(Ab + ((int64_t)c * BM + row) * UB + part * 16)));
        } else if (e < UA + UX) {
          stg[u] = *gld(reinterpret_cast<const u4v*>(Xb + (int64_t)c * BN * UB + (e - UA) * 16));
        }
      }
    };
    auto lstore = [&](uint8_t* buf) {
#pragma unroll
      for (int u = 0; u < UPT; ++u) {
        const int e = tid + u * NT;
        if (e < UA) {
          const int row = e / (2 * S), part = e - row * (2 * S);
          *reinterpret_cast<u4v*>(buf + row * LS + part * 16) = stg[u];
        } else if (e < UA + UX) {
          const int e2 = e - UA;
          const int j = e2 / (2 * S), part = e2 - j * (2 * S);
          *reinterpret_cast<u4v*>(buf + (BM + j) * LS + part * 16) = stg[u];
        }
      }
    };

    // DMA: each lane copies one 16-byte slot from global memory straight into
    // the LDS tile (lane l of a wavefront instruction writes slot 64 ii + l);
    // completion is awaited (vmcnt) before the barrier that publishes it.
    auto dma = [&](uint8_t* buf, int c) {
#pragma unroll
      for (int i = 0; i < IPW; ++i) {
        const int ii = wave + i * NW;
        if (ii < NINS) {
          const int f = ii * 64 + lane;
          const int row = f / SROW, part = f - row * SROW;
          if (f < TSLOTS && part < 2 * S) {
            const uint8_t* src = row < BM ? Ab + ((int64_t)c * BM + row) * UB + part * 16
                                          : Xb + ((int64_t)c * BN + (row - BM)) * UB + part * 16;
            __builtin_amdgcn_global_load_lds(
                (const RFK_GLOBAL void*)src,
                (__attribute__((address_space(3))) void*)(buf + ii * 1024), 16, 0, 0);
          }
        }
      }
    };
    uint8_t* buf0 = smem;
    uint8_t* buf1 = smem + TILE;
    const int xoff = (BM + wj * 32 + l32) * LS + hh * 16 * S;
    const int aoff = (wi * 32 + l32) * LS + hh * 16 * S;
    if (DMA) {
      dma(buf0, c0);
      __builtin_amdgcn_s_waitcnt(0);
    } else {
      gload(c0);
      lstore(buf0);
    }
    __syncthreads();
    for (int c = c0; c < c1; ++c) {
      const bool more = c + 1 < c1;
      const uint8_t* cur = ((c - c0) & 1) ? buf1 : buf0;
      if (more) {
        if (DMA)
          dma(((c - c0) & 1) ? buf0 : buf1, c + 1);
        else
          gload(c + 1);
      }
      v4i xf[S];
#pragma unroll
      for (int q = 0; q < S; ++q) xf[q] = *reinterpret_cast<const v4i*>(cur + xoff + q * 16);
#pragma unroll
      for (int p = 0; p < S; ++p) {
        const v4i af = *reinterpret_cast<const v4i*>(cur + aoff + p * 16);
#pragma unroll
        for (int q = 0; q < S - p; ++q) acc[p + q] = mfma_i8(xf[q], af, acc[p + q]);
      }
      if (DMA)
        __builtin_amdgcn_s_waitcnt(0);
      else if (more)
        lstore(((c - c0) & 1) ? buf0 : buf1);
      __syncthreads();
    }

    split_epilogue<S, WM, WN>(P, item, acc, smem);
    __syncthreads();
  }
}

// Word 3 of a raw buffer resource on gfx9 (32-bit data format, no swizzle).
#define RFK_BUFFER_FLAGS 0x00020000

// One 16-byte-per-lane buffer load straight into LDS: lane l's bytes at
// rsrc base + voff + soff land at lds + 16 l.
__device__ __forceinline__ void buffer_load_lds16(__amdgpu_buffer_rsrc_t r, uint8_t* lds,
                                                  uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds, 16,
                                           voff, soff, 0, 0);
}

// s_waitcnt on the vector-memory counter alone: wait until at most n of this
// wavefront's vector memory operations are outstanding (n wave-uniform).
__device__ __forceinline__ void wait_vmcnt(int n) {
  // gfx9 encoding: vmcnt[3:0] in bits 3:0, expcnt 7 and lgkmcnt 15 (no wait)
  switch (n) {
    case 0: __builtin_amdgcn_s_waitcnt(0xF70); break;
    case 1: __builtin_amdgcn_s_waitcnt(0xF71); break;
    case 2: __builtin_amdgcn_s_waitcnt(0xF72); break;
    case 3: __builtin_amdgcn_s_waitcnt(0xF73); break;
    case 4: __builtin_amdgcn_s_waitcnt(0xF74); break;
    case 5: __builtin_amdgcn_s_waitcnt(0xF75); break;
    case 6: __builtin_amdgcn_s_waitcnt(0xF76); break;
    case 7: __builtin_amdgcn_s_waitcnt(0xF77); break;
    case 8: __builtin_amdgcn_s_waitcnt(0xF78); break;
    case 9: __builtin_amdgcn_s_waitcnt(0xF79); break;
    case 10: __builtin_amdgcn_s_waitcnt(0xF7A); break;
    case 11: __builtin_amdgcn_s_waitcnt(0xF7B); break;
    case 12: __builtin_amdgcn_s_waitcnt(0xF7C); break;
    case 13: __builtin_amdgcn_s_waitcnt(0xF7D); break;
    case 14: __builtin_amdgcn_s_waitcnt(0xF7E); break;
    case 15: __builtin_amdgcn_s_waitcnt(0xF7F); break;
    default: __builtin_amdgcn_s_waitcnt(0xF70); break;
  }
}

// Ring-pipelined form of the product.  The tiles of one 32-wide contraction
// chunk are split in two rings of direct-to-LDS stages: the X^T tile (read
// by every block, so served from L2) one chunk ahead in two stages, and the A
// tile (streamed once from HBM) DA - 1 chunks ahead in DA stages, as many
// as fit in LDS beside the X stages.  Per chunk c a wavefront issues its share
// of X(c + 1), then of A(c + DA - 1); loads complete in issue order, so
// waiting until only the A(c + DA - 1) share is outstanding leaves X(c + 1)
// and A(c + 1) (issued a chunk earlier) in LDS before the barrier that
// publishes them.
template <int S, int WM, int WN>
struct SplitRing {
  static constexpr int NW = WM * WN, BM = 32 * WM, BN = 32 * WN;
  static constexpr int SROW = 2 * S + 1;  // 16-byte slots per tile row (one padding slot)
  static constexpr int LS = 16 * SROW;     // bytes per tile row
  // direct-to-LDS instructions per stage (64 slots each) and stage strides:
  // a stage spans whole instructions, so the lanes of the last one that fall
  // past the tile write into the stage's own tail
  static constexpr int NIX = (BN * SROW + 63) / 64, NIA = (BM * SROW + 63) / 64;
  static constexpr int XSTR = NIX * 1024, ASTR = NIA * 1024;
  static constexpr int IPX = (NIX + NW - 1) / NW, IPA = (NIA + NW - 1) / NW;
  static constexpr int LDS_BYTES = 160 * 1024;
  static constexpr int DA0 = (LDS_BYTES - 2 * XSTR) / ASTR;
  static constexpr int DA = DA0 > 4 ? 4 : DA0;
  static constexpr int TT = 32 * 33;
  static constexpr int EPI = (NW * 2 * TT + 2 * WM * BN) * 8;
  static constexpr int RING = 2 * XSTR + DA * ASTR;
  static constexpr int SMEM = RING > EPI ? RING : EPI;
  static_assert(DA >= 2, "two A stages must fit");
  static_assert(NIA >= NW, "every wavefront issues part of each A stage");
  static_assert(IPA <= 15, "wait_vmcnt covers at most 15 outstanding loads");
};

template <int S, int WM, int WN>
__global__ __launch_bounds__(WM* WN * 64) void gemm_split_ring_kernel(const Prob* __restrict__ probs,
                                                                      const GemmItem* __restrict__ items,
                                                                      int nitems) {
  using R = SplitRing<S, WM, WN>;
  constexpr int NW = R::NW, BN = R::BN, BM = R::BM, LS = R::LS, SROW = R::SROW, DA = R::DA;
  constexpr int UB = 32 * S;  // bytes of one row (or column) of a chunk
  __shared__ __attribute__((aligned(16))) uint8_t smem[R::SMEM];
  uint8_t* ringX = smem;
  uint8_t* ringA = smem + 2 * R::XSTR;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave / WN, wj = wave % WN;
  const int l32 = lane & 31, hh = lane >> 5;
  // this wavefront's A instructions per stage (all waves issue at least one)
  const int wv = __builtin_amdgcn_readfirstlane(wave);  // wave index as a scalar
  const int na_w = (R::NIA - wv + NW - 1) / NW;

  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const GemmItem item = items[it];
    const Prob& P = probs[item.prob];
    // the column maxima of this step have been consumed by the slicing pass
    if (item.row0 == 0 && item.split == 0 && tid < P.kpad)
      reinterpret_cast<unsigned long long*>(P.xmaxp)[tid] = 0ull;
    if (P.ctrl->stopped) continue;
    const int row0 = item.row0;
    const int c0 = item.k0 >> 5, c1 = item.k1 >> 5;
    const int64_t rs = P.asl_rs;
    const uint8_t* __restrict__ Ab = P.asl + (int64_t)row0 * rs;
    const uint8_t* __restrict__ Xb = P.xsl;

    // Per-lane source offsets within a chunk.  Every lane of an instruction
    // loads: a padding slot takes a copy of its row's first unit and a slot
    // past the tile the tile's first unit (both land where nothing reads),
    // so the loads need no per-lane branches.
    uint32_t offX[R::IPX], offA[R::IPA];
#pragma unroll
    for (int i = 0; i < R::IPX; ++i) {
      const int f = (wv + i * NW) * 64 + lane, row = f / SROW, part = f - row * SROW;
      offX[i] = f < BN * SROW ? (uint32_t)(row * UB + (part < 2 * S ? part : 0) * 16) : 0u;
    }
#pragma unroll
    for (int i = 0; i < R::IPA; ++i) {
      const int f = (wv + i * NW) * 64 + lane, row = f / SROW, part = f - row * SROW;
      offA[i] = f < BM * SROW ? (uint32_t)(row * UB + (part < 2 * S ? part : 0) * 16) : 0u;
    }
    // Buffer resources over this item's X slices and A row block: the loads
    // take a fixed per-lane offset and a per-chunk scalar offset, so no
    // per-lane 64-bit address lives across the loop.  Offsets past the
    // resource's size read zeros instead of faulting.
    const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
        (void*)Xb, (short)0, (int)((int64_t)P.nch * BN * UB), RFK_BUFFER_FLAGS);
    const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
        (void*)Ab, (short)0, (int)((int64_t)P.nch * BM * UB), RFK_BUFFER_FLAGS);
    auto dma_x = [&](int stage, int c) {
      const uint32_t soff = (uint32_t)c * (BN * UB);
      uint8_t* dst = ringX + stage * R::XSTR;
#pragma unroll
      for (int i = 0; i < R::IPX; ++i) {
        const int ii = wv + i * NW;
        if (ii < R::NIX)
          buffer_load_lds16(rx, dst + ii * 1024, offX[i], soff);
      }
    };
    auto dma_a = [&](int stage, int c) {
      const uint32_t soff = (uint32_t)c * (BM * UB);
      uint8_t* dst = ringA + stage * R::ASTR;
#pragma unroll
      for (int i = 0; i < R::IPA; ++i) {
        const int ii = wv + i * NW;
        if (ii < R::NIA)
          buffer_load_lds16(ra, dst + ii * 1024, offA[i], soff);
      }
    };

    v16i acc[S];
#pragma unroll
    for (int t = 0; t < S; ++t) acc[t] = v16i{};

    dma_x(0, c0);
#pragma unroll
    for (int d = 0; d < DA - 1; ++d)
      if (c0 + d < c1) dma_a(d, c0 + d);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    const int xoff = (wj * 32 + l32) * LS + hh * 16 * S;
    const int aoff = (wi * 32 + l32) * LS + hh * 16 * S;
    int sx = 0, sa = 0;  // ring stages of chunk c
    for (int c = c0; c < c1; ++c) {
      const bool more_x = c + 1 < c1, more_a = c + DA - 1 < c1;
      if (more_x) dma_x(sx ^ 1, c + 1);
      if (more_a) dma_a(sa == 0 ? DA - 1 : sa - 1, c + DA - 1);
      const uint8_t* xc = ringX + sx * R::XSTR;
      const uint8_t* ac = ringA + sa * R::ASTR;
      v4i xf[S];
#pragma unroll
      for (int q = 0; q < S; ++q) xf[q] = *reinterpret_cast<const v4i*>(xc + xoff + q * 16);
#pragma unroll
      for (int p = 0; p < S; ++p) {
        const v4i af = *reinterpret_cast<const v4i*>(ac + aoff + p * 16);
#pragma unroll
        for (int q = 0; q < S - p; ++q) acc[p + q] = mfma_i8(xf[q], af, acc[p + q]);
      }
      if (DA > 2 && more_x && more_a)
        wait_vmcnt(na_w);
      else
        __builtin_amdgcn_s_waitcnt(0);
      // A bare barrier: the workgroup fence of __syncthreads would wait for
      // every direct-to-LDS load in flight, the A stages ahead included.  The
      // empty asm statements keep the compiler from moving LDS accesses
      // across it; each wavefront's own wait above covers its loads.
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
      sx ^= 1;
      sa = sa + 1 == DA ? 0 : sa + 1;
    }

    split_epilogue<S, WM, WN>(P, item, acc, smem);
    __syncthreads();
  }
}

// K-split sum of the (hi, lo) partials in split order, in double-double.
__global__ __launch_bounds__(256) void split_wsum_kernel(const Prob* __restrict__ probs) {
  const Prob& P = probs[0];
  if (P.ctrl->stopped) return;
  const int64_t nk = (int64_t)P.n * P.k;
  const int ks = P.ksplit;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nk; e += (int64_t)gridDim.x * 256) {
    double s = P.swp[e], t = P.swp[nk + e];
    for (int sp = 1; sp < ks; ++sp) {
      const double* b = P.swp + (int64_t)sp * 2 * nk;
      double s2, e2;
      two_sum(s, b[e], s2, e2);
      s = s2;
      t += e2 + b[nk + e];
    }
    double h, l;
    two_sum(s, t, h, l);
    P.w[e] = h;
    P.wlo[e] = l;
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

namespace {

struct Layout {
  int wm, wn;
};
Layout layout_for(int k) {
  const int wn = (k + 31) / 32;
  return Layout{wn <= 2 ? 4 : 2, wn};
}

template <int S>
hipError_t launch_product_s(const Layout& L, int variant, const Prob* probs, const GemmItem* items,
                            int nitems, hipStream_t st) {
#define RFK_SPLIT(WM, WN)                                                                      \
  if (L.wm == WM && L.wn == WN) {                                                              \
    if (variant == 2)                                                                          \
      hipLaunchKernelGGL((gemm_split_ring_kernel<S, WM, WN>), dim3(nitems), dim3(WM * WN * 64),  \
                         0, st, probs, items, nitems);                                         \
    else if (variant == 1)                                                                     \
      hipLaunchKernelGGL((gemm_split_kernel<S, WM, WN, true>), dim3(nitems), dim3(WM * WN * 64), \
                         0, st, probs, items, nitems);                                         \
    else                                                                                       \
      hipLaunchKernelGGL((gemm_split_kernel<S, WM, WN, false>), dim3(nitems),                  \
                         dim3(WM * WN * 64), 0, st, probs, items, nitems);                     \
    return hipGetLastError();                                                                  \
  }
  RFK_SPLIT(4, 1)
  RFK_SPLIT(4, 2)
  RFK_SPLIT(2, 3)
  RFK_SPLIT(2, 4)
#undef RFK_SPLIT
  return hipErrorInvalidValue;
}

hipError_t launch_product(int s, const Layout& L, int variant, const Prob* probs,
                          const GemmItem* items, int nitems, hipStream_t st) {
  switch (s) {
    case 7: return launch_product_s<7>(L, variant, probs, items, nitems, st);
    case 8: return launch_product_s<8>(L, variant, probs, items, nitems, st);
    case 9: return launch_product_s<9>(L, variant, probs, items, nitems, st);
    case 10: return launch_product_s<10>(L, variant, probs, items, nitems, st);
    default: return hipErrorInvalidValue;
  }
}

template <int S>
hipError_t launch_aslice_s(const double* a, int64_t lda, int n, int nch, int rows_pad, int bm,
                           const int32_t* aexp, uint8_t* asl, hipStream_t st) {
  const int64_t units = (int64_t)rows_pad * nch * 2;
  const int grid = (int)std::min<int64_t>((units + 255) / 256, 16384);
  hipLaunchKernelGGL((split_aslice_kernel<S>), dim3(grid), dim3(256), 0, st, a, lda, n, nch,
                     rows_pad, bm, aexp, asl);
  return hipGetLastError();
}

hipError_t launch_aslice(int s, const double* a, int64_t lda, int n, int nch, int rows_pad, int bm,
                         const int32_t* aexp, uint8_t* asl, hipStream_t st) {
  switch (s) {
    case 7: return launch_aslice_s<7>(a, lda, n, nch, rows_pad, bm, aexp, asl, st);
    case 8: return launch_aslice_s<8>(a, lda, n, nch, rows_pad, bm, aexp, asl, st);
    case 9: return launch_aslice_s<9>(a, lda, n, nch, rows_pad, bm, aexp, asl, st);
    case 10: return launch_aslice_s<10>(a, lda, n, nch, rows_pad, bm, aexp, asl, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_xslice(int s, const Prob* probs, const RowItem* items, int nitems,
                         hipStream_t st) {
  const dim3 grid(std::min(nitems, 16384)), block(256);
  switch (s) {
    case 7: hipLaunchKernelGGL(split_xslice_kernel<7>, grid, block, 0, st, probs, items, nitems); break;
    case 8: hipLaunchKernelGGL(split_xslice_kernel<8>, grid, block, 0, st, probs, items, nitems); break;
    case 9: hipLaunchKernelGGL(split_xslice_kernel<9>, grid, block, 0, st, probs, items, nitems); break;
    case 10: hipLaunchKernelGGL(split_xslice_kernel<10>, grid, block, 0, st, probs, items, nitems); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Longest contraction one K range may have: a bin sums at most s digit
// products of magnitude <= 2^12 per contraction index.
int64_t max_k_range(int s) { return ((((int64_t)1 << 31) - 1) / ((int64_t)s << 12)) / 32 * 32; }

// Product work items: row blocks of every problem (larger problems first)
// times the K ranges of a K split (one problem only).
std::vector<GemmItem> split_items(const std::vector<Prob>& hp, int bm, int ks, int* nks_out) {
  std::vector<GemmItem> gi;
  int nks = 1;
  for (size_t p = 0; p < hp.size(); ++p) {
    const int nch = hp[p].nch;
    const int64_t kc = ((int64_t)nch + ks - 1) / ks * 32;
    nks = (int)(((int64_t)nch * 32 + kc - 1) / kc);
    const int nrb = (hp[p].n + bm - 1) / bm;
    for (int rb = 0; rb < nrb; ++rb)
      for (int sp = 0; sp < nks; ++sp) {
        GemmItem g{};
        g.prob = (int)p;
        g.row0 = rb * bm;
        g.k0 = (int)(sp * kc);
        g.k1 = (int)std::min<int64_t>((int64_t)nch * 32, (sp + 1) * kc);
        g.split = sp;
        gi.push_back(g);
      }
  }
  if (hp.size() > 1)
    std::stable_sort(gi.begin(), gi.end(), [&](const GemmItem& x, const GemmItem& y) {
      return hp[x.prob].n > hp[y.prob].n;
    });
  *nks_out = nks;
  return gi;
}


template <class T>
hipError_t upload_vec(T** dst, const std::vector<T>& v) {
  (void)hipFree(*dst);
  *dst = nullptr;
  if (v.empty()) return hipSuccess;
  hipError_t e = hipMalloc((void**)dst, sizeof(T) * v.size());
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
}

int install_items(SplitPlan& sp, int ks, std::vector<Prob>& hp, Prob* dprob) {
  int nks = 1;
  std::vector<GemmItem> gi = split_items(hp, sp.bm, ks, &nks);
  if (upload_vec(&sp.items, gi) != hipSuccess) return REFINE_ENOMEM;
  sp.nitems = (int)gi.size();
  sp.ks = nks;
  for (Prob& P : hp) {
    P.ksplit = nks;
    P.ndp = (P.n + sp.bm - 1) / sp.bm * nks;
  }
  if (hipMemcpy(dprob, hp.data(), sizeof(Prob) * hp.size(), hipMemcpyHostToDevice) != hipSuccess)
    return REFINE_EHIP;
  return REFINE_OK;
}

}  // namespace

int split_rows_per_block(int k) { return 32 * layout_for(k).wm; }

hipError_t split_xmax(const SplitPlan& sp, const Prob* dprob, hipStream_t st) {
  hipLaunchKernelGGL(split_xmax_kernel, dim3(std::min(sp.n_xmax, 8192)), dim3(256), 0, st, dprob,
                     sp.xmax_items, sp.n_xmax);
  product_mark(st);
  return hipGetLastError();
}

hipError_t split_aexp(const refine_matrix& A, int rows_pad, int32_t* aexp, hipStream_t st) {
  hipLaunchKernelGGL(split_aexp_kernel, dim3((unsigned)((rows_pad + 3) / 4)), dim3(256), 0, st,
                     A.a, A.lda, (int)A.n, rows_pad, aexp);
  return hipGetLastError();
}

hipError_t split_product(const SplitPlan& sp, const Prob* dprob, hipStream_t st) {
  if (sp.crt) return crt_product(sp, dprob, st);
  hipError_t e;
  if ((e = split_xmax(sp, dprob, st)) != hipSuccess) return e;
  if ((e = launch_xslice(sp.s, dprob, sp.xsl_items, sp.n_xsl, st)) != hipSuccess) return e;
  product_mark(st);
  if ((e = launch_product(sp.s, layout_for(sp.kmax), sp.variant, dprob, sp.items, sp.nitems, st)) !=
      hipSuccess)
    return e;
  product_mark(st);
  if (sp.ks > 1) {
    const int64_t nk = sp.nk0;
    const int grid = (int)std::min<int64_t>((nk + 255) / 256, 4096);
    hipLaunchKernelGGL(split_wsum_kernel, dim3(grid), dim3(256), 0, st, dprob);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    product_mark(st);
  }
  return hipSuccess;
}

int split_init(SplitPlan& sp, const std::vector<refine_matrix>& As, const std::vector<int>& ks,
               int slices, int crt, std::vector<Prob>& hp, Prob* dprob, hipStream_t st) {
  sp = SplitPlan();
  const int np = (int)As.size();
  if (crt) {
    // modular form: one problem; the column-maximum pass is shared
    if (np != 1 || ks[0] < 1 || ks[0] > KMAX) return REFINE_EINVAL;
    const Layout L = layout_for(ks[0]);
    sp.kmax = ks[0];
    sp.kpad = 32 * L.wn;
    sp.np = 1;
    sp.nk0 = As[0].n * ks[0];
    constexpr int XROWS = 64;
    std::vector<RowItem> xm;
    Prob& P = hp[0];
    P.xrows = XROWS;
    P.nbx = (int)((As[0].n + XROWS - 1) / XROWS);
    for (int b = 0; b < P.nbx; ++b) xm.push_back(RowItem{0, b});
    if (hipMalloc((void**)&sp.xexp, sizeof(int32_t) * sp.kpad) != hipSuccess ||
        hipMalloc((void**)&sp.xmaxp, sizeof(double) * sp.kpad) != hipSuccess ||
        upload_vec(&sp.xmax_items, xm) != hipSuccess) {
      split_free(sp);
      return REFINE_ENOMEM;
    }
    sp.n_xmax = (int)xm.size();
    P.xexp = sp.xexp;
    P.xmaxp = sp.xmaxp;
    if (hipMemsetAsync(sp.xmaxp, 0, sizeof(double) * sp.kpad, st) != hipSuccess ||
        hipMemsetAsync(sp.xexp, 0, sizeof(int32_t) * sp.kpad, st) != hipSuccess) {
      split_free(sp);
      return REFINE_EHIP;
    }
    const int rc = crt_init(sp, As[0], ks[0], crt, hp, dprob, st);
    if (rc != REFINE_OK) split_free(sp);
    return rc;
  }
  if (np < 1 || slices < SPLIT_S_MIN || slices > SPLIT_S_MAX) return REFINE_EINVAL;
  int kmax = 0;
  for (int p = 0; p < np; ++p) {
    if (As[p].kind != REFINE_DENSE || ks[p] < 1 || ks[p] > KMAX || As[p].n > SPLIT_NMAX)
      return REFINE_EINVAL;
    kmax = std::max(kmax, ks[p]);
  }
  const int s = slices;
  const Layout L = layout_for(kmax);
  sp.s = s;
  sp.kmax = kmax;
  sp.kpad = 32 * L.wn;
  sp.bm = 32 * L.wm;
  sp.np = np;
  sp.nk0 = As[0].n * ks[0];
  // rows per column-maximum item: 64 gives a few hundred items at n = 8k-16k
  // (256-row items left most CUs idle and each thread a long chain of loads)
  // at a few hundred atomic merges per column
  constexpr int XROWS = 64;
  // one allocation per array for all problems
  std::vector<size_t> o_asl(np), o_aexp(np), o_xsl(np);
  size_t t_asl = 0, t_aexp = 0, t_xsl = 0;
  for (int p = 0; p < np; ++p) {
    const int64_t n = As[p].n, nch = (n + 31) / 32;
    const int64_t rows_pad = (n + SPLIT_ROW_PAD - 1) / SPLIT_ROW_PAD * SPLIT_ROW_PAD;
    o_asl[p] = t_asl;
    t_asl += ((size_t)rows_pad * nch * 32 * s + 255) / 256 * 256;
    o_aexp[p] = t_aexp;
    t_aexp += (size_t)rows_pad;
    o_xsl[p] = t_xsl;
    t_xsl += ((size_t)nch * sp.kpad * 32 * s + 255) / 256 * 256;
  }
  if (hipMalloc((void**)&sp.asl, t_asl) != hipSuccess ||
      hipMalloc((void**)&sp.aexp, sizeof(int32_t) * t_aexp) != hipSuccess ||
      hipMalloc((void**)&sp.xsl, t_xsl) != hipSuccess ||
      hipMalloc((void**)&sp.xexp, sizeof(int32_t) * sp.kpad * np) != hipSuccess ||
      hipMalloc((void**)&sp.xmaxp, sizeof(double) * sp.kpad * np) != hipSuccess ||
      (np == 1 &&
       hipMalloc((void**)&sp.swp, sizeof(double) * 2 * SPLIT_KS_MAX * As[0].n * ks[0]) != hipSuccess)) {
    split_free(sp);
    return REFINE_ENOMEM;
  }
  hipError_t e = hipMemsetAsync(sp.xmaxp, 0, sizeof(double) * sp.kpad * np, st);
  if (e == hipSuccess) e = hipMemsetAsync(sp.xexp, 0, sizeof(int32_t) * sp.kpad * np, st);
  std::vector<RowItem> xm, xs;
  for (int p = 0; p < np && e == hipSuccess; ++p) {
    const refine_matrix& A = As[p];
    const int64_t n = A.n;
    const int nch = (int)((n + 31) / 32);
    const int64_t rows_pad = (n + SPLIT_ROW_PAD - 1) / SPLIT_ROW_PAD * SPLIT_ROW_PAD;
    hipLaunchKernelGGL(split_aexp_kernel, dim3((unsigned)((rows_pad + 3) / 4)), dim3(256), 0, st,
                       A.a, A.lda, (int)n, (int)rows_pad, sp.aexp + o_aexp[p]);
    e = hipGetLastError();
    if (e == hipSuccess)
      e = launch_aslice(s, A.a, A.lda, (int)n, nch, (int)rows_pad, sp.bm, sp.aexp + o_aexp[p],
                        sp.asl + o_asl[p], st);
    Prob& P = hp[p];
    P.asl = sp.asl + o_asl[p];
    P.asl_rs = (int64_t)nch * 32 * s;
    P.aexp = sp.aexp + o_aexp[p];
    P.xsl = sp.xsl + o_xsl[p];
    P.xexp = sp.xexp + (size_t)sp.kpad * p;
    P.xmaxp = sp.xmaxp + (size_t)sp.kpad * p;
    P.swp = np == 1 ? sp.swp : nullptr;
    P.nch = nch;
    P.kpad = sp.kpad;
    P.xrows = XROWS;
    P.nbx = (int)((n + XROWS - 1) / XROWS);
    for (int b = 0; b < P.nbx; ++b) xm.push_back(RowItem{p, b});
    const int64_t units = (int64_t)nch * sp.kpad * 2;
    for (int64_t b = 0; b < (units + 255) / 256; ++b) xs.push_back(RowItem{p, (int)b});
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = upload_vec(&sp.xmax_items, xm);
  if (e == hipSuccess) e = upload_vec(&sp.xsl_items, xs);
  if (e != hipSuccess) {
    split_free(sp);
    return REFINE_EHIP;
  }
  sp.n_xmax = (int)xm.size();
  sp.n_xsl = (int)xs.size();

  // K split (one problem only) and tile-loading variant: REFINE_SPLIT_KS=
  // "ks[,variant]" forces them; otherwise the candidates (K splits 1, 2, 4, 8
  // whose K range fits the exact INT32 bins; the three variants) are timed
  // once per shape and process.
  const int64_t kmax_range = max_k_range(s);
  int64_t nch_max = 0, nsum = 0;
  for (const Prob& P : hp) {
    nch_max = std::max<int64_t>(nch_max, P.nch);
    nsum += P.n;
  }
  auto fits = [&](int ksp) { return (nch_max + ksp - 1) / ksp * 32 <= kmax_range; };
  const int ks_cap = np == 1 ? SPLIT_KS_MAX : 1;
  int best_ks = 0, best_var = 0;
  if (const char* env = getenv("REFINE_SPLIT_KS")) {
    int ksp = 0, var = 0;
    const int got = sscanf(env, "%d,%d", &ksp, &var);
    if (got >= 1 && ksp >= 1 && ksp <= ks_cap && fits(ksp) && var >= 0 && var <= 2) {
      best_ks = ksp;
      best_var = got == 2 ? var : 0;
    }
  }
  const std::vector<int64_t> key{np == 1 ? As[0].n : nsum, kmax, s, np};
  if (!best_ks) {
    std::vector<int> hit;
    if (tune_cache_get("split", key, &hit) && hit.size() == 2 && hit[0] >= 1 &&
        hit[0] <= ks_cap && fits(hit[0]) && hit[1] >= 0 && hit[1] <= 2) {
      best_ks = hit[0];
      best_var = hit[1];
    }
  }
  if (!best_ks) {
    // time on a zero X (the workspace copy of the update)
    std::vector<std::pair<double*, int64_t>> saved;
    for (Prob& P : hp) {
      saved.push_back({P.x, P.ldx});
      P.x = P.xn;
      P.ldx = P.k;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      split_free(sp);
      return REFINE_EHIP;
    }
    float best = 1e30f;
    for (int var = 0; var <= 2; ++var)
      for (int ksp = 1; ksp <= ks_cap; ksp *= 2) {
        if (!fits(ksp)) continue;
        sp.variant = var;
        int rc = install_items(sp, ksp, hp, dprob);
        if (rc != REFINE_OK) {
          split_free(sp);
          return rc;
        }
        float t = 0.f;
        e = split_product(sp, dprob, st);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int r = 0; r < 3 && e == hipSuccess; ++r) e = split_product(sp, dprob, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess) {
          split_free(sp);
          return REFINE_EHIP;
        }
        if (getenv("REFINE_LOG") && atoi(getenv("REFINE_LOG")) >= 2)
          fprintf(stderr, "refine: tune split np=%d n=%lld k=%d s=%d variant %d ks %d: %.1f us\n",
                  np, (long long)key[0], kmax, s, var, ksp, t * 1000.f / 3.f);
        if (t < best) {
          best = t;
          best_ks = ksp;
          best_var = var;
        }
      }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (size_t p = 0; p < hp.size(); ++p) {
      hp[p].x = saved[p].first;
      hp[p].ldx = saved[p].second;
    }
    sp.ms = best / 3.f;
    tune_cache_put("split", key, {best_ks, best_var});
    if (getenv("REFINE_LOG"))
      fprintf(stderr, "refine: split product np=%d n=%lld k=%d s=%d: variant %d, K split %d, %.1f us\n",
              np, (long long)key[0], kmax, s, best_var, best_ks, best * 1000.f / 3.f);
  }
  if (!best_ks) {
    split_free(sp);
    return REFINE_EINVAL;
  }
  sp.variant = best_var;
  return install_items(sp, best_ks, hp, dprob);
}

void split_free(SplitPlan& sp) {
  (void)hipFree(sp.asl);
  (void)hipFree(sp.aexp);
  (void)hipFree(sp.xsl);
  (void)hipFree(sp.xexp);
  (void)hipFree(sp.xmaxp);
  (void)hipFree(sp.swp);
  (void)hipFree(sp.items);
  (void)hipFree(sp.xmax_items);
  (void)hipFree(sp.xsl_items);
  (void)hipFree(sp.ares);
  (void)hipFree(sp.xres);
  (void)hipFree(sp.cres);
  (void)hipFree(sp.adiag);
  (void)hipFree(sp.rec_items);
  sp = SplitPlan();
}

}  // namespace rfk
