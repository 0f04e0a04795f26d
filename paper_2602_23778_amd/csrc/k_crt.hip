// Modular form of the product step of Algorithm 4, W = A X, for the
// accelerator direction of Sec. 3.1.3: the integer route of Ozaki scheme II
// (Ozaki, Uchino and Imamura 2025).  Where the slice form multiplies s digit
// slices pairwise (s(s+1)/2 INT8 products), this form multiplies residues:
// one INT8 product per modulus.
//
// Diagonal.  The diagonal of A stays out of the integer image; its part of
// the product, a_ii x_ij, is added exactly in the reconstruction.  The row
// scales then come from the off-diagonal entries, which keeps more of their
// bits where the diagonal dominates a row (as in A = Q diag(lambda) Q^T,
// whose diagonal is the mean eigenvalue while the rest shrinks like
// 1/sqrt(n)).
//
// Scaling.  Row i of A gets the exponent E_i (max_{l != i} |a_il| < 2^E_i)
// and column j of X the exponent F_j (max_l |x_lj| < 2^F_j), the smallest
// such integers (0 for a zero line), and
//     A'_il = rint(a_il 2^(bA - E_i)) (l != i; A'_ii = 0),
//     X'_lj = rint(x_lj 2^(bX - F_j)),
// integers with |A'| <= 2^bA, |X'| <= 2^bX.  Each is the rounding of one
// double, so it is itself a double (at most 53 significant bits).
//
// Moduli.  N pairwise coprime moduli m_0..m_{N-1} (256, 255, 253, ...: the
// largest whose balanced residues fit a signed byte), M their product, L the
// bit length of M.  The budget bA + bX = L - 3 - ceil(log2 n) (bA the larger
// half) keeps |(A'X')_ij| <= n 2^(bA+bX) <= 2^(L-3) < M/2, so A'X' is the one
// integer in [-M/2, M/2) with the residues of the N products
//     C_t = (A' mod m_t)(X' mod m_t)  (mod m_t),
// each an INT8 x INT8 product summed exactly in INT32 (|terms| <= 2^14, so
// n <= 2^17 keeps the sums exact).
//
// Reconstruction (Chinese remainder sum).  With e_t = (M/m_t)((M/m_t)^-1 mod
// m_t) < M (so e_t = 1 mod m_t and 0 modulo the other moduli), the balanced
// residues c_t of the products give S = sum_t c_t e_t = A'X' (mod M), and
// A'X' = S - q M with q the integer nearest S/M: |A'X'| <= 2^(L-3) <= M/4
// puts S/M within 1/4 of q, so an FP64 estimate of S/M rounds to q.  All of
// it is exact in FP64 pieces: e_t and M are split into four 32-bit pieces,
// S_k = sum_t c_t e_tk (|S_k| < 2^43) and D_k = S_k - q M_k (|D_k| < 2^44)
// are exact, and A'X' = sum_k D_k 2^(32k) is summed into a double-double
// from the top (relative error about 2^-105 when it needs more than 106
// bits).  The pair is scaled by 2^(E_i + F_j - bA - bX), and a_ii x_ij (an
// exact product pair) is added with both parts' errors kept:
// W = (W_hi, W_lo).  Against Garner's mixed radix (N^2/2 modular steps and
// a Horner evaluation) this is 4N fused multiply-adds per entry.
//
// Layouts (bytes).  A's residues: N planes, each tile-major like the slices
// of the slice form with one digit per value: rows in blocks of BM, per
// block the 32-wide contraction chunks one after another, per chunk the BM
// rows of 32 bytes: plane t, row i = BM b + r, chunk c at
//     ares + t ares_plane + ((b nchp + c) BM + r) 32.
// X^T's residues: N planes of nchp chunks, each chunk kpad columns of 32
// bytes: xres + t xres_plane + (c kpad + j) 32.  The residues of the
// products: N planes of rows_pad x kpad bytes, residue t of entry (i, j)
// at cres + t cres_plane + i kpad + j, so that each wavefront of the product
// writes whole lines of one plane (an entry-major layout, 16 bytes per
// entry, made the product's 16 workgroups per line each write back a
// partial line: 10x the written bytes).  Chunks are padded with zeros to a
// multiple of XG_PAD (nchp), rows to a multiple of 256.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "dev_util.h"
#include "split.h"
#include "tune_cache.h"

namespace rfk {

namespace {

typedef int v16i __attribute__((ext_vector_type(16)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

// The moduli: pairwise coprime, the largest that fit a signed byte as
// balanced residues.
constexpr int CRT_MOD[CRT_N_MAX] = {256, 255, 253, 251, 247, 241, 239, 233,
                                    229, 227, 223, 217, 211, 199, 197, 193};

// Chunk counts of the contraction are padded to a multiple of this (the
// largest chunk group of the product), and the residue planes of A are laid
// out in tiles of CRT_TILE rows.
constexpr int XG_PAD = 8;
constexpr int CRT_TILE = 128;

// Constants of the Chinese remainder sum for the first N moduli, in 32-bit
// pieces held exactly as doubles: e_t = (M/m_t) ((M/m_t)^-1 mod m_t) and M
// (M < 2^126 for N <= 16, so 128-bit integers hold every value).
constexpr unsigned __int128 cmul_mod(unsigned __int128 a, unsigned b, unsigned m) {
  return (a % m) * b % m;
}
template <int N>
struct CrtSum {
  double e[N][4];
  double mk[4];
  double m_d;     // M rounded to a double
  double minv;    // 1 / M rounded
  constexpr CrtSum() : e(), mk(), m_d(0.0), minv(0.0) {
    unsigned __int128 M = 1;
    for (int t = 0; t < N; ++t) M *= (unsigned)CRT_MOD[t];
    for (int t = 0; t < N; ++t) {
      const unsigned m = (unsigned)CRT_MOD[t];
      const unsigned __int128 Mt = M / m;
      // inverse of Mt modulo m by exponentiation-free search (m <= 256)
      unsigned r = (unsigned)(Mt % m), inv = 0;
      for (unsigned c = 1; c < m; ++c)
        if ((unsigned __int128)r * c % m == 1) {
          inv = c;
          break;
        }
      const unsigned __int128 et = Mt * inv;
      for (int k = 0; k < 4; ++k) e[t][k] = (double)(unsigned long long)((et >> (32 * k)) & 0xffffffffu);
    }
    for (int k = 0; k < 4; ++k) mk[k] = (double)(unsigned long long)((M >> (32 * k)) & 0xffffffffu);
    double md = 0.0;
    for (int k = 3; k >= 0; --k) md = md * 4294967296.0 + mk[k];
    m_d = md;
    minv = 1.0 / md;
  }
};

// Balanced residue of an integer-valued double v (|v| < 2^62) modulo m, in
// [-128, 127] for m = 256 and [-(m-1)/2, (m-1)/2] for odd m.  Both steps are
// exact: q is an integer near v/m (|v/m - q| < 6 from the rounding of v/m),
// so v - q m is a small integer and the fused multiply-add returns it
// exactly; the second step then rounds a small quotient correctly (an odd m
// leaves no halfway case, m = 256 maps the one tie, 128, to -128).
__device__ __forceinline__ int bal_res(double v, int m, double inv) {
  double r = __builtin_fma(-__builtin_rint(v * inv), (double)m, v);
  r = __builtin_fma(-__builtin_rint(r * inv), (double)m, r);
  int ri = (int)r;
  if (ri == 128) ri = -128;  // only m = 256 can produce it
  return ri;
}

// The same residue with one rounded quotient per modulus, for values split
// once as v = vh 2^28 + vl (vh = rint(v 2^-28), both parts exact):
// t = vh (2^28 mod m) + vl is congruent to v and exact (|t| < 2^43), so
// rint(t / m) is correct (its rounding error is far below 1/(2m)), and
// r = t - m rint(t / m) in [-m/2, m/2] is exact.  The byte is read from the
// binary64 of r + 1.5 2^52, whose low mantissa bits hold r in two's
// complement (a plain add instead of a conversion; the tie of m = 256, +-128,
// gives the byte 0x80 either way).  Equal to bal_res byte for byte.
__device__ __forceinline__ int bal_res_split(double vh, double vl, int m, double inv) {
  const double t = __builtin_fma(vh, (double)((1 << 28) % m), vl);
  const double r = __builtin_fma(-__builtin_rint(t * inv), (double)m, t);
  return (int)(unsigned)(unsigned long long)__double_as_longlong(r + 0x1.8p52);
}

__device__ __forceinline__ int scale_exp(double mx) {
  int e = 0;
  if (mx > 0.0) (void)frexp(mx, &e);  // mx = f 2^e, f in [1/2, 1): mx < 2^e
  return e;
}

__device__ __forceinline__ unsigned pack4(int a, int b, int c, int d) {
  return ((unsigned)a & 0xffu) | (((unsigned)b & 0xffu) << 8) | (((unsigned)c & 0xffu) << 16) |
         ((unsigned)d << 24);
}

struct CrtArgs {
  const int8_t* ares;
  int64_t ares_plane;
  int8_t* xres;
  int64_t xres_plane;
  int8_t* cres;        // residues of the products, N planes
  int64_t cres_plane;  // rows_pad * kpad
  const double* adiag; // a_ii (rows_pad entries, 0 past n)
  int nchp;            // contraction chunks, padded to a multiple of XG_PAD
  int ba, bx;
};

// ---------------------------------------------------------------------------
// Row exponents of A from the off-diagonal maxima, and the diagonal (once, at
// init): one wavefront per row (rows >= n get 0).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void crt_aexp_kernel(const double* __restrict__ a, int64_t lda,
                                                       int n, int rows_pad,
                                                       int32_t* __restrict__ aexp,
                                                       double* __restrict__ adiag) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows_pad) return;
  double m = 0.0;
  if (row < n)
    for (int c = lane; c < n; c += 64)
      if (c != row) m = fmax(m, fabs(a[(int64_t)row * lda + c]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if (lane == 0) {
    aexp[row] = scale_exp(m);
    adiag[row] = row < n ? a[(int64_t)row * lda + row] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Residues of A (once, at init): one thread per 16-column unit (row, chunk,
// half), the diagonal entry imaged as 0.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void crt_ares_kernel(const double* __restrict__ a, int64_t lda,
                                                       int n, int rows_pad, int bm, CrtArgs ca,
                                                       const int32_t* __restrict__ aexp) {
  const int nchp = ca.nchp;
  const int64_t units = (int64_t)rows_pad * nchp * 2;
  for (int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x; u < units;
       u += (int64_t)gridDim.x * 256) {
    const int row = (int)(u / (2 * nchp));
    const int cu = (int)(u - (int64_t)row * 2 * nchp);  // 2 * chunk + half
    const int col0 = cu * 16;
    const int sh = ca.ba - aexp[row];
    double v[16];
#pragma unroll
    for (int b = 0; b < 16; ++b)
      v[b] = (row < n && col0 + b < n && col0 + b != row)
                 ? __builtin_rint(ldexp(a[(int64_t)row * lda + col0 + b], sh))
                 : 0.0;
    const int rb = row / bm, c = cu >> 1;
    const int64_t off = (((int64_t)rb * nchp + c) * bm + (row - rb * bm)) * 32 + (cu & 1) * 16;
#pragma unroll
    for (int t = 0; t < N; ++t) {
      const int m = CRT_MOD[t];
      const double inv = 1.0 / CRT_MOD[t];
      int r[16];
#pragma unroll
      for (int b = 0; b < 16; ++b) r[b] = bal_res(v[b], m, inv);
      const u4v o = {pack4(r[0], r[1], r[2], r[3]), pack4(r[4], r[5], r[6], r[7]),
                     pack4(r[8], r[9], r[10], r[11]), pack4(r[12], r[13], r[14], r[15])};
      *reinterpret_cast<u4v*>(const_cast<int8_t*>(ca.ares) + t * ca.ares_plane + off) = o;
    }
  }
}

// ---------------------------------------------------------------------------
// Residues of X^T (every step): one thread per half unit, 8 rows of one
// column (a unit is a chunk, column and half: 16 rows, 16 bytes per modulus
// plane), so that the residue arithmetic spreads over twice the wavefronts
// of a thread per unit; the column exponent comes from the maxima of |X|.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void crt_xres_kernel(const Prob* __restrict__ probs, CrtArgs ca) {
  typedef unsigned u2v __attribute__((ext_vector_type(2)));
  const Prob& P = probs[0];
  if (P.ctrl->stopped) return;
  const int kpad = P.kpad, k = P.k, n = P.n;
  const int64_t halves = (int64_t)ca.nchp * kpad * 4;
  const unsigned long long* mx = reinterpret_cast<const unsigned long long*>(P.xmaxp);
  for (int64_t su = (int64_t)blockIdx.x * 256 + threadIdx.x; su < halves;
       su += (int64_t)gridDim.x * 256) {
    const int64_t u = su >> 1;
    const int q = (int)(su & 1), h = (int)(u & 1);
    const int64_t cj = u >> 1;
    const int c = (int)(cj / kpad);
    const int j = (int)(cj - (int64_t)c * kpad);
    // the column maximum and the 8 entries are requested together (indices
    // clamped into X, entries past it masked to zero afterwards)
    const bool jok = j < k;
    const int jc = jok ? j : k - 1;
    const int r0 = c * 32 + h * 16 + q * 8;
    const unsigned long long mxj = *gld(mx + jc);
    double xv[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) xv[b] = *gld(P.x + (int64_t)min(r0 + b, n - 1) * P.ldx + jc);
    const int e = jok ? scale_exp(__longlong_as_double((long long)mxj)) : 0;
    if (c == 0 && h == 0 && q == 0) P.xexp[j] = e;
    const int sh = ca.bx - e;
    double vh[8], vl[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const double v = (jok && r0 + b < n) ? __builtin_rint(ldexp(xv[b], sh)) : 0.0;
      vh[b] = __builtin_rint(v * 0x1p-28);
      vl[b] = __builtin_fma(-vh[b], 0x1p28, v);
    }
#pragma unroll
    for (int t = 0; t < N; ++t) {
      const int m = CRT_MOD[t];
      const double inv = 1.0 / CRT_MOD[t];
      int r[8];
#pragma unroll
      for (int b = 0; b < 8; ++b) r[b] = bal_res_split(vh[b], vl[b], m, inv);
      const u2v o = {pack4(r[0], r[1], r[2], r[3]), pack4(r[4], r[5], r[6], r[7])};
      *reinterpret_cast<u2v*>(ca.xres + t * ca.xres_plane + su * 8) = o;
    }
  }
}

// ---------------------------------------------------------------------------
// The residue products.  Work item (modulus t = item.split, row block
// row0 = item.row0 of BM = 32 WAVES W rows); item.k0 < 0 marks an empty slot.
// Wavefront w owns the rows row0 + 32 w .. +31 of W and all kpad columns (KT
// tiles of 32).  Per group of XG 32-wide contraction chunks a wavefront loads
// its A fragments (16 bytes per lane per chunk) straight from the residue
// plane into registers, and the block its share of the group's X^T residues,
// both PF groups ahead through PF + 1 register stages (the group loop is
// unrolled by PF + 1 so that every stage keeps its registers); the X^T group
// one ahead, requested a group earlier, goes to the LDS stage the next group
// reads (double buffered, rows padded to 48 bytes so that the 16-byte
// fragment reads of 16 lanes fall on distinct banks), so the wait before
// that store is for loads a whole group old.  Loads past the last group are
// clamped to it (valid memory, never used), which keeps the compiler's wait
// counts exact across the loop.  A variant that staged X^T only one group
// ahead spent about 20 % more time (it waited each group for the X^T
// requests just issued); one that read the X^T fragments straight from
// memory per wavefront, without LDS, took twice as long (eight wavefronts
// re-reading each fragment through the vector L1).
//
// v_mfma_i32_32x32x32_i8 (gfx950): lane l supplies a[m = l%32][kk = 16(l/32)
// + b] and b[kk = 16(l/32) + b][n = l%32] for the bytes b of its 16-byte
// operand; register r of the result holds c[m = 8(r/4) + 4(l/32) + r%4][n =
// l%32].  The X^T fragment is the a operand (m = column j of W), the A
// fragment the b operand (n = row i of W).
// ---------------------------------------------------------------------------
template <int KT, int WAVES, int XG, int PF>
__global__ __launch_bounds__(WAVES * 64) void crt_gemm_kernel(const Prob* __restrict__ probs,
                                                              const GemmItem* __restrict__ items,
                                                              CrtArgs ca) {
  constexpr int NT = WAVES * 64, KP = 32 * KT;
  constexpr int XROW = 48;                    // padded LDS row (bytes)
  constexpr int XSTAGE = XG * KP * XROW;      // bytes per stage
  constexpr int XUNITS = XG * KP * 2;         // 16-byte units per stage
  constexpr int XPT = (XUNITS + NT - 1) / NT; // units per thread
  constexpr int S = PF + 1;                   // register stages
  __shared__ __attribute__((aligned(16))) int8_t xs[2 * XSTAGE];

  const GemmItem item = items[blockIdx.x];
  const Prob& P = probs[0];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // the column maxima of this step have been consumed by the residue pass
  if (item.k0 == 0 && item.row0 == 0 && item.split == 0 && tid < KP)
    reinterpret_cast<unsigned long long*>(P.xmaxp)[tid] = 0ull;
  if (item.k0 < 0 || P.ctrl->stopped) return;
  const int t = item.split;
  const int nchp = ca.nchp, ngroups = nchp / XG;
  // this wavefront's 32 rows sit in the plane's tile of CRT_TILE rows that
  // holds them
  const int wrow = item.row0 + 32 * wave;
  const int8_t* __restrict__ Ab = ca.ares + t * ca.ares_plane +
                                  (int64_t)(wrow / CRT_TILE) * nchp * CRT_TILE * 32 +
                                  ((wrow % CRT_TILE) + (lane & 31)) * 32 + (lane >> 5) * 16;
  const int8_t* __restrict__ Xp = ca.xres + t * ca.xres_plane;

  v16i acc[KT];
#pragma unroll
  for (int q = 0; q < KT; ++q) acc[q] = v16i{};

  v4i a[S][XG];
  u4v x[S][XPT];
  auto load_a = [&](v4i(&dst)[XG], int g) {
    g = min(g, ngroups - 1);
#pragma unroll
    for (int cc = 0; cc < XG; ++cc)
      dst[cc] = __builtin_nontemporal_load(
          gld(reinterpret_cast<const v4i*>(Ab + (int64_t)(g * XG + cc) * CRT_TILE * 32)));
  };
  auto load_x = [&](u4v(&dst)[XPT], int g) {
    g = min(g, ngroups - 1);
#pragma unroll
    for (int u = 0; u < XPT; ++u) {
      const int e = min(tid + u * NT, XUNITS - 1);
      dst[u] = *gld(reinterpret_cast<const u4v*>(Xp + (int64_t)g * XG * KP * 32 + e * 16));
    }
  };
  auto store_x = [&](const u4v(&src)[XPT], int8_t* dst) {
#pragma unroll
    for (int u = 0; u < XPT; ++u) {
      const int e = tid + u * NT;
      if (e < XUNITS) {
        const int row = e >> 1;  // chunk-in-group * KP + column
        *reinterpret_cast<u4v*>(dst + row * XROW + (e & 1) * 16) = src[u];
      }
    }
  };
  // group g (register stage g % S): request the X^T and A groups PF ahead,
  // multiply group g, store the X^T group one ahead for the next group
  auto group = [&](int g, const v4i(&cur)[XG], v4i(&ahead)[XG], const u4v(&xnext)[XPT],
                   u4v(&xahead)[XPT]) {
    const int8_t* xst = xs + (g & 1) * XSTAGE;
    load_x(xahead, g + PF);
    load_a(ahead, g + PF);
#pragma unroll
    for (int cc = 0; cc < XG; ++cc) {
#pragma unroll
      for (int q = 0; q < KT; ++q) {
        const v4i xf = *reinterpret_cast<const v4i*>(
            xst + (cc * KP + 32 * q + (lane & 31)) * XROW + (lane >> 5) * 16);
        acc[q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xf, cur[cc], acc[q], 0, 0, 0);
      }
    }
    store_x(xnext, xs + ((g + 1) & 1) * XSTAGE);
    __syncthreads();
  };

#pragma unroll
  for (int u = 0; u < PF; ++u) {
    load_x(x[u], u);
    load_a(a[u], u);
  }
  store_x(x[0], xs);
  __syncthreads();
  for (int g = 0; g < ngroups; g += S) {
#pragma unroll
    for (int u = 0; u < S; ++u)
      if (g + u < ngroups) group(g + u, a[u], a[(u + PF) % S], x[(u + 1) % S], x[(u + PF) % S]);
  }

  // residues of the INT32 sums (|sum| <= n 2^14 < 2^31), one byte each;
  // registers 4 g4 .. 4 g4 + 3 of tile q hold the columns 32 q + 8 g4 +
  // 4 (l/32) + 0..3 of row i
  const int m = CRT_MOD[t];
  const double inv = 1.0 / (double)m;
  const int i = wrow + (lane & 31);
  int8_t* out = ca.cres + t * ca.cres_plane + (int64_t)i * KP;
#pragma unroll
  for (int q = 0; q < KT; ++q)
#pragma unroll
    for (int g4 = 0; g4 < 4; ++g4) {
      int r4[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) r4[e] = bal_res((double)acc[q][4 * g4 + e], m, inv);
      *gst(reinterpret_cast<unsigned*>(out + 32 * q + 8 * g4 + 4 * (lane >> 5))) =
          pack4(r4[0], r4[1], r4[2], r4[3]);
    }
}

// ---------------------------------------------------------------------------
// Reconstruction: work item = row block of RROWS rows; thread (row, column)
// with the columns spread over pow2ceil(k) threads.  Writes W_hi, W_lo and
// the block's Rayleigh partials (x w_hi, x x).
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(512) void crt_recon_kernel(const Prob* __restrict__ probs,
                                                        const RowItem* __restrict__ items,
                                                        int rrows, CrtArgs ca) {
  constexpr int NT = 512;
  constexpr CrtSum<N> K{};
  __shared__ double red[8 * NT];
  const Prob& P = probs[0];
  if (P.ctrl->stopped) return;
  const int blk = items[blockIdx.x].blk;
  const int n = P.n, k = P.k, kpad = P.kpad;
  // thread (trow, quad): columns 4 quad .. 4 quad + 3 of the rows trow,
  // trow + tr, ...; the Rayleigh partials then go through the column layout
  // of rayleigh_block_partial (thread (row, column) of pow2ceil(k) columns)
  const int nq = kpad / 4, tr = NT / nq;
  const int tid = threadIdx.x, quad = tid % nq, trow = tid / nq;
  const int r0 = blk * rrows, r1 = min(n, r0 + rrows);
  int sbase[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int j = 4 * quad + e;
    const int xe = *gld(P.xexp + min(j, k - 1));  // requested together
    sbase[e] = (trow < tr && j < k) ? xe - ca.ba - ca.bx : 0;
  }
  double sxw[4] = {0.0, 0.0, 0.0, 0.0}, sxx[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = r0 + trow; i < r1 && trow < tr; i += tr) {
    unsigned raw[N];
#pragma unroll
    for (int t = 0; t < N; ++t)
      raw[t] = *gld(reinterpret_cast<const unsigned*>(ca.cres + t * ca.cres_plane +
                                                     (int64_t)i * kpad + 4 * quad));
    const int ea = *gld(P.aexp + i);
    const double dii = *gld(ca.adiag + i);
    // the row's X entries with its residue words (columns past k clamped)
    double xr[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) xr[e] = *gld(P.x + (int64_t)i * P.ldx + min(4 * quad + e, k - 1));
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = 4 * quad + e;
      if (j >= k) continue;
      // S_k = sum_t c_t e_tk, exact (|S_k| < 2^43)
      double S[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < N; ++t) {
        const double c = (double)(int)(int8_t)((raw[t] >> (8 * e)) & 0xffu);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) S[kk] = __builtin_fma(c, K.e[t][kk], S[kk]);
      }
      // q = round(S / M); D_k = S_k - q M_k exact; A'X' = sum_k D_k 2^(32 k)
      const double sapp =
          ((S[3] * 4294967296.0 + S[2]) * 4294967296.0 + S[1]) * 4294967296.0 + S[0];
      const double q = __builtin_rint(sapp * K.minv);
      double D[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) D[kk] = __builtin_fma(-q, K.mk[kk], S[kk]);
      double h = D[3] * 0x1p96, l = 0.0;
#pragma unroll
      for (int kk = 2; kk >= 0; --kk) {
        double s1, e1;
        two_sum(h, D[kk] * (kk == 2 ? 0x1p64 : kk == 1 ? 0x1p32 : 1.0), s1, e1);
        e1 += l;
        two_sum(s1, e1, h, l);
      }
      const int sc = sbase[e] + ea;
      h = ldexp(h, sc);
      l = ldexp(l, sc);
      // + a_ii x_ij: (h, l) + (p, pe), both parts' errors kept
      const double xv = xr[e];
      double p, pe, s1, e1, s2, e2, wh, wl;
      two_prod(dii, xv, p, pe);
      two_sum(h, p, s1, e1);
      two_sum(l, pe, s2, e2);
      e1 += s2;
      two_sum(s1, e1, s1, e1);
      e1 += e2;
      two_sum(s1, e1, wh, wl);
      P.w[(int64_t)i * k + j] = wh;
      P.wlo[(int64_t)i * k + j] = wl;
      sxw[e] = __builtin_fma(xv, wh, sxw[e]);
      sxx[e] = __builtin_fma(xv, xv, sxx[e]);
    }
  }
  // column sums of the block (the Rayleigh partials): thread (trow, quad)
  // holds its 4 columns at red[trow kpad + 4 quad + e] = red[4 tid + e]; the
  // rows of threads are then added in a fixed order, so the sums do not
  // depend on scheduling
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    red[4 * tid + e] = trow < tr ? sxw[e] : 0.0;
    red[4 * NT + 4 * tid + e] = trow < tr ? sxx[e] : 0.0;
  }
  __syncthreads();
  for (int c = tid; c < k; c += NT) {
    double a = 0.0, b = 0.0;
    for (int r = 0; r < tr; ++r) {
      a += red[r * kpad + c];
      b += red[4 * NT + r * kpad + c];
    }
    P.dpart[(int64_t)blk * 2 * k + c] = a;
    P.dpart[(int64_t)blk * 2 * k + k + c] = b;
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

// rows per reconstruction block: 512 threads on 64 rows keep two wavefronts
// per SIMD at n = 16384 while halving the Rayleigh partials that the
// reduction after the product reads, against 256 threads on 32 rows
constexpr int CRT_RROWS = 64;

// Launch shapes of the residue products: wavefronts per block (32 W rows
// each) and chunks per group.  The tuner times each at init.
struct CrtShape {
  int waves, xg, pf;
};
constexpr CrtShape CRT_SHAPES[] = {{8, 2, 2}, {8, 2, 3}, {8, 1, 4}, {8, 4, 2}, {4, 2, 3},
                                     {4, 4, 2}, {16, 2, 2}, {16, 2, 3}};
constexpr int CRT_NSHAPES = sizeof(CRT_SHAPES) / sizeof(CRT_SHAPES[0]);
// order in which the tuner times them: 16 wavefronts (512 W rows, half the
// blocks of 8) first, since they lead where the row count allows them
constexpr int CRT_TRY_ORDER[CRT_NSHAPES] = {6, 7, 0, 1, 2, 3, 4, 5};

int rows_pad_of(int64_t n) { return (int)((n + SPLIT_ROW_PAD - 1) / SPLIT_ROW_PAD * SPLIT_ROW_PAD); }

CrtArgs args_of(const SplitPlan& sp, int64_t n) {
  CrtArgs ca{};
  const int64_t nch = (n + 31) / 32;
  ca.ares = sp.ares;
  ca.ares_plane = sp.ares_plane;
  ca.xres = sp.xres;
  ca.xres_plane = sp.xres_plane;
  ca.cres = sp.cres;
  ca.cres_plane = (int64_t)rows_pad_of(n) * sp.kpad;
  ca.adiag = sp.adiag;
  ca.nchp = (int)((nch + XG_PAD - 1) / XG_PAD * XG_PAD);
  ca.ba = sp.crt_ba;
  ca.bx = sp.crt_bx;
  return ca;
}

template <int KT, int WAVES, int XG, int PF>
void launch_gemm_shape(const SplitPlan& sp, const Prob* dprob, const CrtArgs& ca, hipStream_t st) {
  hipLaunchKernelGGL((crt_gemm_kernel<KT, WAVES, XG, PF>), dim3(sp.nitems), dim3(WAVES * 64), 0,
                     st, dprob, sp.items, ca);
}

template <int KT>
hipError_t launch_gemm_kt(const SplitPlan& sp, const Prob* dprob, const CrtArgs& ca,
                          hipStream_t st) {
  const CrtShape s = CRT_SHAPES[sp.crt_shape];
#define RFK_SHAPE(W, G, F) \
  if (s.waves == W && s.xg == G && s.pf == F) launch_gemm_shape<KT, W, G, F>(sp, dprob, ca, st); else
  RFK_SHAPE(8, 2, 2)
  RFK_SHAPE(8, 2, 3)
  RFK_SHAPE(8, 1, 4)
  RFK_SHAPE(8, 4, 2)
  RFK_SHAPE(4, 2, 3)
  RFK_SHAPE(4, 4, 2)
  RFK_SHAPE(16, 2, 2)
  RFK_SHAPE(16, 2, 3)
  { return hipErrorInvalidValue; }
#undef RFK_SHAPE
  return hipGetLastError();
}

template <int N>
hipError_t launch_all_n(const SplitPlan& sp, const Prob* dprob, const CrtArgs& ca, int64_t units,
                        hipStream_t st) {
  const int grid = (int)std::min<int64_t>((2 * units + 255) / 256, 16384);
  hipLaunchKernelGGL((crt_xres_kernel<N>), dim3(grid), dim3(256), 0, st, dprob, ca);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  product_mark(st);
  switch (sp.kpad / 32) {
    case 1: e = launch_gemm_kt<1>(sp, dprob, ca, st); break;
    case 2: e = launch_gemm_kt<2>(sp, dprob, ca, st); break;
    case 3: e = launch_gemm_kt<3>(sp, dprob, ca, st); break;
    case 4: e = launch_gemm_kt<4>(sp, dprob, ca, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  product_mark(st);
  hipLaunchKernelGGL((crt_recon_kernel<N>), dim3(sp.n_rec), dim3(512), 0, st, dprob, sp.rec_items,
                     sp.crt_rrows, ca);
  e = hipGetLastError();
  product_mark(st);
  return e;
}

template <int N>
hipError_t launch_ares_n(const refine_matrix& A, int rows_pad, const CrtArgs& ca,
                         const int32_t* aexp, hipStream_t st) {
  const int64_t units = (int64_t)rows_pad * ca.nchp * 2;
  const int grid = (int)std::min<int64_t>((units + 255) / 256, 16384);
  hipLaunchKernelGGL((crt_ares_kernel<N>), dim3(grid), dim3(256), 0, st, A.a, A.lda, (int)A.n,
                     rows_pad, CRT_TILE, ca, aexp);
  return hipGetLastError();
}

#define RFK_CRT_SWITCH(N, CALL) \
  switch (N) {                  \
    case 12: return CALL(12);   \
    case 13: return CALL(13);   \
    case 14: return CALL(14);   \
    case 15: return CALL(15);   \
    case 16: return CALL(16);   \
    default: return hipErrorInvalidValue; \
  }

template <class T>
hipError_t upload_items(T** dst, const std::vector<T>& v) {
  (void)hipFree(*dst);
  *dst = nullptr;
  if (v.empty()) return hipSuccess;
  hipError_t e = hipMalloc((void**)dst, sizeof(T) * v.size());
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
}

// Product items for blocks of bm rows: the (modulus, row block) pairs in
// modulus-major order, so that the blocks running together share one or a
// few moduli, whose X^T residues every XCD's L2 then holds.  Giving each XCD
// a contiguous range of the pairs instead (dispatch slot s to XCD s % 8)
// measured 2-8 % slower.
std::vector<GemmItem> product_items(int nmod, int64_t n, int bm) {
  const int nrb = (int)((n + bm - 1) / bm);
  std::vector<GemmItem> gi((size_t)nmod * nrb);
  for (int lin = 0; lin < nmod * nrb; ++lin) {
    GemmItem g{};
    g.split = lin / nrb;
    g.row0 = (lin % nrb) * bm;
    g.k0 = 0;
    gi[lin] = g;
  }
  return gi;
}

int install_shape(SplitPlan& sp, int shape, int nmod, int64_t n) {
  sp.crt_shape = shape;
  sp.crt_bm = 32 * CRT_SHAPES[shape].waves;
  const std::vector<GemmItem> gi = product_items(nmod, n, sp.crt_bm);
  if (upload_items(&sp.items, gi) != hipSuccess) return REFINE_ENOMEM;
  sp.nitems = (int)gi.size();
  return REFINE_OK;
}

}  // namespace

int crt_bits(int nmod, int64_t n, int* ba, int* bx) {
  if (nmod < CRT_N_MIN || nmod > CRT_N_MAX || n < 1) return REFINE_EINVAL;
  // M < 2^126 for N <= 16: exact in 128 bits
  unsigned __int128 M = 1;
  for (int t = 0; t < nmod; ++t) M *= (unsigned)CRT_MOD[t];
  int L = 0;
  while (L < 128 && (M >> L) != 0) ++L;
  int c = 0;
  while (((int64_t)1 << c) < n) ++c;
  const int B = L - 3 - c;
  if (B < 2) return REFINE_EINVAL;
  *ba = (B + 1) / 2;
  *bx = B / 2;
  return REFINE_OK;
}

hipError_t crt_product(const SplitPlan& sp, const Prob* dprob, hipStream_t st) {
  hipError_t e = split_xmax(sp, dprob, st);
  if (e != hipSuccess) return e;
  const int64_t n = sp.nk0 / sp.kmax;
  const CrtArgs ca = args_of(sp, n);
  const int64_t units = (int64_t)ca.nchp * sp.kpad * 2;
#define RFK_CRT_ALL(N) launch_all_n<N>(sp, dprob, ca, units, st)
  RFK_CRT_SWITCH(sp.crt, RFK_CRT_ALL)
#undef RFK_CRT_ALL
}

int crt_init(SplitPlan& sp, const refine_matrix& A, int k, int nmod, std::vector<Prob>& hp,
             Prob* dprob, hipStream_t st) {
  const int64_t n = A.n;
  int ba = 0, bx = 0;
  if (A.kind != REFINE_DENSE || n > SPLIT_NMAX || crt_bits(nmod, n, &ba, &bx) != REFINE_OK)
    return REFINE_EINVAL;
  sp.crt = nmod;
  sp.crt_ba = ba;
  sp.crt_bx = bx;
  sp.crt_rrows = CRT_RROWS;
  const int rows_pad = rows_pad_of(n);
  const int64_t nch = (n + 31) / 32, nchp = (nch + XG_PAD - 1) / XG_PAD * XG_PAD;
  sp.ares_plane = (int64_t)rows_pad * nchp * 32;
  sp.xres_plane = nchp * sp.kpad * 32;
  const int64_t cres_bytes = (int64_t)rows_pad * sp.kpad * nmod;
  if (hipMalloc((void**)&sp.ares, (size_t)sp.ares_plane * nmod) != hipSuccess ||
      hipMalloc((void**)&sp.aexp, sizeof(int32_t) * rows_pad) != hipSuccess ||
      hipMalloc((void**)&sp.adiag, sizeof(double) * rows_pad) != hipSuccess ||
      hipMalloc((void**)&sp.xres, (size_t)sp.xres_plane * nmod) != hipSuccess ||
      hipMalloc((void**)&sp.cres, (size_t)cres_bytes) != hipSuccess)
    return REFINE_ENOMEM;
  hipError_t e = hipMemsetAsync(sp.xres, 0, (size_t)sp.xres_plane * nmod, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(crt_aexp_kernel, dim3((unsigned)((rows_pad + 3) / 4)), dim3(256), 0, st,
                       A.a, A.lda, (int)n, rows_pad, sp.aexp, sp.adiag);
    e = hipGetLastError();
  }
  const CrtArgs ca = args_of(sp, n);
  if (e == hipSuccess) {
#define RFK_CRT_ARES(N) launch_ares_n<N>(A, rows_pad, ca, sp.aexp, st)
    e = [&]() -> hipError_t { RFK_CRT_SWITCH(nmod, RFK_CRT_ARES) }();
#undef RFK_CRT_ARES
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return REFINE_EHIP;

  std::vector<RowItem> rec;
  const int nrec = (int)((n + CRT_RROWS - 1) / CRT_RROWS);
  for (int b = 0; b < nrec; ++b) rec.push_back(RowItem{0, b});
  if (upload_items(&sp.rec_items, rec) != hipSuccess) return REFINE_ENOMEM;
  sp.n_rec = nrec;
  sp.ks = 1;
  Prob& P = hp[0];
  P.aexp = sp.aexp;
  P.ksplit = 1;
  P.ndp = nrec;
  P.nch = (int)nch;
  P.kpad = sp.kpad;
  if (hipMemcpy(dprob, hp.data(), sizeof(Prob) * hp.size(), hipMemcpyHostToDevice) != hipSuccess)
    return REFINE_EHIP;

  // Launch shape of the residue products: REFINE_CRT_SHAPE=<index> forces
  // one; otherwise each is timed once (on a zero X, the workspace copy of
  // the update) in the order above, and a later shape replaces the one kept
  // only when it is more than 2 % faster, so that shapes within the timing noise of each
  // other do not alternate between processes.
  // a shape's row block (32 W rows per wavefront) must divide the padded row
  // count, which bounds the residue planes the products read and write
  auto fits = [&](int sh) {
    return sh >= 0 && sh < CRT_NSHAPES && rows_pad % (32 * CRT_SHAPES[sh].waves) == 0;
  };
  int best = -1;
  if (const char* env = getenv("REFINE_CRT_SHAPE")) {
    const int v = atoi(env);
    if (fits(v)) best = v;
  }
  const std::vector<int64_t> key{n, k, nmod};
  if (best < 0) {
    std::vector<int> hit;
    if (tune_cache_get("crt", key, &hit) && hit.size() == 1 && fits(hit[0])) best = hit[0];
  }
  if (best < 0) {
    const double* saved_x = hp[0].x;
    const int64_t saved_ld = hp[0].ldx;
    hp[0].x = hp[0].xn;
    hp[0].ldx = hp[0].k;
    if (hipMemcpy(dprob, hp.data(), sizeof(Prob) * hp.size(), hipMemcpyHostToDevice) != hipSuccess)
      return REFINE_EHIP;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return REFINE_EHIP;
    float best_t = 1e30f;
    for (int i = 0; i < CRT_NSHAPES && e == hipSuccess; ++i) {
      const int sh = CRT_TRY_ORDER[i];
      if (!fits(sh)) continue;
      int rc = install_shape(sp, sh, nmod, n);
      if (rc != REFINE_OK) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return rc;
      }
      float t = 0.f;
      e = crt_product(sp, dprob, st);  // warm-up
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      for (int r = 0; r < 3 && e == hipSuccess; ++r) e = crt_product(sp, dprob, st);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
      if (getenv("REFINE_LOG") && atoi(getenv("REFINE_LOG")) >= 2)
        fprintf(stderr, "refine: tune crt n=%lld k=%d N=%d shape %d (waves %d, group %d, ahead %d): %.1f us\n",
                (long long)n, k, nmod, sh, CRT_SHAPES[sh].waves, CRT_SHAPES[sh].xg,
                CRT_SHAPES[sh].pf, t * 1000.f / 3.f);
      if (e == hipSuccess && t < 0.98f * best_t) {
        best_t = t;
        best = sh;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    hp[0].x = const_cast<double*>(saved_x);
    hp[0].ldx = saved_ld;
    if (e != hipSuccess || best < 0) return REFINE_EHIP;
    sp.ms = best_t / 3.f;
    tune_cache_put("crt", key, {best});
    if (getenv("REFINE_LOG"))
      fprintf(stderr, "refine: crt product n=%lld k=%d N=%d: shape %d, %.1f us\n", (long long)n, k,
              nmod, best, best_t * 1000.f / 3.f);
  }
  int rc = install_shape(sp, best, nmod, n);
  if (rc != REFINE_OK) return rc;
  if (hipMemcpy(dprob, hp.data(), sizeof(Prob) * hp.size(), hipMemcpyHostToDevice) != hipSuccess)
    return REFINE_EHIP;
  return REFINE_OK;
}

}  // namespace rfk
