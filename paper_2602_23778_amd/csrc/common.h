// Device-side data structures shared by the refinement kernels and the host
// runtime of the library.  Nothing here is part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rfk {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef int v4i __attribute__((ext_vector_type(4)));

// Largest number of target vectors a problem may have on this path.
constexpr int KMAX = 128;

// Per-problem control word block (device memory, one per problem).
//   stopped: set when the iteration must not continue (error, converged,
//            diverged); every kernel of later steps checks it first.
//   apply:   cleared by the k-by-k kernel at the start of each step and set
//            by the update kernel when the step's correction is accepted;
//            the final normalisation pass writes X only when it is set.
struct Ctrl {
  int32_t stopped;
  int32_t apply;
  int32_t status;     // sticky status code of the first failing step
  int32_t iters;      // steps applied since the last reset
  int32_t stop_mode;  // 0 fixed count, 1 ||E_L||_F <= tol, 2 residual <= tol
  int32_t converged;
  double tol;
  double corr_fro;    // statistics of the last step
  double resid_rel;
  double hist[4];     // ||E_L||_F of the last applied steps (ring)
  int32_t kxk_fb;     // this step's k-by-k work falls back to the one-workgroup solver
  int32_t rr_top;     // X is a Rayleigh-Ritz basis: the next applied step takes E11 = 0
};

// One problem: a symmetric matrix, its iterate and its workspace slices.
struct Prob {
  // matrix
  const double* a;        // dense, row-major, lda
  int64_t lda;
  const int32_t* rp;      // CSR
  const int32_t* ci;
  const double* av;
  // caller's iterate, n x k row-major with leading dimension ldx
  double* x;
  int64_t ldx;
  int32_t n, k;
  int32_t kind;           // 0 dense, 1 CSR
  int32_t ksplit;         // K splits of the dense product (1: W written directly)
  int32_t nrb;            // row blocks of the streaming passes
  int32_t rbrows;         // rows per row block (multiple of 128)
  int32_t ngb;            // row blocks of the Gram pass
  int32_t gbrows;         // rows per Gram block (>= 128, so rows < k sit in block 0)
  // workspace
  double* wp;             // ksplit partial products, each n x k (ld k)
  double* w;              // W = A X (high part in split mode), n x k
  double* wlo;            // low part of W (split mode) or nullptr
  double* xn;             // unnormalised update, n x k
  double* part;           // row-block partials of the update, nrb x (5 k)
  double* dpart;          // Rayleigh-quotient partials, ndp x (2 k): sums of x*w, x*x
  int32_t ndp;
  double* gpart;          // Gram partials, ngb x (2 k k + k)
  double* kk;             // k-by-k area (see KK_* offsets)
  double* kpp;            // partial sums of the k-by-k panel pipeline (16 + 16 k doubles)
  double* vec;            // vectors of length k (see VEC_* offsets)
  Ctrl* ctrl;
  double mu;              // shift: targets are the largest |lambda - mu|
  double delta;           // cluster threshold c ||A|| u
  double norm_a;          // ||A|| used in the residual statistic
  int32_t beta_zero;
  int32_t normalize;
  // squared variant (B = A^2 - mu I): W = A W1 with W1 = A X; the products run
  // from two derived descriptors, the first writing its Rayleigh partials
  // (x*w1, x*x) to dpx, the second (w1*w, w1*w1) to dpart
  int32_t square;
  double* w1;             // A X, n x k (ld k), or nullptr
  double* dpx;            // partials of the first product, ndp x (2 k), or nullptr
  // split form of the dense product (INT8 slices); unused otherwise
  const uint8_t* asl;     // slices of A in tiles of bm rows x 32 columns: the row block
                          // starting at row i0 at asl + i0*asl_rs, its chunk c, row r at
                          // + (c*bm + r)*32*s
  int64_t asl_rs;         // bytes of asl per row of A (nch chunks)
  const int32_t* aexp;    // per-row scale exponents of A (rows padded with 0)
  uint8_t* xsl;           // slices of X^T: chunk c, column j at xsl + (c*kpad + j)*32*s
  int32_t* xexp;          // per-column scale exponents of X (kpad entries)
  double* xmaxp;          // column maxima of |X| (kpad entries), merged by atomic maximum
  double* swp;            // K-split partials of the split product: ksplit x (hi, lo) x n x k
  int32_t nch;            // 32-wide contraction chunks (ceil(n / 32))
  int32_t kpad;           // k rounded up to 32
  int32_t nbx;            // row blocks of the column-maximum pass
  int32_t xrows;          // rows per such block
};

// Offsets (in units of k*k doubles) inside Prob::kk.
enum {
  KK_P2 = 0,    // X2^T R2 (rows >= k)
  KK_G2 = 1,    // X2^T X2
  KK_PT = 2,    // X1^T R1 (rows < k)
  KK_GT = 3,    // X1^T X1
  KK_R1 = 4,    // R1, the leading k rows of R
  KK_CM = 5,    // [M | N], k x 2k (occupies 5 and 6)
  KK_X1N = 7,   // updated leading rows
  KK_S0 = 8,    // scratch for the k-by-k solver when it does not fit in LDS (8..11)
  KK_FC = 9,    // fused update after the panel pipeline: C = M Delta + N (in the slot of X^T R - R1,
                //   which the product for M consumed)
  KK_FQ = 10,   // fused update after the panel pipeline: per-panel column parts of the statistics
                //   (in the slot of E11, which X1's update consumed)
  KK_Z = 12,    // Y1^{-1} of the previous step (warm start)
  KK_Q = 13,    // Y1 Z^T (panel pipeline)
  KK_COUNT = 14
};
// Offsets (in units of k doubles) inside Prob::vec.
enum {
  VEC_D = 0,       // Rayleigh quotients
  VEC_ALPHA = 1,   // x_j^T x_j
  VEC_DINV = 2,    // 1 / (d_j - mu)
  VEC_SCALE = 3,   // column normalisation factors
  VEC_RSQ = 4,     // column sums of r^2 (reduced)
  VEC_E1SQ = 5,    // slot 0: ||E11||_F^2
  VEC_COUNT = 6
};

// Work items.  Dense product: rows [row0, row0 + BM) against K range [k0, k1)
// of problem `prob`, written to partial `split`.
struct GemmItem {
  int32_t prob, row0, k0, k1;
  int32_t split, pad0, pad1, pad2;
};
// Streaming passes: row block `blk` of problem `prob`.
struct RowItem {
  int32_t prob, blk;
};

constexpr double UNIT_ROUNDOFF = 1.1102230246251565e-16;  // 2^-53

// v_mfma_f64_16x16x4_f64: lane l supplies a[i = l%16][k = l/16] and
// b[k = l/16][j = l%16]; the 16x16 result sits in four registers per lane,
// register r of lane l holding d[i = l/16 + 4r][j = l%16] (checked on gfx950
// with a lane-layout probe).
__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// Row of the 16x16 result held in register r by a lane of group g = l/16.
__device__ __forceinline__ int mfma_row(int g, int r) { return g + 4 * r; }

// Global-memory views of generic pointers.  A load or store through a
// generic pointer (every pointer read from a Prob) compiles to a FLAT
// instruction, which also counts against the LDS wait counter: a kernel that
// waits for its LDS reads then waits for its global prefetches as well.  The
// global forms keep the two apart.
#define RFK_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const RFK_GLOBAL T* gld(const T* p) {
  return (const RFK_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ RFK_GLOBAL T* gst(T* p) {
  return (RFK_GLOBAL T*)p;
}

// base[i] where ok holds, else zero, by an unconditional load of base[ok ? i
// : 0] (base[0] must be readable).  A guarded load (ok ? base[i] : 0) becomes
// a branch around the load, and the join waits for it, so a run of them
// costs one memory round trip each; these can all be in flight at once.
template <class T>
__device__ __forceinline__ T ld_or0(bool ok, const T* base, int64_t i) {
  const T v = *gld(base + (ok ? i : 0));
  return ok ? v : T(0);
}

// Exact transformations used by the accurate residual (Dekker / Knuth).
// Floating-point contraction is off inside them: a product fused into a
// later subtraction would be rounded differently from the product the error
// term describes (the compiler fuses by default in device code).
__device__ __forceinline__ void two_prod(double a, double b, double& p, double& e) {
#pragma clang fp contract(off)
  p = a * b;
  e = __builtin_fma(a, b, -p);
}
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = a + b;
  double z = s - a;
  e = (a - (s - z)) + (b - z);
}

// r = (w_hi + w_lo) - x d with x d formed exactly; without a low part it is
// w - x d rounded once (a fused multiply-add).
__device__ __forceinline__ double residual(double w, double wlo, double x, double d, bool has_lo) {
#pragma clang fp contract(off)
  if (!has_lo) return __builtin_fma(-x, d, w);
  double p, pe;
  two_prod(x, d, p, pe);
  return (w - p) + (wlo - pe);
}

// Launchers implemented in the .hip files.
struct LaunchCfg {
  hipStream_t stream;
};

}  // namespace rfk
