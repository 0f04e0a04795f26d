// Split form of the dense product W = A X (product step of Algorithm 4, computed
// the accelerator way that Sec. 3.1.3 points to): error-free splitting of A and
// X into INT8 digit slices (Ozaki, Ogita, Oishi and Rump 2012, with integer
// slices as in Ootomo, Ozaki and Yokota 2024), exact INT32 products on the
// matrix cores, and a double-double result (Prob::w, Prob::wlo).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "common.h"
#include "refine.h"

namespace rfk {

// Supported slice counts and the default.
constexpr int SPLIT_S_MIN = 7;
constexpr int SPLIT_S_MAX = 10;
constexpr int SPLIT_S_DEFAULT = 9;
// Largest K split of the split product.
constexpr int SPLIT_KS_MAX = 8;
// Largest n: the slices of A take s * n^2 bytes, and the int32 row offsets
// of the kernels stay in range.
constexpr int64_t SPLIT_NMAX = 65536;
// Rows of A's slices are padded to a multiple of this (the largest row block).
constexpr int SPLIT_ROW_PAD = 256;

// Modular form (Ozaki scheme II): supported moduli counts and the default.
constexpr int CRT_N_MIN = 12;
constexpr int CRT_N_MAX = 16;
constexpr int CRT_N_DEFAULT = 16;

struct SplitPlan {
  int s = 0;                  // slices per operand
  int ks = 1;                 // K split (one problem only)
  int variant = 0;            // 0: tiles staged through registers, 1: direct-to-LDS loads,
                              // 2: direct-to-LDS rings (X two stages, A deeper)
  int bm = 0;                 // rows per block of the product
  int kmax = 0;               // largest k of the problems
  int kpad = 0;               // kmax rounded up to 32 (the column tile of every problem)
  int np = 0;                 // problems
  int64_t nk0 = 0;            // n k of problem 0 (K-split sum)
  uint8_t* asl = nullptr;     // slices of every A (per problem s * rows_pad * nch * 32 bytes)
  int32_t* aexp = nullptr;    // per-row exponents
  uint8_t* xsl = nullptr;     // slices of every X^T (per problem s * nch * kpad * 32 bytes)
  int32_t* xexp = nullptr;    // per-column exponents, kpad per problem
  double* xmaxp = nullptr;    // column maxima, kpad per problem
  double* swp = nullptr;      // K-split partials (hi, lo), one problem only
  GemmItem* items = nullptr;  // product work items
  int nitems = 0;
  RowItem* xmax_items = nullptr;  // (problem, row block) of the column-maximum pass
  int n_xmax = 0;
  RowItem* xsl_items = nullptr;   // (problem, 256 units) of the X slicing pass
  int n_xsl = 0;
  float ms = 0.f;             // product time measured by the tuner
  // modular form (crt > 0: that many moduli; the fields above that hold
  // slices are unused, xmaxp/xexp/items serve both forms)
  int crt = 0;
  int crt_ba = 0, crt_bx = 0; // bit budgets of the scaled operands
  int crt_bm = 0;             // rows per block of the residue products
  int crt_shape = 0;          // launch shape of the residue products (tuned)
  double* adiag = nullptr;    // diagonal of A (rows_pad entries)
  int crt_rrows = 0;          // rows per block of the reconstruction
  int8_t* ares = nullptr;     // residues of A, crt planes of rows_pad x nch*32 bytes
  int64_t ares_plane = 0;     // bytes per plane
  int8_t* xres = nullptr;     // residues of X^T, crt planes of nch x kpad x 32 bytes
  int64_t xres_plane = 0;
  int8_t* cres = nullptr;     // residues of A'X', 16 bytes per entry (rows_pad x kpad)
  RowItem* rec_items = nullptr;   // (problem, row block) of the reconstruction
  int n_rec = 0;
};

// Slices every A (read only here), chooses the K split (one problem) and the
// tile-loading variant, fills the split fields of hp and uploads hp to dprob.
// Returns a REFINE_* status.
// crt > 0 selects the modular form with that many moduli (one problem; slices
// is then ignored).
int split_init(SplitPlan& sp, const std::vector<refine_matrix>& As, const std::vector<int>& ks,
               int slices, int crt, std::vector<Prob>& hp, Prob* dprob, hipStream_t st);
// Enqueues the whole split product of every problem: column maxima and
// slices of X, the INT8 products, and the K-split sum.
hipError_t split_product(const SplitPlan& sp, const Prob* dprob, hipStream_t st);
void split_free(SplitPlan& sp);
// Rows per block of the split product for k columns (for sizing partials).
int split_rows_per_block(int k);

// Modular form of the product (Ozaki scheme II, one problem): bit budgets
// for nmod moduli and contraction length n (REFINE_EINVAL when out of range).
int crt_bits(int nmod, int64_t n, int* ba, int* bx);
// Residues of A (read only here), the work items and partial slots.  The
// plan's xmaxp/xexp/xmax_items are set by the caller's split_init.
int crt_init(SplitPlan& sp, const refine_matrix& A, int k, int nmod, std::vector<Prob>& hp,
             Prob* dprob, hipStream_t st);
// Column maxima and residues of X, the residue products and the
// reconstruction of W (hi, lo) with the Rayleigh partials.
hipError_t crt_product(const SplitPlan& sp, const Prob* dprob, hipStream_t st);
// Measurement hook of refine_time_product_parts (in refine_api.hip): while a
// timing is armed, records an event on `st` after each launch of the
// product; otherwise does nothing.
void product_mark(hipStream_t st);
// Column maxima of |X| for both forms, and row exponents of A (in k_split.hip).
hipError_t split_xmax(const SplitPlan& sp, const Prob* dprob, hipStream_t st);
hipError_t split_aexp(const refine_matrix& A, int rows_pad, int32_t* aexp, hipStream_t st);

}  // namespace rfk
