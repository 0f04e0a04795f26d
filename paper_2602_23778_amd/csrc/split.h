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
};

// Slices every A (read only here), chooses the K split (one problem) and the
// tile-loading variant, fills the split fields of hp and uploads hp to dprob.
// Returns a REFINE_* status.
int split_init(SplitPlan& sp, const std::vector<refine_matrix>& As, const std::vector<int>& ks,
               int slices, std::vector<Prob>& hp, Prob* dprob, hipStream_t st);
// Enqueues the whole split product of every problem: column maxima and
// slices of X, the INT8 products, and the K-split sum.
hipError_t split_product(const SplitPlan& sp, const Prob* dprob, hipStream_t st);
void split_free(SplitPlan& sp);
// Rows per block of the split product for k columns (for sizing partials).
int split_rows_per_block(int k);

}  // namespace rfk
