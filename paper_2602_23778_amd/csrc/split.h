// Split form of the dense product W = A X (line 1 of Algorithm 4, computed
// the accelerator way that Sec. 3.3 points to): error-free splitting of A and
// X into INT8 digit slices (Ozaki, Ogita, Oishi and Rump 2012, with integer
// slices as in Ootomo, Ozaki and Yokota 2024), exact INT32 products on the
// matrix cores, and a double-double result (Prob::w, Prob::wlo).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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
  int ks = 1;                 // K split
  int variant = 0;            // 0: tiles staged through registers, 1: direct-to-LDS loads
  int bm = 0;                 // rows per block of the product
  int64_t n = 0;
  int k = 0;
  int nch = 0;                // 32-wide contraction chunks
  int kpad = 0;               // k rounded up to 32
  int nbx = 0;                // blocks of the column-maximum pass
  int xrows = 0;              // rows per such block
  uint8_t* asl = nullptr;     // slices of A (s * rows_pad * nch * 32 bytes)
  int32_t* aexp = nullptr;    // per-row exponents
  uint8_t* xsl = nullptr;     // slices of X^T (s * nch * kpad * 32 bytes)
  int32_t* xexp = nullptr;
  double* xmaxp = nullptr;    // column-maximum partials
  double* swp = nullptr;      // K-split partials (hi, lo)
  GemmItem* items = nullptr;
  int nitems = 0;
  float ms = 0.f;             // product time measured by the tuner
};

// Slices A (read only here), chooses the K split, fills the split fields of
// hp and uploads hp to dprob.  Returns a REFINE_* status.
int split_init(SplitPlan& sp, const refine_matrix& A, int k, int slices, Prob& hp, Prob* dprob,
               hipStream_t st);
// Enqueues the whole split product for problem dprob[0]: column maxima and
// slices of X, the INT8 products, and the K-split sum.
hipError_t split_product(const SplitPlan& sp, const Prob* dprob, hipStream_t st);
void split_free(SplitPlan& sp);
// Rows per block of the split product for k columns (for sizing partials).
int split_rows_per_block(int k);

}  // namespace rfk
