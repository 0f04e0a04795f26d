// Split-precision product W = A X (line 1 of Algorithm 4) by error-free
// splitting of A and X into INT8 slices with exact INT32 accumulation on the
// matrix cores; W comes back as a double-double pair (Prob::w, Prob::wlo).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"
#include "refine.h"

namespace rfk {

// Largest n the INT32 accumulators can take exactly (see k_split.hip).
constexpr int64_t SPLIT_NMAX = 65536;

struct SplitPlan {
  int s = 0;                // slices per operand
  int64_t n = 0;
  int k = 0;
  int8_t* a_sl = nullptr;   // s slices of A, each n x n row-major (ld = lda_sl)
  int64_t lda_sl = 0;
  int32_t* a_exp = nullptr; // per-row exponents of A
  int8_t* x_sl = nullptr;   // s slices of X^T, each kpad x n (column j of X contiguous)
  int32_t* x_exp = nullptr; // per-column exponents of X
  double* x_part = nullptr; // per-block column maxima
  int32_t* c_acc = nullptr; // INT32 sums, per diagonal p+q
  int nblk = 0;
  int kpad = 0;
  int ksplit = 1;
  void* items = nullptr;
  int nitems = 0;
  Prob* dprob = nullptr;
};

int split_init(SplitPlan& sp, const refine_matrix& A, int k, int slices, const Prob& hp,
               Prob* dprob, hipStream_t st);
hipError_t split_product(SplitPlan& sp, const Prob* dprob, hipStream_t st);
void split_free(SplitPlan& sp);

}  // namespace rfk
