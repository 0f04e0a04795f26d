/*
 * oracle.c -- plain, slow CPU reference for one refinement step of the
 * subset-eigenvector iterative refinement of Terao, Ozaki, Imamura and Ogita
 * ("Iterative Refinement for a Subset of Eigenvectors of Symmetric Matrices
 * via Matrix Multiplications", arXiv 2602.23778).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
 * CPU-baseline leg of the benchmark may call this code.  It shares nothing
 * (no header, helper, table or constant) with the GPU library.
 *
 * Every routine below is written in plain loops, in IEEE double precision,
 * with a fixed ascending summation order.  OpenMP only splits independent
 * output rows across threads, so results do not depend on the thread count.
 * Build with -ffp-contract=off so that no multiply-add is fused behind our
 * back; the only fused multiply-adds are the explicit fma() calls of the
 * error-free product (Dekker / Knuth TwoProduct).
 *
 * Readings of the paper that this file takes (each is also listed with its
 * reason in the design notes):
 *   - the off-diagonal top block of the correction uses v_ij / (d_j - d_i),
 *     as in eq. (Eoffdiag) and the correction step of Algorithm 4; the sign printed in
 *     eq. (V-def) is inconsistent with eqs. (R) and (S) (a test plants that
 *     sign here, on purpose, to show it diverges);
 *   - a spectral shift mu is applied as the paper's variant does: the method
 *     runs on B = A - mu*I, i.e. W_B = A*X - mu*X and d_B = d - mu;
 *   - delta = c * normA * u with u = 2^-53 and normA supplied by the caller;
 *   - a tie |d_j - d_i| == delta takes the beta branch (the "<=" of Alg. 4);
 *   - Y1 counts as singular when a pivot is exactly zero or when the
 *     1-norm condition number of Y1 exceeds 1/(n*u);
 *   - the statistics (||E_L||_F and ||R||_F / normA) describe the input X.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_SINGULAR (-4)
#define ORC_NONFINITE (-6)

static const double ORC_U = 1.1102230246251565e-16; /* 2^-53, unit roundoff */

/* ------------------------------------------------------------------------ */
/* Error-free transformations (Knuth TwoSum, Dekker TwoProduct via fma).    */
/* ------------------------------------------------------------------------ */
static void two_sum(double a, double b, double* s, double* e) {
  double x = a + b;
  double z = x - a;
  *e = (a - (x - z)) + (b - z);
  *s = x;
}
static void two_prod(double a, double b, double* p, double* e) {
  double x = a * b;
  *e = fma(a, b, -x);
  *p = x;
}

/* ------------------------------------------------------------------------ */
/* The product step of Algorithm 4: W = A * X.                              */
/* Dense A is row-major n x n with leading dimension lda; X and W are        */
/* row-major n x k.  For each output entry the products are summed in        */
/* ascending l; looping l outside j keeps that order while reading rows.     */
/* ------------------------------------------------------------------------ */
void orc_gemm_dense(int64_t n, int64_t k, const double* A, int64_t lda,
                    const double* X, int64_t ldx, double* W, int64_t ldw) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double* w = W + i * ldw;
    for (int64_t j = 0; j < k; ++j) w[j] = 0.0;
    for (int64_t l = 0; l < n; ++l) {
      double a = A[i * lda + l];
      const double* x = X + l * ldx;
      for (int64_t j = 0; j < k; ++j) w[j] += a * x[j];
    }
  }
}

/* Same product, each entry accumulated by the compensated dot product Dot2
 * of Ogita, Rump and Oishi (2005).  Returns W as an unevaluated pair
 * Whi + Wlo with Whi = fl(Whi + Wlo).                                        */
void orc_gemm_dense_dd(int64_t n, int64_t k, const double* A, int64_t lda,
                       const double* X, int64_t ldx, double* Whi, double* Wlo,
                       int64_t ldw) {
#pragma omp parallel
  {
    double* p = (double*)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
    double* s = (double*)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      for (int64_t j = 0; j < k; ++j) { p[j] = 0.0; s[j] = 0.0; }
      for (int64_t l = 0; l < n; ++l) {
        double a = A[i * lda + l];
        const double* x = X + l * ldx;
        for (int64_t j = 0; j < k; ++j) {
          double h, r, q;
          two_prod(a, x[j], &h, &r);
          two_sum(p[j], h, &p[j], &q);
          s[j] += q + r;
        }
      }
      for (int64_t j = 0; j < k; ++j) {
        double hi, lo;
        two_sum(p[j], s[j], &hi, &lo);
        Whi[i * ldw + j] = hi;
        Wlo[i * ldw + j] = lo;
      }
    }
    free(p);
    free(s);
  }
}

/* ------------------------------------------------------------------------ */
/* Split form of the product step of Algorithm 4 (as Sec. 3.1.3 suggests for  */
/* accelerators): the error-free splitting of Ozaki, Ogita, Oishi and Rump  */
/* (2012) with integer slices, as Ootomo, Ozaki and Yokota (2024) run it on  */
/* integer matrix units.                                                     */
/*                                                                           */
/* Slicing.  Every row of A (every column of X) gets a power-of-two scale    */
/* 2^E with E the smallest integer such that max |entry| < 2^E (E = 0 for an */
/* all-zero line).  The scaled value v = m * 2^(6-E) lies in (-64, 64) and   */
/* is peeled into s signed digits by rounding to nearest (ties to even):     */
/*     d_1 = rint(v),  v <- (v - d_1) * 2^7,  d_2 = rint(v),  ...            */
/* so every digit lies in [-64, 64] and                                      */
/*     m = 2^(E-6) * sum_p d_p 2^(-7(p-1))  +  r,   |r| <= 2^(E-7s).        */
/* Each step is exact in FP64 (scaling by powers of two, and subtracting the */
/* nearest integer).                                                         */
/*                                                                           */
/* Product.  With A_p, X_q the digit matrices, every product A_p X_q is an   */
/* exact integer matrix.  The products with p + q <= s + 1 are kept and      */
/* binned by t = p + q (the leading s(s+1)/2 terms of the expansion); the    */
/* result is                                                                 */
/*     W_ij = 2^(E_i + F_j - 12) * sum_t B_t[i][j] * 2^(-7(t-2)),            */
/* computed here exactly as a 128-bit integer and returned as a double-      */
/* double pair (hi, lo) with hi + lo equal to that value.                    */
/* ------------------------------------------------------------------------ */

/* Digits of a rows x cols row-major matrix M (leading dimension ld).
 * by_row = 1: one scale per row (A); 0: one scale per column (X).
 * D is s x rows x cols (plane p at D + p*rows*cols); Eexp has rows (or
 * cols) entries. */
void orc_split_digits(int64_t rows, int64_t cols, const double* M, int64_t ld,
                      int32_t by_row, int32_t s, int8_t* D, int32_t* Eexp) {
  const int64_t nline = by_row ? rows : cols;
  for (int64_t a = 0; a < nline; ++a) {
    double mx = 0.0;
    const int64_t len = by_row ? cols : rows;
    for (int64_t b = 0; b < len; ++b) {
      double v = by_row ? M[a * ld + b] : M[b * ld + a];
      if (fabs(v) > mx) mx = fabs(v);
    }
    int e = 0;
    if (mx > 0.0) frexp(mx, &e); /* mx = f 2^e with f in [1/2, 1): mx < 2^e */
    Eexp[a] = e;
  }
  for (int64_t i = 0; i < rows; ++i)
    for (int64_t j = 0; j < cols; ++j) {
      const int e = Eexp[by_row ? i : j];
      double v = ldexp(M[i * ld + j], 6 - e);
      for (int32_t p = 0; p < s; ++p) {
        double d = rint(v);
        D[(int64_t)p * rows * cols + i * cols + j] = (int8_t)d;
        v = ldexp(v - d, 7);
      }
    }
}

/* W = A X by the split form with s slices per operand (1 <= s <= 12).
 * A is n x n (row-major, lda), X is n x k (ldx); W and Wlo are n x k (ldw).
 * Bins are accumulated in 64-bit integers (exact for any n here). */
int orc_gemm_split(int64_t n, int64_t k, const double* A, int64_t lda,
                   const double* X, int64_t ldx, int32_t s, double* Whi,
                   double* Wlo, int64_t ldw) {
  if (s < 1 || s > 12) return ORC_EINVAL;
  int8_t* DA = (int8_t*)malloc((size_t)s * (size_t)(n * n));
  int8_t* DX = (int8_t*)malloc((size_t)s * (size_t)(n * k));
  int32_t* EA = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* EX = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  if (!DA || !DX || !EA || !EX) {
    free(DA); free(DX); free(EA); free(EX);
    return ORC_ENOMEM;
  }
  orc_split_digits(n, n, A, lda, 1, s, DA, EA);
  orc_split_digits(n, k, X, ldx, 0, s, DX, EX);
#pragma omp parallel
  {
    int64_t* bins = (int64_t*)malloc(sizeof(int64_t) * (size_t)(s + 2));
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < k; ++j) {
        for (int t = 0; t < s + 2; ++t) bins[t] = 0;
        for (int32_t p = 1; p <= s; ++p)
          for (int32_t q = 1; p + q <= s + 1; ++q) {
            const int8_t* ap = DA + (int64_t)(p - 1) * n * n + i * n;
            const int8_t* xq = DX + (int64_t)(q - 1) * n * k + j;
            int64_t acc = 0;
            for (int64_t l = 0; l < n; ++l) acc += (int64_t)ap[l] * (int64_t)xq[l * k];
            bins[p + q] += acc;
          }
        /* exact integer value of sum_t B_t 2^(7(s+1-t)) */
        __int128 tot = 0;
        for (int t = 2; t <= s + 1; ++t) tot += (__int128)bins[t] << (7 * (s + 1 - t));
        double hi = (double)tot;
        double lo = (double)(tot - (__int128)hi); /* |.| <= ulp(hi): exact */
        double h2, l2;
        two_sum(hi, lo, &h2, &l2);
        const int sc = EA[i] + EX[j] - 12 - 7 * (s - 1);
        Whi[i * ldw + j] = ldexp(h2, sc);
        Wlo[i * ldw + j] = ldexp(l2, sc);
      }
    free(bins);
  }
  free(DA); free(DX); free(EA); free(EX);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Modular form of the split product (the accelerator direction of          */
/* Sec. 3.1.3 by the integer route of Ozaki scheme II: Ozaki, Uchino and     */
/* Imamura 2025).                                                            */
/*                                                                           */
/* Diagonal.  The diagonal of A is kept out of the integer image and its     */
/* part of the product, a_ii x_ij, is added exactly: the off-diagonal row    */
/* maxima then set the scales, which keeps several more bits of the         */
/* off-diagonal entries where the diagonal dominates the row (as in          */
/* A = Q diag(lambda) Q^T, whose diagonal is the mean eigenvalue while the   */
/* off-diagonal entries shrink like 1/sqrt(n)).                              */
/*                                                                           */
/* Scaling to integers.  Row i of A gets the exponent E_i (the smallest       */
/* integer with max_{l != i} |a_il| < 2^E_i, 0 for a zero line) and column j */
/* of X the exponent F_j (the same over the column), and                     */
/*     A'_il = rint(a_il 2^(bA - E_i)) (l != i, A'_ii = 0),                  */
/*     X'_lj = rint(x_lj 2^(bX - F_j)),                                       */
/* integers with |A'| <= 2^bA and |X'| <= 2^bX (each is the rounding of one   */
/* double, so it is itself a double; the scaling is exact).                  */
/*                                                                           */
/* Moduli.  N pairwise coprime moduli, the largest that fit one signed byte  */
/* as balanced residues: 256, 255, 253, ... (table below); M = m_1 ... m_N,   */
/* L = the bit length of M.  The bit budget bA + bX = L - 3 - c with          */
/* c = ceil(log2 n) and bA = ceil, bX = floor of half of it gives             */
/*     |sum_l A'_il X'_lj| <= n 2^(bA + bX) <= 2^(L-3) < M/2,                 */
/* so the integer product A'X' is fixed by its residues modulo every m_t:    */
/* the method forms the N residue products (A' mod m_t)(X' mod m_t) with      */
/* INT8 operands and exact INT32 sums, and recovers A'X' by the Chinese       */
/* remainder theorem.  The recovered value is the exact integer product, so   */
/* this oracle forms that product directly (128-bit integer sums; N <= 16     */
/* keeps every sum below 2^125) and returns                                   */
/*     W_ij = 2^(E_i + F_j - bA - bX) (A'X')_ij + a_ii x_ij                   */
/* as a double-double pair: the scaled integer rounded to a pair (hi the     */
/* nearest double, lo the nearest double to the rest), a_ii x_ij as an exact */
/* pair (TwoProduct), and the two pairs added with both parts' errors kept  */
/* (relative error of the sum about 2^-105).                                 */
/* ------------------------------------------------------------------------ */
static const int32_t ORC_CRT_MODULI[16] = {256, 255, 253, 251, 247, 241, 239, 233,
                                           229, 227, 223, 217, 211, 199, 197, 193};
#define ORC_CRT_NMIN 8
#define ORC_CRT_NMAX 16

/* Bit budgets of the scaled operands for N moduli and contraction length n.
 * M is formed exactly in 32-bit limbs.  Returns ORC_EINVAL when N is out of
 * range or the budget leaves fewer than one bit per operand. */
int orc_crt_bits(int32_t nmod, int64_t n, int32_t* bA, int32_t* bX) {
  if (nmod < ORC_CRT_NMIN || nmod > ORC_CRT_NMAX || n < 1) return ORC_EINVAL;
  uint32_t limb[8] = {1, 0, 0, 0, 0, 0, 0, 0};
  for (int t = 0; t < nmod; ++t) {
    uint64_t carry = 0;
    for (int w = 0; w < 8; ++w) {
      uint64_t v = (uint64_t)limb[w] * (uint64_t)ORC_CRT_MODULI[t] + carry;
      limb[w] = (uint32_t)v;
      carry = v >> 32;
    }
  }
  int L = 0;
  for (int w = 7; w >= 0; --w)
    if (limb[w]) {
      int b = 32;
      while (!(limb[w] >> (b - 1))) --b;
      L = 32 * w + b;
      break;
    }
  int c = 0;
  while (((int64_t)1 << c) < n) ++c;
  const int B = L - 3 - c;
  if (B < 2) return ORC_EINVAL;
  *bA = (B + 1) / 2;
  *bX = B / 2;
  return ORC_OK;
}

/* Integer images of a rows x cols row-major matrix (leading dimension ld):
 * Q = rint(m 2^(b - E)) with one exponent per row (by_row) or per column. */
/* skip_diag: the entries (i, i) are left out of the maxima and imaged as 0. */
static void orc_crt_scale(int64_t rows, int64_t cols, const double* M, int64_t ld,
                          int by_row, int skip_diag, int32_t b, int64_t* Q, int32_t* Eexp) {
  const int64_t nline = by_row ? rows : cols;
  for (int64_t a = 0; a < nline; ++a) {
    double mx = 0.0;
    const int64_t len = by_row ? cols : rows;
    for (int64_t t = 0; t < len; ++t) {
      if (skip_diag && t == a) continue;
      double v = by_row ? M[a * ld + t] : M[t * ld + a];
      if (fabs(v) > mx) mx = fabs(v);
    }
    int e = 0;
    if (mx > 0.0) frexp(mx, &e);
    Eexp[a] = e;
  }
  for (int64_t i = 0; i < rows; ++i)
    for (int64_t j = 0; j < cols; ++j) {
      const int e = Eexp[by_row ? i : j];
      Q[i * cols + j] = (skip_diag && i == j) ? 0 : (int64_t)rint(ldexp(M[i * ld + j], b - e));
    }
}

/* W = A X by the modular form with N moduli (ORC_CRT_NMIN..ORC_CRT_NMAX).
 * A is n x n (row-major, lda; rows of A are scaled), X is n x k (ldx,
 * columns scaled); W and Wlo are n x k (ldw). */
int orc_gemm_crt(int64_t n, int64_t k, const double* A, int64_t lda,
                 const double* X, int64_t ldx, int32_t nmod, double* Whi,
                 double* Wlo, int64_t ldw) {
  int32_t bA = 0, bX = 0;
  if (orc_crt_bits(nmod, n, &bA, &bX) != ORC_OK) return ORC_EINVAL;
  int64_t* QA = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n * n));
  int64_t* QX = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n * k));
  int32_t* EA = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* EX = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  if (!QA || !QX || !EA || !EX) {
    free(QA); free(QX); free(EA); free(EX);
    return ORC_ENOMEM;
  }
  orc_crt_scale(n, n, A, lda, 1, 1, bA, QA, EA);
  orc_crt_scale(n, k, X, ldx, 0, 0, bX, QX, EX);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < k; ++j) {
      __int128 tot = 0;
      for (int64_t l = 0; l < n; ++l) tot += (__int128)QA[i * n + l] * (__int128)QX[l * k + j];
      double hi = (double)tot;
      double lo = (double)(tot - (__int128)hi);
      const int sc = EA[i] + EX[j] - bA - bX;
      hi = ldexp(hi, sc);
      lo = ldexp(lo, sc);
      /* + a_ii x_ij: (hi, lo) + (p, pe), both parts' errors kept */
      double p, pe, s1, e1, s2, e2;
      two_prod(A[i * lda + i], X[i * ldx + j], &p, &pe);
      two_sum(hi, p, &s1, &e1);
      two_sum(lo, pe, &s2, &e2);
      e1 += s2;
      two_sum(s1, e1, &s1, &e1);
      e1 += e2;
      two_sum(s1, e1, &Whi[i * ldw + j], &Wlo[i * ldw + j]);
    }
  free(QA); free(QX); free(EA); free(EX);
  return ORC_OK;
}

/* W = A * X for A in CSR form (row_ptr[n+1], col_idx[nnz], val[nnz]).        */
void orc_gemm_csr(int64_t n, int64_t k, const int32_t* row_ptr,
                  const int32_t* col_idx, const double* val, const double* X,
                  int64_t ldx, double* W, int64_t ldw) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double* w = W + i * ldw;
    for (int64_t j = 0; j < k; ++j) w[j] = 0.0;
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      double a = val[e];
      const double* x = X + (int64_t)col_idx[e] * ldx;
      for (int64_t j = 0; j < k; ++j) w[j] += a * x[j];
    }
  }
}

void orc_gemm_csr_dd(int64_t n, int64_t k, const int32_t* row_ptr,
                     const int32_t* col_idx, const double* val,
                     const double* X, int64_t ldx, double* Whi, double* Wlo,
                     int64_t ldw) {
#pragma omp parallel
  {
    double* p = (double*)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
    double* s = (double*)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      for (int64_t j = 0; j < k; ++j) { p[j] = 0.0; s[j] = 0.0; }
      for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        double a = val[e];
        const double* x = X + (int64_t)col_idx[e] * ldx;
        for (int64_t j = 0; j < k; ++j) {
          double h, r, q;
          two_prod(a, x[j], &h, &r);
          two_sum(p[j], h, &p[j], &q);
          s[j] += q + r;
        }
      }
      for (int64_t j = 0; j < k; ++j) {
        double hi, lo;
        two_sum(p[j], s[j], &hi, &lo);
        Whi[i * ldw + j] = hi;
        Wlo[i * ldw + j] = lo;
      }
    }
    free(p);
    free(s);
  }
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 (Yamamoto's compact WY construction):                         */
/*   Y = Q - I_{n,k},   T = -Y1^{-T},  Y1 the leading k x k block of Y.       */
/* Y1^{-T} is formed column by column from an LU factorisation of Y1^T with  */
/* partial pivoting.  cond1 receives ||Y1||_1 * ||Y1^{-1}||_1.                */
/* Y is n x k row-major (ld k), T is k x k row-major.                         */
/* ------------------------------------------------------------------------ */
int orc_compact_wy(int64_t n, int64_t k, const double* X, int64_t ldx,
                   double* Y, double* T, double* cond1) {
  if (n <= 0 || k <= 0 || k >= n) return ORC_EINVAL;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < k; ++j)
      Y[i * k + j] = X[i * ldx + j] - (i == j ? 1.0 : 0.0);

  /* LU of B = Y1^T (k x k) with row pivoting: P*B = L*U. */
  double* B = (double*)malloc(sizeof(double) * (size_t)(k * k));
  int64_t* piv = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
  if (!B || !piv) { free(B); free(piv); return ORC_ENOMEM; }
  for (int64_t i = 0; i < k; ++i)
    for (int64_t j = 0; j < k; ++j) B[i * k + j] = Y[j * k + i];
  int singular = 0;
  for (int64_t c = 0; c < k; ++c) {
    int64_t p = c;
    double best = fabs(B[c * k + c]);
    for (int64_t r = c + 1; r < k; ++r)
      if (fabs(B[r * k + c]) > best) { best = fabs(B[r * k + c]); p = r; }
    piv[c] = p;
    if (best == 0.0) { singular = 1; break; }
    if (p != c)
      for (int64_t j = 0; j < k; ++j) {
        double t = B[c * k + j]; B[c * k + j] = B[p * k + j]; B[p * k + j] = t;
      }
    for (int64_t r = c + 1; r < k; ++r) {
      double m = B[r * k + c] / B[c * k + c];
      B[r * k + c] = m;
      for (int64_t j = c + 1; j < k; ++j) B[r * k + j] -= m * B[c * k + j];
    }
  }
  if (singular) { free(B); free(piv); if (cond1) *cond1 = INFINITY; return ORC_SINGULAR; }

  /* Solve B * Z = I for Z = Y1^{-T}, one column e_c at a time. */
  double* z = (double*)malloc(sizeof(double) * (size_t)k);
  for (int64_t c = 0; c < k; ++c) {
    for (int64_t i = 0; i < k; ++i) z[i] = (i == c) ? 1.0 : 0.0;
    for (int64_t i = 0; i < k; ++i) {         /* apply the row swaps */
      int64_t p = piv[i];
      if (p != i) { double t = z[i]; z[i] = z[p]; z[p] = t; }
    }
    for (int64_t i = 0; i < k; ++i)           /* L y = Pb (unit lower) */
      for (int64_t j = 0; j < i; ++j) z[i] -= B[i * k + j] * z[j];
    for (int64_t i = k - 1; i >= 0; --i) {    /* U z = y */
      for (int64_t j = i + 1; j < k; ++j) z[i] -= B[i * k + j] * z[j];
      z[i] /= B[i * k + i];
    }
    for (int64_t i = 0; i < k; ++i) T[i * k + c] = -z[i]; /* T = -Y1^{-T} */
  }
  free(z);
  free(B);
  free(piv);

  /* ||Y1||_1 = max column sum; ||Y1^{-1}||_1 = max row sum of Y1^{-T} = -T. */
  double ny = 0.0, ninv = 0.0;
  for (int64_t j = 0; j < k; ++j) {
    double s = 0.0;
    for (int64_t i = 0; i < k; ++i) s += fabs(Y[i * k + j]);
    if (s > ny) ny = s;
  }
  for (int64_t i = 0; i < k; ++i) {
    double s = 0.0;
    for (int64_t j = 0; j < k; ++j) s += fabs(T[i * k + j]);
    if (s > ninv) ninv = s;
  }
  double c1 = ny * ninv;
  if (cond1) *cond1 = c1;
  if (!(c1 <= 1.0 / ((double)n * ORC_U))) return ORC_SINGULAR;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Application of H = I - Y T Y^T without forming it (Sec. 3.1.2, after Table 1):*/
/*   H B   = B - Y (T   (Y^T B)),                                            */
/*   H^T B = B - Y (T^T (Y^T B)).                                            */
/* B and out are n x m row-major (ld m); trans != 0 selects H^T.             */
/* ------------------------------------------------------------------------ */
void orc_apply_h(int64_t n, int64_t k, const double* Y, const double* T,
                 int trans, const double* Bm, int64_t m, double* out) {
  double* G = (double*)calloc((size_t)(k * m), sizeof(double));  /* Y^T B */
  double* H = (double*)calloc((size_t)(k * m), sizeof(double));  /* T(^T) G */
  for (int64_t a = 0; a < k; ++a)
    for (int64_t c = 0; c < m; ++c) {
      double s = 0.0;
      for (int64_t i = 0; i < n; ++i) s += Y[i * k + a] * Bm[i * m + c];
      G[a * m + c] = s;
    }
  for (int64_t a = 0; a < k; ++a)
    for (int64_t c = 0; c < m; ++c) {
      double s = 0.0;
      for (int64_t b = 0; b < k; ++b)
        s += (trans ? T[b * k + a] : T[a * k + b]) * G[b * m + c];
      H[a * m + c] = s;
    }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    for (int64_t c = 0; c < m; ++c) {
      double s = 0.0;
      for (int64_t a = 0; a < k; ++a) s += Y[i * k + a] * H[a * m + c];
      out[i * m + c] = Bm[i * m + c] - s;
    }
  free(G);
  free(H);
}

/* ------------------------------------------------------------------------ */
/* One step of Algorithm 4.                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t n;
  int32_t kind;          /* 0 dense, 1 CSR */
  const double* a;       /* dense, row-major */
  int64_t lda;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const double* val;
} orc_matrix;

typedef struct {
  double mu;             /* spectral shift: the method runs on A - mu*I */
  double delta_c;        /* delta = delta_c * norm_a * u (the paper uses 10) */
  double norm_a;         /* ||A|| used in delta and in the residual statistic */
  int32_t beta_zero;     /* 1: beta_ij = 0 (after Rayleigh-Ritz preprocessing) */
  int32_t normalize;     /* 1: normalise the columns of the update */
  int32_t dd;            /* 1: W = A*X as a double-double pair, R from it */
  int32_t shift_in_denominators; /* 1: derived form, mu only in d_j - mu */
  int32_t plant_printed_sign;    /* 1: use the sign printed in eq. (V-def) */
  int32_t split_slices;  /* > 0: W by the split form with that many slices
                            (dense only), kept as a pair like dd */
  int32_t rr_zero_top;   /* 1: X is a Rayleigh-Ritz basis (Sec. 3.4, clustered
                            eigenvalues): the leading k x k block of E_L is
                            zero, so no d_j - d_i denominator is formed */
  int32_t square;        /* 1: the method runs on B = A^2 - mu I (Sec. 5.2, the
                            smallest |lambda|): line 1 forms A (A X), so A^2 is
                            never formed (plain FP64 only) */
  int32_t crt_moduli;    /* > 0: W by the modular form with that many moduli
                            (dense only), kept as a pair like dd */
} orc_opts;

typedef struct {
  double corr_fro;       /* ||E_L||_F */
  double resid_rel;      /* ||A X - X D||_F / norm_a */
  double cond_y1;        /* ||Y1||_1 ||Y1^{-1}||_1 */
} orc_stats;

int orc_refine_step(const orc_matrix* M, int64_t k, const double* X,
                    int64_t ldx, double* Xout, int64_t ldo, const orc_opts* o,
                    orc_stats* st, double* d_out, double* E_out) {
  const int64_t n = M->n;
  if (n <= 0 || k <= 0 || k >= n) return ORC_EINVAL;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < k; ++j)
      if (!isfinite(X[i * ldx + j])) return ORC_NONFINITE;

  size_t nk = (size_t)(n * k), kk = (size_t)(k * k);
  double* W = (double*)malloc(sizeof(double) * nk);
  double* Wlo = (double*)malloc(sizeof(double) * nk);
  double* Y = (double*)malloc(sizeof(double) * nk);
  double* T = (double*)malloc(sizeof(double) * kk);
  double* R = (double*)malloc(sizeof(double) * nk);
  double* V = (double*)malloc(sizeof(double) * nk);
  double* E = (double*)malloc(sizeof(double) * nk);
  double* HE = (double*)malloc(sizeof(double) * nk);
  double* alpha = (double*)malloc(sizeof(double) * (size_t)k);
  double* d = (double*)malloc(sizeof(double) * (size_t)k);
  int rc = ORC_OK;
  if (!W || !Wlo || !Y || !T || !R || !V || !E || !HE || !alpha || !d) {
    rc = ORC_ENOMEM;
    goto done;
  }

  /* Product: W = A X  (double-double pair when o->dd, split or modular). */
  const int pair = o->dd || o->split_slices > 0 || o->crt_moduli > 0;
  if (o->crt_moduli > 0) {
    if (M->kind != 0 || o->split_slices > 0) { rc = ORC_EINVAL; goto done; }
    rc = orc_gemm_crt(n, k, M->a, M->lda, X, ldx, o->crt_moduli, W, Wlo, k);
    if (rc != ORC_OK) goto done;
  } else if (o->split_slices > 0) {
    if (M->kind != 0) { rc = ORC_EINVAL; goto done; }
    rc = orc_gemm_split(n, k, M->a, M->lda, X, ldx, o->split_slices, W, Wlo, k);
    if (rc != ORC_OK) goto done;
  } else if (M->kind == 0) {
    if (o->dd) orc_gemm_dense_dd(n, k, M->a, M->lda, X, ldx, W, Wlo, k);
    else orc_gemm_dense(n, k, M->a, M->lda, X, ldx, W, k);
  } else {
    if (o->dd) orc_gemm_csr_dd(n, k, M->row_ptr, M->col_idx, M->val, X, ldx, W, Wlo, k);
    else orc_gemm_csr(n, k, M->row_ptr, M->col_idx, M->val, X, ldx, W, k);
  }
  if (!pair) memset(Wlo, 0, sizeof(double) * nk);

  /* Squared variant: W <- A W, so that W = A^2 X; the shift below then gives
   * W_B = A^2 X - mu X. */
  if (o->square) {
    if (pair) { rc = ORC_EINVAL; goto done; }
    double* W2 = (double*)malloc(sizeof(double) * nk);
    if (!W2) { rc = ORC_ENOMEM; goto done; }
    if (M->kind == 0) orc_gemm_dense(n, k, M->a, M->lda, W, k, W2, k);
    else orc_gemm_csr(n, k, M->row_ptr, M->col_idx, M->val, W, k, W2, k);
    memcpy(W, W2, sizeof(double) * nk);
    free(W2);
  }

  /* Shift, as the paper's variant does it: the method runs on B = A - mu I,
   * so W_B = W - mu X.  The derived form keeps W and puts mu only into the
   * bottom-block denominators. */
  const int literal_shift = (o->mu != 0.0) && !o->shift_in_denominators;
  if (literal_shift) {
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < k; ++j) {
        if (pair) {
          /* (W_hi + W_lo) - mu x, kept as a pair */
          double p, pe, s, se;
          two_prod(o->mu, X[i * ldx + j], &p, &pe);
          two_sum(W[i * k + j], -p, &s, &se);
          se += Wlo[i * k + j] - pe;
          two_sum(s, se, &W[i * k + j], &Wlo[i * k + j]);
        } else {
          W[i * k + j] = W[i * k + j] - o->mu * X[i * ldx + j];
        }
      }
  }

  /* Compact WY factors of X (Algorithm 1). */
  double cond1 = 0.0;
  rc = orc_compact_wy(n, k, X, ldx, Y, T, &cond1);
  if (st) st->cond_y1 = cond1;
  if (rc != ORC_OK) goto done;

  /* Rayleigh quotients: alpha_j = x_j^T x_j, d_j = x_j^T w_j / alpha_j (eq. Rayleigh). */
  for (int64_t j = 0; j < k; ++j) {
    double sa = 0.0, sd = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double x = X[i * ldx + j];
      sa += x * x;
      sd += x * W[i * k + j];
    }
    alpha[j] = sa;
    d[j] = sd / sa;
  }

  /* Line 5, first half: R = W - X D.  With a double-double W the product
   * x*d is formed exactly and the low parts are added after the leading
   * cancellation. */
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < k; ++j) {
      double x = X[i * ldx + j];
      if (pair) {
        double p, pe;
        two_prod(x, d[j], &p, &pe);
        R[i * k + j] = (W[i * k + j] - p) + (Wlo[i * k + j] - pe);
      } else {
        R[i * k + j] = W[i * k + j] - x * d[j];
      }
    }

  /* Line 5, second half: V = H^T R through the WY factors. */
  orc_apply_h(n, k, Y, T, 1, R, k, V);

  /* Correction step: the correction matrix E_L (n x k). */
  {
    const double delta = o->delta_c * o->norm_a * ORC_U;
    for (int64_t i = 0; i < k; ++i)
      for (int64_t j = 0; j < k; ++j) {
        double e;
        if (o->rr_zero_top) {
          e = 0.0;                                            /* Sec. 3.4 (clusters) */
        } else if (i == j) {
          e = (1.0 - alpha[i]) / 2.0;                         /* eq. Ediag */
        } else if (fabs(d[j] - d[i]) <= delta) {
          if (o->beta_zero) {
            e = 0.0;
          } else {                                            /* beta_ij */
            double g = 0.0;
            for (int64_t l = 0; l < n; ++l) g += X[l * ldx + i] * X[l * ldx + j];
            e = -g / 2.0;
          }
        } else {
          e = V[i * k + j] / (d[j] - d[i]);                   /* eq. Eoffdiag */
          if (o->plant_printed_sign) e = -e;
        }
        E[i * k + j] = e;
      }
    for (int64_t i = k; i < n; ++i)
      for (int64_t j = 0; j < k; ++j) {
        /* literal shift: d already is the Rayleigh quotient of B = A - mu I */
        double den = literal_shift ? d[j] : (d[j] - o->mu);
        E[i * k + j] = V[i * k + j] / den;
      }
  }

  /* Update step: X~ = X + H E_L. */
  orc_apply_h(n, k, Y, T, 0, E, k, HE);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < k; ++j)
      Xout[i * ldo + j] = X[i * ldx + j] + HE[i * k + j];

  /* Column normalisation after the update. */
  if (o->normalize) {
    for (int64_t j = 0; j < k; ++j) {
      double s = 0.0;
      for (int64_t i = 0; i < n; ++i) s += Xout[i * ldo + j] * Xout[i * ldo + j];
      double nr = sqrt(s);
      for (int64_t i = 0; i < n; ++i) Xout[i * ldo + j] /= nr;
    }
  }

  /* Statistics of the input X: ||E_L||_F and ||R||_F / ||A||. */
  if (st) {
    double se = 0.0, sr = 0.0;
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < k; ++j) {
        se += E[i * k + j] * E[i * k + j];
        sr += R[i * k + j] * R[i * k + j];
      }
    st->corr_fro = sqrt(se);
    st->resid_rel = sqrt(sr) / o->norm_a;
  }
  if (d_out)
    for (int64_t j = 0; j < k; ++j) d_out[j] = literal_shift ? d[j] + o->mu : d[j];
  if (E_out) memcpy(E_out, E, sizeof(double) * nk);

done:
  free(W); free(Wlo); free(Y); free(T); free(R); free(V); free(E); free(HE);
  free(alpha); free(d);
  return rc;
}

/* ||A||_inf = max_i sum_j |a_ij| for dense and CSR storage. */
double orc_norm_inf_dense(int64_t n, const double* A, int64_t lda) {
  double best = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) s += fabs(A[i * lda + j]);
    if (s > best) best = s;
  }
  return best;
}
double orc_norm_inf_csr(int64_t n, const int32_t* row_ptr, const double* val) {
  double best = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) s += fabs(val[e]);
    if (s > best) best = s;
  }
  return best;
}
