"""CPU oracle for one refinement step (Algorithm 4 with Algorithm 1) of
Terao, Ozaki, Imamura and Ogita, arXiv 2602.23778.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
never links, imports or calls it, and it shares no code with that library.

The arithmetic lives in ``oracle.c`` (plain C loops, IEEE double, fixed
ascending summation order); this module only marshals numpy arrays into it.
Every function states the passage of the paper it follows.  Functions that
are not pinned by an independent check say "parity unpinned" here; at present
every exported function is pinned by ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK = 0
EINVAL = -1
SINGULAR = -4
NONFINITE = -6


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-std=c11", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class _Matrix(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("kind", ctypes.c_int32),
                ("a", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("val", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("delta_c", ctypes.c_double),
                ("norm_a", ctypes.c_double), ("beta_zero", ctypes.c_int32),
                ("normalize", ctypes.c_int32), ("dd", ctypes.c_int32),
                ("shift_in_denominators", ctypes.c_int32),
                ("plant_printed_sign", ctypes.c_int32),
                ("split_slices", ctypes.c_int32), ("rr_zero_top", ctypes.c_int32),
                ("square", ctypes.c_int32), ("crt_moduli", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("corr_fro", ctypes.c_double), ("resid_rel", ctypes.c_double),
                ("cond_y1", ctypes.c_double)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i64, vp, dbl = ctypes.c_int64, ctypes.c_void_p, ctypes.c_double
        lib.orc_gemm_dense.argtypes = [i64, i64, vp, i64, vp, i64, vp, i64]
        lib.orc_gemm_dense_dd.argtypes = [i64, i64, vp, i64, vp, i64, vp, vp, i64]
        lib.orc_gemm_csr.argtypes = [i64, i64, vp, vp, vp, vp, i64, vp, i64]
        lib.orc_gemm_csr_dd.argtypes = [i64, i64, vp, vp, vp, vp, i64, vp, vp, i64]
        lib.orc_compact_wy.argtypes = [i64, i64, vp, i64, vp, vp, vp]
        lib.orc_compact_wy.restype = ctypes.c_int
        lib.orc_apply_h.argtypes = [i64, i64, vp, vp, ctypes.c_int, vp, i64, vp]
        lib.orc_refine_step.argtypes = [ctypes.POINTER(_Matrix), i64, vp, i64, vp, i64,
                                        ctypes.POINTER(_Opts), ctypes.POINTER(_Stats), vp, vp]
        lib.orc_refine_step.restype = ctypes.c_int
        lib.orc_split_digits.argtypes = [i64, i64, vp, i64, ctypes.c_int32, ctypes.c_int32,
                                         vp, vp]
        lib.orc_gemm_split.argtypes = [i64, i64, vp, i64, vp, i64, ctypes.c_int32, vp, vp, i64]
        lib.orc_gemm_split.restype = ctypes.c_int
        lib.orc_crt_bits.argtypes = [ctypes.c_int32, i64, vp, vp]
        lib.orc_crt_bits.restype = ctypes.c_int
        lib.orc_gemm_crt.argtypes = [i64, i64, vp, i64, vp, i64, ctypes.c_int32, vp, vp, i64]
        lib.orc_gemm_crt.restype = ctypes.c_int
        lib.orc_norm_inf_dense.argtypes = [i64, vp, i64]
        lib.orc_norm_inf_dense.restype = dbl
        lib.orc_norm_inf_csr.argtypes = [i64, vp, vp]
        lib.orc_norm_inf_csr.restype = dbl
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Csr:
    """Symmetric matrix in CSR form (int32 indices, float64 values)."""
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray

    def __post_init__(self):
        self.row_ptr = np.ascontiguousarray(self.row_ptr, dtype=np.int32)
        self.col_idx = np.ascontiguousarray(self.col_idx, dtype=np.int32)
        self.val = np.ascontiguousarray(self.val, dtype=np.float64)


def matmul(A, X, dd: bool = False):
    """The product step of Algorithm 4, W = A X (dense ndarray or Csr).  With dd=True
    returns (W_hi, W_lo) from the compensated dot product Dot2."""
    lib = _load()
    X = _f64(X)
    n, k = X.shape
    W = np.empty((n, k))
    Wlo = np.empty((n, k))
    if isinstance(A, Csr):
        if dd:
            lib.orc_gemm_csr_dd(n, k, _p(A.row_ptr), _p(A.col_idx), _p(A.val), _p(X), k,
                                _p(W), _p(Wlo), k)
        else:
            lib.orc_gemm_csr(n, k, _p(A.row_ptr), _p(A.col_idx), _p(A.val), _p(X), k, _p(W), k)
    else:
        A = _f64(A)
        if dd:
            lib.orc_gemm_dense_dd(n, k, _p(A), A.shape[1], _p(X), k, _p(W), _p(Wlo), k)
        else:
            lib.orc_gemm_dense(n, k, _p(A), A.shape[1], _p(X), k, _p(W), k)
    return (W, Wlo) if dd else W


def split_digits(M, s: int, by_row: bool):
    """Slicing of the split form (Sec. 3.1.3; Ozaki et al. 2012): returns
    (D, E) with D of shape (s, rows, cols), int8 digits in [-64, 64], and E
    the per-row (by_row) or per-column power-of-two exponents, such that
    M = 2^(E-6) sum_p D_p 2^(-7(p-1)) + r with |r| <= 2^(E-7s)."""
    lib = _load()
    M = _f64(M)
    rows, cols = M.shape
    D = np.empty((s, rows, cols), dtype=np.int8)
    E = np.empty(rows if by_row else cols, dtype=np.int32)
    lib.orc_split_digits(rows, cols, _p(M), cols, int(by_row), s, _p(D), _p(E))
    return D, E


def matmul_split(A, X, s: int):
    """The product step of Algorithm 4 by the split form with s slices per operand: the
    products of digit matrices with p + q <= s + 1, combined exactly; returns
    (W_hi, W_lo) with W_hi + W_lo equal to that sum.  A need not be
    symmetric (rows of A are scaled, columns of X)."""
    lib = _load()
    A, X = _f64(A), _f64(X)
    n, k = X.shape
    W = np.empty((n, k))
    Wlo = np.empty((n, k))
    rc = lib.orc_gemm_split(n, k, _p(A), A.shape[1], _p(X), k, s, _p(W), _p(Wlo), k)
    if rc != OK:
        raise ValueError("orc_gemm_split: status %d" % rc)
    return W, Wlo


CRT_MODULI_MIN = 8
CRT_MODULI_MAX = 16


def crt_bits(nmod: int, n: int):
    """Bit budgets (bA, bX) of the modular form (Sec. 3.1.3's accelerator
    direction; Ozaki scheme II): with L the bit length of the product M of the
    first nmod moduli 256, 255, 253, ..., bA + bX = L - 3 - ceil(log2 n),
    bA = ceil and bX = floor of half of it, so that n 2^(bA+bX) < M/2."""
    lib = _load()
    a = ctypes.c_int32(0)
    b = ctypes.c_int32(0)
    rc = lib.orc_crt_bits(int(nmod), int(n), ctypes.byref(a), ctypes.byref(b))
    if rc != OK:
        raise ValueError("orc_crt_bits: status %d" % rc)
    return a.value, b.value


def matmul_crt(A, X, nmod: int):
    """The product step of Algorithm 4 by the modular form with nmod moduli:
    A' = rint(A_il 2^(bA - E_i)) off the diagonal (A'_ii = 0; E_i from the
    off-diagonal row maxima), X' = rint(X_lj 2^(bX - F_j)) (column exponents
    F), W = 2^(E_i + F_j - bA - bX) (A'X')_ij + a_ii x_ij with the integer
    product exact (what the Chinese remainder theorem recovers from the
    residue products) and the diagonal's part added exactly; returns
    (W_hi, W_lo).  A need not be symmetric (it must be square)."""
    lib = _load()
    A, X = _f64(A), _f64(X)
    n, k = X.shape
    W = np.empty((n, k))
    Wlo = np.empty((n, k))
    rc = lib.orc_gemm_crt(n, k, _p(A), A.shape[1], _p(X), k, int(nmod), _p(W), _p(Wlo), k)
    if rc != OK:
        raise ValueError("orc_gemm_crt: status %d" % rc)
    return W, Wlo


def compact_wy(X):
    """Algorithm 1: Y = X - I_{n,k}, T = -Y1^{-T}.  Returns (status, Y, T, cond1)."""
    lib = _load()
    X = _f64(X)
    n, k = X.shape
    Y = np.empty((n, k))
    T = np.empty((k, k))
    c = ctypes.c_double(0.0)
    rc = lib.orc_compact_wy(n, k, _p(X), k, _p(Y), _p(T), ctypes.byref(c))
    return rc, Y, T, c.value


def modified_lu(Q):
    """Algorithm 2 (Ballard's modified LU): for each column j the sign
    sigma_j = -sign(q_jj) of the current diagonal entry is subtracted from it
    before the elimination, so the pivot is at least 1 in magnitude for
    orthonormal columns.  Returns (Y, U, sigma) with Q - Sigma = Y U, Y n x k
    unit lower trapezoidal and U k x k upper triangular (sign(0) = +1)."""
    Qw = np.array(_f64(Q), dtype=np.float64, copy=True)
    n, k = Qw.shape
    sigma = np.zeros(k)
    for j in range(k):
        sigma[j] = -1.0 if Qw[j, j] >= 0.0 else 1.0
        Qw[j, j] -= sigma[j]
        Qw[j + 1:, j] /= Qw[j, j]
        Qw[j + 1:, j + 1:] -= np.outer(Qw[j + 1:, j], Qw[j, j + 1:])
    U = np.triu(Qw[:k, :])
    Y = np.tril(Qw, -1)
    Y[np.arange(k), np.arange(k)] = 1.0
    return Y, U, sigma


def compact_wy_lu(Q):
    """Algorithm 3: [Y, U, Sigma] = modified_LU(Q), T = -U Sigma Y1^{-T};
    for orthonormal Q, H = I - Y T Y^T is orthogonal and its first k columns
    are Q Sigma (the stated identity holds up to these column signs, since
    I_{n,k} + Y U Sigma = I_{n,k} + (Q - Sigma) Sigma).  Returns (Y, T, sigma)."""
    Y, U, sigma = modified_lu(Q)
    k = U.shape[0]
    T = -(U * sigma) @ np.linalg.inv(Y[:k].T)
    return Y, T, sigma


def sign_flip(X):
    """The one-time transformation X <- X Sigma of Sec. 3.1.1 (Sigma from the
    modified LU), after which Algorithm 1 applies.  Returns (X Sigma, sigma)."""
    _, _, sigma = modified_lu(X)
    return _f64(X) * sigma, sigma


def apply_h(Y, T, B, trans: bool = False):
    """H B or H^T B with H = I - Y T Y^T, without forming H (after Table 1)."""
    lib = _load()
    Y, T, B = _f64(Y), _f64(T), _f64(B)
    n, k = Y.shape
    m = B.shape[1]
    out = np.empty((n, m))
    lib.orc_apply_h(n, k, _p(Y), _p(T), 1 if trans else 0, _p(B), m, _p(out))
    return out


def norm_inf(A) -> float:
    lib = _load()
    if isinstance(A, Csr):
        return lib.orc_norm_inf_csr(A.n, _p(A.row_ptr), _p(A.val))
    A = _f64(A)
    return lib.orc_norm_inf_dense(A.shape[0], _p(A), A.shape[1])


@dataclass
class StepResult:
    status: int
    X: np.ndarray
    corr_fro: float
    resid_rel: float
    cond_y1: float
    d: np.ndarray
    E: np.ndarray


def refine_step(A, X, *, mu: float = 0.0, norm_a: float | None = None,
                delta_c: float = 10.0, beta_zero: bool = False,
                normalize: bool = True, dd: bool = False,
                shift_in_denominators: bool = False,
                plant_printed_sign: bool = False, split: int = 0,
                rr_top: bool = False, square: bool = False, crt: int = 0) -> StepResult:
    """One step of Algorithm 4 (with Algorithm 1) on A (dense or Csr).

    mu: the method runs on A - mu I (Sec. 5.1); norm_a: ||A|| in delta and in
    the residual statistic (default ||A||_inf); dd: line 1 in double-double;
    split: line 1 by the split form with that many slices (dense A), its
    pair (W_hi, W_lo) then used like the double-double one; crt: line 1 by
    the modular form with that many moduli (dense A), used the same way.
    rr_top: X is a Rayleigh-Ritz basis (the output of rayleigh_ritz); the
    leading k x k block of E_L is then zero (Sec. 3.4, clustered eigenvalues).
    square: the method runs on B = A^2 - mu I (Sec. 5.2, eigenvectors of the
    smallest |lambda|), line 1 as A (A X); norm_a then stands for ||B||.
    plant_printed_sign exists only so that a test can show that the sign
    printed in eq. (V-def) makes the iteration diverge."""
    lib = _load()
    X = _f64(X)
    n, k = X.shape
    if norm_a is None:
        norm_a = norm_inf(A)
    m = _Matrix()
    m.n = n
    keep = []
    if isinstance(A, Csr):
        m.kind = 1
        m.row_ptr, m.col_idx, m.val = _p(A.row_ptr), _p(A.col_idx), _p(A.val)
        m.a, m.lda = None, 0
    else:
        A = _f64(A)
        keep.append(A)
        m.kind = 0
        m.a, m.lda = _p(A), A.shape[1]
    o = _Opts(mu, delta_c, norm_a, int(beta_zero), int(normalize), int(dd),
              int(shift_in_denominators), int(plant_printed_sign), int(split), int(rr_top),
              int(square), int(crt))
    st = _Stats()
    Xout = np.zeros((n, k))
    d = np.zeros(k)
    E = np.zeros((n, k))
    rc = lib.orc_refine_step(ctypes.byref(m), k, _p(X), k, _p(Xout), k, ctypes.byref(o),
                             ctypes.byref(st), _p(d), _p(E))
    return StepResult(rc, Xout, st.corr_fro, st.resid_rel, st.cond_y1, d, E)


def rayleigh_ritz(A, X, mu: float = 0.0, square: bool = False):
    """Rayleigh-Ritz preprocessing on span(X) (Sec. 3.4, clustered eigenvalues):
    the symmetric-definite k x k problem (X^T A X) S = (X^T X) S Theta is
    solved by a library eigensolver (the step's one library primitive; A X is
    the oracle's own product), and Z = X S has Z^T Z = I and Z^T A Z = Theta.

    Conventions shared with the GPU path (the paper fixes neither): the
    columns are ordered by |theta - mu| descending (the refinement's targets
    first, ties in ascending theta), and each column's sign makes z_jj <= 0,
    so that the leading block Z1 - I of the compact-WY factor keeps its
    diagonal at or below -1.  square: the pencil of B = A^2 - mu I (Sec. 5.2),
    with A X replaced by A (A X); theta are then eigenvalues of A^2.
    Returns (Z, theta)."""
    import scipy.linalg
    X = _f64(X)
    n, k = X.shape
    W = matmul(A, X)
    if square:
        W = matmul(A, W)
    H = X.T @ W
    H = 0.5 * (H + H.T)
    G = X.T @ X
    theta, S = scipy.linalg.eigh(H, G)
    order = np.lexsort((theta, -np.abs(theta - mu)))
    theta, S = theta[order], S[:, order]
    Z = X @ S
    for j in range(k):
        if Z[j, j] > 0.0:
            Z[:, j] = -Z[:, j]
    return Z, theta


def refine(A, X, steps: int, **kw):
    """Repeated steps (the paper's outer loop); returns (X, [StepResult])."""
    hist = []
    for _ in range(steps):
        r = refine_step(A, X, **kw)
        hist.append(r)
        if r.status != OK:
            break
        X = r.X
    return X, hist
