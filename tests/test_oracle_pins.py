"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names the passage of the paper (or the mathematical fact) it checks.
They are chosen so that a plausible slip in the oracle -- a dropped term, a
wrong sign or index, T instead of T^T, a missing shift -- fails at least one.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from tests._util import align_signs, max_abs_diff_aligned

U = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _sym_problem(n, lam, seed):
    Q = synth.householder_q(n, n, seed).numpy()
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    return A, Q


def _orthonormal(n, k, seed):
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.standard_normal((n, k)))
    return q * np.sign(np.diag(r))


# --------------------------------------------------------------------------
# Algorithm 1 (compact WY)
# --------------------------------------------------------------------------
def test_wy_maps_first_columns_to_x_for_any_x():
    """Alg. 1 ensures (I - Y T Y^T) I_{n,k} = Q.  The identity holds for any X
    with a nonsingular Y1, orthonormal or not: H I_{n,k} = I_{n,k} + Y."""
    rng = np.random.default_rng(1)
    for n, k in ((9, 1), (30, 4), (64, 13)):
        X = 0.3 * rng.standard_normal((n, k))
        rc, Y, T, _ = oracle.compact_wy(X)
        assert rc == oracle.OK
        Ink = np.eye(n)[:, :k]
        HX = oracle.apply_h(Y, T, Ink)
        assert np.max(np.abs(HX - X)) < 1e-14
        # Y itself is X - I_{n,k}
        assert np.max(np.abs(Y - (X - Ink))) == 0.0


def test_wy_is_orthogonal_for_orthonormal_x():
    """Alg. 1 ensures I - Y T Y^T is orthogonal when Q has orthonormal columns."""
    n, k = 50, 7
    X = _orthonormal(n, k, 2)
    rc, Y, T, _ = oracle.compact_wy(X)
    assert rc == oracle.OK
    H = oracle.apply_h(Y, T, np.eye(n))
    assert np.max(np.abs(H.T @ H - np.eye(n))) < 1e-14
    HT = oracle.apply_h(Y, T, np.eye(n), trans=True)
    assert np.max(np.abs(HT - H.T)) < 1e-15
    # H^T maps X onto I_{n,k} (eq. HX-and-HAX, first half)
    assert np.max(np.abs(H.T @ X - np.eye(n)[:, :k])) < 1e-14


def test_wy_singular_leading_block_is_reported():
    """Sec. 3.1.1: Alg. 1 needs a nonsingular Y1; X = I_{n,k} gives Y1 = 0."""
    n, k = 12, 3
    rc, *_ = oracle.compact_wy(np.eye(n)[:, :k])
    assert rc == oracle.SINGULAR
    # nearly singular: first row of Y1 is (-2^-51, 0, 0), cond1(Y1) ~ 2^51 > 1/(n u)
    X = _orthonormal(n, k, 3) * 1e-3
    X[0, :] = 0.0
    X[0, 0] = 1.0 - 2.0 ** -51
    rc, *_ = oracle.compact_wy(X)
    assert rc == oracle.SINGULAR


# --------------------------------------------------------------------------
# The product step: W = A X, plain and double-double
# --------------------------------------------------------------------------
def _exact_product(A, X):
    n, k = X.shape
    Af = [[Fraction(float(v)) for v in row] for row in A]
    Xf = [[Fraction(float(v)) for v in row] for row in X]
    return [[sum(Af[i][l] * Xf[l][j] for l in range(n)) for j in range(k)] for i in range(n)]


def test_matmul_error_bounds_against_exact_rationals():
    """The plain product meets the textbook bound |W - AX| <= n u |A||X|; the
    Dot2 pair meets u|AX| + (n u)^2 |A||X| (Ogita, Rump and Oishi 2005)."""
    rng = np.random.default_rng(4)
    n, k = 23, 3
    A = rng.standard_normal((n, n))
    A = A + A.T
    # strong cancellation: make the last column nearly orthogonal to the rows
    X = rng.standard_normal((n, k))
    W = oracle.matmul(A, X)
    Whi, Wlo = oracle.matmul(A, X, dd=True)
    ex = _exact_product(A, X)
    absAX = np.abs(A) @ np.abs(X)
    for i in range(n):
        for j in range(k):
            e = ex[i][j]
            assert abs(Fraction(W[i, j]) - e) <= Fraction(n * U * absAX[i, j])
            err_dd = abs(Fraction(Whi[i, j]) + Fraction(Wlo[i, j]) - e)
            bound = Fraction(U) * abs(e) * Fraction(1, 2 ** 50) + Fraction((n * U) ** 2 * absAX[i, j])
            assert err_dd <= bound
            # the high part is the nearest double (or next to it)
            assert abs(Fraction(Whi[i, j]) - e) <= Fraction(U) * abs(e) * 2 + Fraction((n * U) ** 2 * absAX[i, j])


def test_csr_matmul_matches_dense_library_product():
    P = synth.laplacian3d(5, seed=11)
    n = P.n
    D = np.zeros((n, n))
    for i in range(n):
        for e in range(P.row_ptr[i], P.row_ptr[i + 1]):
            D[i, P.col_idx[e]] = P.val[e]
    assert np.array_equal(D, D.T)
    X = np.random.default_rng(5).standard_normal((n, 6))
    C = oracle.Csr(n, P.row_ptr, P.col_idx, P.val)
    W = oracle.matmul(C, X)
    assert np.max(np.abs(W - D @ X)) < 1e-13
    Whi, Wlo = oracle.matmul(C, X, dd=True)
    assert np.max(np.abs(Whi - D @ X)) < 1e-13
    assert oracle.norm_inf(C) == pytest.approx(np.max(np.abs(D).sum(1)), rel=1e-15)


def _cancelling_csr(n, per_row, k, seed):
    """A CSR matrix and an X whose row products cancel: each row's last
    nonzero is chosen so that its products with column 0 of X sum to about
    the rounding error of the others (magnitudes spread over 2^-12..2^12)."""
    rng = np.random.default_rng(seed)
    rp, ci, va = [0], [], []
    X = rng.standard_normal((n, k)) * np.exp2(rng.integers(-6, 7, (n, k)))
    for i in range(n):
        cols = np.sort(rng.choice(n, per_row, replace=False))
        v = rng.standard_normal(per_row) * np.exp2(rng.integers(-12, 13, per_row))
        last = cols[-1]
        v[-1] = -float(np.dot(v[:-1], X[cols[:-1], 0])) / X[last, 0]
        ci.extend(cols.tolist())
        va.extend(v.tolist())
        rp.append(len(ci))
    return oracle.Csr(n, np.array(rp), np.array(ci), np.array(va)), X


def test_csr_dot2_pair_against_exact_rationals():
    """The CSR double-double product is Dot2 per row (Ogita, Rump and Oishi
    2005): hi + lo is the compensated sum itself, within (m u)^2 |A||X| of
    the exact value for a row of m nonzeros, on rows whose products cancel
    (where the plain sum is off by about u |A||X|, many times more)."""
    n, m, k = 30, 9, 3
    C, X = _cancelling_csr(n, m, k, 42)
    Whi, Wlo = oracle.matmul(C, X, dd=True)
    W = oracle.matmul(C, X)
    worst_plain = 0.0
    for i in range(n):
        cols = C.col_idx[C.row_ptr[i]:C.row_ptr[i + 1]]
        vals = C.val[C.row_ptr[i]:C.row_ptr[i + 1]]
        for j in range(k):
            e = sum(Fraction(float(a)) * Fraction(float(X[c, j])) for a, c in zip(vals, cols))
            absax = float(np.sum(np.abs(vals) * np.abs(X[cols, j])))
            err_dd = abs(Fraction(Whi[i, j]) + Fraction(Wlo[i, j]) - e)
            assert err_dd <= Fraction((m * U) ** 2 * absax) * Fraction(11, 10), (i, j)
            # hi is the pair's rounded sum
            assert Whi[i, j] + Wlo[i, j] == Whi[i, j]
            err_plain = abs(Fraction(W[i, j]) - e)
            assert err_plain <= Fraction(m * U * absax)
            if j == 0:
                worst_plain = max(worst_plain, float(err_plain) / absax)
    # the cancelling column really exercises the compensation
    assert worst_plain > 1e3 * (m * U) ** 2


# --------------------------------------------------------------------------
# The steps of Algorithm 4 after the product
# --------------------------------------------------------------------------
def test_top_block_of_v_is_xt_r():
    """From eqs. (HhatX-block)-(HhatAX-block): the leading k rows of
    H^T (W - X D) equal X^T (W - X D) for H built by Alg. 1 from X."""
    n, k = 40, 6
    A, Q = _sym_problem(n, np.linspace(0.1, 1.0, n), 6)
    X = synth.fp32_round(Q[:, -k:]) + 1e-4 * np.random.default_rng(6).standard_normal((n, k))
    rc, Y, T, _ = oracle.compact_wy(X)
    W = A @ X
    d = np.sum(X * W, 0) / np.sum(X * X, 0)
    R = W - X * d
    V = oracle.apply_h(Y, T, R, trans=True)
    assert np.max(np.abs(V[:k] - X.T @ R)) < 1e-17


def test_correction_structure_and_update():
    """Correction step of Alg. 4: e_jj = (1 - x_j^T x_j)/2; for i != j in the top block
    e_ij + e_ji = -x_i^T x_j (the two branches v_ij/(d_j - d_i) and
    v_ji/(d_i - d_j) combine to that); update step: X~ - X = H E_L."""
    n, k = 48, 7
    A, Q = _sym_problem(n, np.linspace(0.05, 1.0, n), 7)
    rng = np.random.default_rng(7)
    X = Q[:, -k:] + 1e-5 * rng.standard_normal((n, k))
    r = oracle.refine_step(A, X, norm_a=1.0, normalize=False)
    assert r.status == 0
    E = r.E
    G = X.T @ X
    assert np.max(np.abs(np.diag(E[:k]) - (1 - np.diag(G)) / 2)) < 1e-16
    S = E[:k] + E[:k].T
    off = ~np.eye(k, dtype=bool)
    # rounding of v_ij is about u ||A||, divided by the gap d_j - d_i
    gaps = np.abs(r.d[:, None] - r.d[None, :])[off]
    tol = 64 * U / np.min(gaps)
    assert np.max(np.abs(S[off] + G[off])) < tol
    assert np.max(np.abs(G[off])) > 1e4 * tol   # the identity is not vacuous
    # bottom block: e_ij = v_ij / d_j with V = H^T R
    rc, Y, T, _ = oracle.compact_wy(X)
    W = A @ X
    d = np.sum(X * W, 0) / np.sum(X * X, 0)
    V = oracle.apply_h(Y, T, W - X * d, trans=True)
    assert np.max(np.abs(E[k:] - V[k:] / d)) < 64 * U / np.min(np.abs(d))
    # update: H E = X~ - X with H formed explicitly by numpy
    H = np.eye(n) - Y @ T @ Y.T
    assert np.max(np.abs((r.X - X) - H @ E)) < 1e-15
    # statistics describe the input
    assert r.corr_fro == pytest.approx(np.linalg.norm(E), rel=1e-12)
    assert r.resid_rel == pytest.approx(np.linalg.norm(W - X * d), rel=1e-6)


def test_exact_eigenvectors_are_a_fixed_point():
    """eq. (update-X): with E = 0 the correction vanishes; Q's columns are the
    eigenvectors of A up to the rounding of A."""
    n, k = 64, 8
    A, Q = _sym_problem(n, np.arange(1, n + 1) / n, 8)
    X = Q[:, -k:]
    r = oracle.refine_step(A, X, norm_a=1.0)
    assert r.status == 0
    assert r.corr_fro < 1e-13
    assert r.resid_rel < 1e-14
    assert max_abs_diff_aligned(r.X, X) < 1e-14


@pytest.mark.parametrize("mu", [0.0, 1.7])
def test_k1_is_the_power_method(mu):
    """For k = 1 the step reduces to one power iteration on A - mu I:
    x~ = (A - mu I) x / ||(A - mu I) x|| for a unit x (Ĥ is then a reflector,
    Ĥ Ĥ^T = I and v_1 = x^T r = 0)."""
    n = 37
    A, Q = _sym_problem(n, np.linspace(-1.0, 0.9, n), 9)
    rng = np.random.default_rng(9)
    x = Q[:, :1] + 0.05 * rng.standard_normal((n, 1))
    x /= np.linalg.norm(x)
    r = oracle.refine_step(A, x, mu=mu, norm_a=2.0)
    y = A @ x - mu * x
    y /= np.linalg.norm(y)
    assert max_abs_diff_aligned(r.X, y) < 1e-15
    r2 = oracle.refine_step(A, x, mu=mu, norm_a=2.0, shift_in_denominators=True)
    assert max_abs_diff_aligned(r2.X, y) < 1e-15


def test_linear_rate_matches_gamma():
    """Sec. 3.2: each target converges linearly with factor
    max_{i>k}|lam_i| / |lam_j|.  lam_i = i/64, k = 8: the slowest target
    (lam = 57/64) has gamma = 56/57."""
    n, k = 64, 8
    A, Q = _sym_problem(n, np.arange(1, n + 1) / n, 10)
    Xt = Q[:, ::-1][:, :k]
    rng = np.random.default_rng(10)
    X = Xt + 1e-4 * rng.standard_normal((n, k))
    errs = []
    for _ in range(420):
        r = oracle.refine_step(A, X, norm_a=1.0)
        X = r.X
        errs.append(np.linalg.norm(align_signs(X, Xt) - Xt, axis=0))
    errs = np.array(errs)
    rate_slowest = (errs[400, k - 1] / errs[300, k - 1]) ** (1 / 100)
    assert rate_slowest == pytest.approx(56 / 57, abs=2e-3)
    # second slowest (lam = 58/64): gamma = 56/58
    rate2 = (errs[200, k - 2] / errs[100, k - 2]) ** (1 / 100)
    assert rate2 == pytest.approx(56 / 58, abs=3e-3)


def test_printed_sign_of_v_def_diverges():
    """eq. (V-def) prints the top block as D E11 - E11 D; eqs. (R) and (S) give
    E11 D - D E11, which is what eq. (Eoffdiag) and Alg. 4 use.  Planting the
    printed sign in the oracle makes the top-block error double every step,
    while the oracle as written converges."""
    n, k = 64, 8
    A, Q = _sym_problem(n, np.arange(1, n + 1) / n, 11)
    Xt = Q[:, ::-1][:, :k]
    rng = np.random.default_rng(11)
    X0 = Xt + 1e-9 * rng.standard_normal((n, k))
    good, bad = X0.copy(), X0.copy()
    eg, eb = [], []
    for _ in range(12):
        good = oracle.refine_step(A, good, norm_a=1.0).X
        bad = oracle.refine_step(A, bad, norm_a=1.0, plant_printed_sign=True).X
        eg.append(np.abs(align_signs(good, Xt) - Xt).max())
        eb.append(np.abs(align_signs(bad, Xt) - Xt).max())
    assert eg[-1] < eg[0]
    ratio = (eb[-1] / eb[-5]) ** (1 / 4)
    assert ratio == pytest.approx(2.0, rel=0.02)


def test_shift_forms_agree():
    """Sec. 5.1: refining the smallest eigenvalues through B = A - mu I.
    The literal form (W_B = A X - mu X), the derived form (mu only in the
    bottom denominators) and the method applied to mu I - A all give the same
    update up to rounding."""
    n, k = 60, 5
    lam = np.concatenate([[0.1, 0.2, 0.3, 0.4, 0.5], np.linspace(1.5, 3.0, n - k)])
    A, Q = _sym_problem(n, lam, 12)
    mu = 3.5   # makes the k smallest the dominant ones of A - mu I (gamma = 2/3)
    Xt = Q[:, :k]
    X = synth.fp32_round(Xt)
    r1 = oracle.refine_step(A, X, mu=mu, norm_a=3.0)
    r2 = oracle.refine_step(A, X, mu=mu, norm_a=3.0, shift_in_denominators=True)
    r3 = oracle.refine_step(-A, X, mu=-mu, norm_a=3.0)
    assert np.max(np.abs(r1.X - r2.X)) < 1e-14
    assert np.max(np.abs(r1.X - r3.X)) < 1e-14
    # and it converges to the k smallest
    Xc, hist = oracle.refine(A, X, 60, mu=mu, norm_a=3.0)
    assert max_abs_diff_aligned(Xc, Xt) < 1e-12


def test_converged_against_high_precision_jacobi():
    """Known answer: the refined vectors of a small FP64 matrix agree with its
    exact eigenvectors computed by cyclic Jacobi at 40 digits to a few u
    (Sec. 4.2: the attainable accuracy is set by double-precision rounding)."""
    from tests.mp_jacobi import jacobi_eigh
    n, k = 20, 4
    lam = np.concatenate([np.linspace(0.05, 0.5, n - k), [0.8, 0.85, 0.9, 1.0]])
    A, Q = _sym_problem(n, lam, 13)
    lam_mp, V = jacobi_eigh(A.tolist(), dps=40)
    order = sorted(range(n), key=lambda i: -float(lam_mp[i]))[:k]
    Xex = np.array([[float(V[r][c]) for c in order] for r in range(n)])
    X = synth.fp32_round(Q[:, ::-1][:, :k])
    Xd, _ = oracle.refine(A, X, 80, norm_a=1.0, dd=True)
    Xf, _ = oracle.refine(A, X, 80, norm_a=1.0)
    assert max_abs_diff_aligned(Xd, Xex) < 8 * U
    assert max_abs_diff_aligned(Xf, Xex) < 40 * U
    # the Rayleigh quotients of the result equal the exact eigenvalues
    r = oracle.refine_step(A, Xd, norm_a=1.0, dd=True)
    lam_ex = np.array([float(lam_mp[i]) for i in order])
    assert np.max(np.abs(r.d - lam_ex)) < 4 * U
    # residual floor O(u)||A|| (Sec. 4.2)
    assert r.resid_rel < 20 * U


def test_clustered_pair_needs_accurate_residual():
    """Two target eigenvalues 1e-6 apart: the double-double residual lets the
    iteration reach the exact eigenvectors (Jacobi, 40 digits) far more
    closely than plain FP64, whose error is about u / gap."""
    from tests.mp_jacobi import jacobi_eigh
    n, k = 24, 4
    lam = np.concatenate([np.linspace(0.05, 0.6, n - k), [0.98, 0.98 + 1e-6, 0.99, 0.99 + 1e-6]])
    A, Q = _sym_problem(n, lam, 14)
    lam_mp, V = jacobi_eigh(A.tolist(), dps=40)
    order = sorted(range(n), key=lambda i: -float(lam_mp[i]))[:k]
    Xex = np.array([[float(V[r][c]) for c in order] for r in range(n)])
    X = synth.fp32_round(Q[:, ::-1][:, :k])     # descending lam, like Xex
    Xd, hd = oracle.refine(A, X, 120, norm_a=1.0, dd=True)
    Xf, hf = oracle.refine(A, X, 120, norm_a=1.0)
    ed = max_abs_diff_aligned(Xd, Xex)
    ef = max_abs_diff_aligned(Xf, Xex)
    assert ed < 1e-13
    assert ed < ef


def test_clustered_pair_with_a_literal_shift():
    """The double-double product with the shift applied literally, W_B =
    (W_hi + W_lo) - mu X kept as a pair (Sec. 5.1): two clusters of gap 1e-6
    at the top of the spectrum, targeted through mu = -0.55 below it, so that
    both the low part of A X (|A x| about 1) and the exact product mu x
    (|mu x| about 0.55; not a power of two, so fl(mu x) is inexact) decide
    the residual.  The pair reaches the exact eigenvectors (Jacobi, 40
    digits) as closely as it does with the shift in the denominators, and far
    more closely than plain FP64 with the literal shift."""
    from tests.mp_jacobi import jacobi_eigh
    n, k = 24, 4
    lam = np.concatenate([np.linspace(0.05, 0.6, n - k), [0.98, 0.98 + 1e-6, 0.99, 0.99 + 1e-6]])
    A, Q = _sym_problem(n, lam, 16)
    mu = -0.55
    lam_mp, V = jacobi_eigh(A.tolist(), dps=40)
    order = sorted(range(n), key=lambda i: -float(lam_mp[i]))[:k]
    Xex = np.array([[float(V[r][c]) for c in order] for r in range(n)])
    X = synth.fp32_round(Q[:, ::-1][:, :k])
    Xl, _ = oracle.refine(A, X, 60, mu=mu, norm_a=1.0, dd=True)
    Xd, _ = oracle.refine(A, X, 60, mu=mu, norm_a=1.0, dd=True, shift_in_denominators=True)
    Xf, _ = oracle.refine(A, X, 60, mu=mu, norm_a=1.0)
    el = max_abs_diff_aligned(Xl, Xex)
    ed = max_abs_diff_aligned(Xd, Xex)
    ef = max_abs_diff_aligned(Xf, Xex)
    assert el < 1e-14 and ed < 1e-14
    assert max_abs_diff_aligned(Xl, Xd) < 1e-14
    assert ef > 100 * el


def test_forced_failures():
    """Status codes: singular Y1 (Sec. 3.1.1), non-finite input, invalid sizes."""
    n, k = 16, 3
    A, Q = _sym_problem(n, np.linspace(0.1, 1, n), 15)
    r = oracle.refine_step(A, np.eye(n)[:, :k], norm_a=1.0)
    assert r.status == oracle.SINGULAR
    X = Q[:, -k:].copy()
    X[3, 1] = np.nan
    assert oracle.refine_step(A, X, norm_a=1.0).status == oracle.NONFINITE
    assert oracle.refine_step(A, Q, norm_a=1.0).status == oracle.EINVAL   # k == n


def test_beta_branch_for_exact_ties():
    """Correction step of Alg. 4: equal Rayleigh quotients take beta_ij = -x_i^T x_j/2
    (or 0 after preprocessing) instead of dividing by d_j - d_i."""
    n, k = 30, 2
    lam = np.concatenate([np.linspace(0.1, 0.5, n - 2), [1.0, 1.0]])
    A, Q = _sym_problem(n, lam, 16)
    # two vectors spanning the exact double eigenvalue: their Rayleigh
    # quotients coincide to rounding
    X = Q[:, -2:] @ np.array([[np.cos(0.3), -np.sin(0.3)], [np.sin(0.3), np.cos(0.3)]])
    X = X + 1e-12 * np.random.default_rng(16).standard_normal((n, k))
    r = oracle.refine_step(A, X, norm_a=1.0, normalize=False, delta_c=1e6)
    G = X.T @ X
    assert abs(r.d[0] - r.d[1]) < 1e6 * 10 * U      # the tie is detected
    assert r.E[0, 1] == pytest.approx(-G[0, 1] / 2, abs=1e-15)
    assert r.E[1, 0] == pytest.approx(-G[1, 0] / 2, abs=1e-15)
    r0 = oracle.refine_step(A, X, norm_a=1.0, normalize=False, delta_c=1e6, beta_zero=True)
    assert r0.E[0, 1] == 0.0 and r0.E[1, 0] == 0.0


def test_golden_k1_power_iteration_values():
    """Golden fixture: a 3x3 closed-form case (tests/golden/k1_power_3x3.json)
    whose expected vector is the normalised A x, written out by hand."""
    with open(os.path.join(GOLDEN, "k1_power_3x3.json")) as f:
        g = json.load(f)
    A = np.array(g["A"], dtype=np.float64)
    x = np.array(g["x"], dtype=np.float64)[:, None]
    r = oracle.refine_step(A, x, norm_a=g["norm_a"])
    exp = np.array(g["expected"], dtype=np.float64)[:, None]
    assert max_abs_diff_aligned(r.X, exp) < 4 * U
    assert r.d[0] == pytest.approx(g["rayleigh"], abs=4 * U)


# --------------------------------------------------------------------------
# Split form of the product step (Sec. 3.1.3; Ozaki, Ogita, Oishi and Rump 2012)
# --------------------------------------------------------------------------
def _wide_range_matrix(rows, cols, seed):
    """Entries spanning many binades within each row and column."""
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((rows, cols)) * np.exp2(rng.integers(-30, 4, (rows, cols)))
    M[rng.random((rows, cols)) < 0.05] = 0.0
    return M


@pytest.mark.parametrize("s", [1, 3, 8, 9])
def test_split_digits_reconstruct_within_bound(s):
    """Every digit lies in [-64, 64]; the digits reconstruct each entry to
    within 2^(E-7s) in exact rational arithmetic, E being the line's scale
    (the smallest power of two above the line's largest magnitude); entries
    whose last bit lies above the last digit's unit are reconstructed exactly."""
    M = _wide_range_matrix(9, 13, 40 + s)
    M[4, :] = 0.0                                   # an all-zero row
    for by_row in (True, False):
        D, E = oracle.split_digits(M, s, by_row)
        assert D.min() >= -64 and D.max() <= 64
        lines = M if by_row else M.T
        for a, line in enumerate(lines):
            mx = np.max(np.abs(line))
            e = int(E[a])
            if mx == 0.0:
                assert e == 0
            else:
                assert Fraction(2) ** (e - 1) <= Fraction(float(mx)) < Fraction(2) ** e
        for i in range(M.shape[0]):
            for j in range(M.shape[1]):
                e = int(E[i] if by_row else E[j])
                rec = sum(Fraction(int(D[p, i, j])) * Fraction(2) ** (e - 6 - 7 * p) for p in range(s))
                err = abs(Fraction(float(M[i, j])) - rec)
                assert err <= Fraction(2) ** (e - 7 * s)
                m, ex = math.frexp(float(M[i, j]))
                if M[i, j] != 0.0 and ex - 53 >= e - 6 - 7 * (s - 1):
                    assert err == 0


def _short_digit_matrix(rows, cols, digits, seed, by_row):
    """Entries m * 2^(e - 6 - 7(digits-1)) with |m| < 2^(6 + 7(digits-1)), so
    that, whatever the line scale comes out as, each entry is an exact
    multiple of the unit of digit number `digits`."""
    rng = np.random.default_rng(seed)
    bits = 6 + 7 * (digits - 1)
    m = rng.integers(-(2 ** bits) + 1, 2 ** bits, (rows, cols)).astype(np.float64)
    ex = rng.integers(-8, 8, rows if by_row else cols)
    scale = np.exp2(ex - bits)
    return m * (scale[:, None] if by_row else scale[None, :])


@pytest.mark.parametrize("s", [8, 9])
def test_split_product_is_exact_when_nothing_is_truncated(s):
    """With at most floor((s+1)/2) digits per entry every term of the digit
    expansion has p + q <= s + 1, so the split form must return the exact
    product (Python integers), to the last bit of the (hi, lo) pair.  A is not
    symmetric here, so a transposed operand or a swapped scale fails."""
    n, k = 37, 5
    half = (s + 1) // 2
    A = _short_digit_matrix(n, n, half, 71 + s, True)
    X = _short_digit_matrix(n, k, half, 72 + s, False)
    assert not np.array_equal(A, A.T)
    hi, lo = oracle.matmul_split(A, X, s)
    ex = _exact_product(A, X)
    for i in range(n):
        for j in range(k):
            assert Fraction(float(hi[i, j])) + Fraction(float(lo[i, j])) == ex[i][j]
            assert abs(lo[i, j]) <= 0.5 * np.spacing(abs(hi[i, j])) or hi[i, j] == 0.0


def test_split_product_truncation_bound_and_rate():
    """Full 53-bit operands: the split product stays within the truncation
    bound n (s + 2) 2^(E_i + F_j - 7s) of the exact product (the dropped terms
    p + q > s + 1 and the slicing remainders), and each extra slice cuts the
    error by about 2^7."""
    n, k = 29, 4
    A = _wide_range_matrix(n, n, 81)
    X = _wide_range_matrix(n, k, 82)
    ex = _exact_product(A, X)
    _, EA = oracle.split_digits(A, 1, True)
    _, EX = oracle.split_digits(X, 1, False)
    worst = {}
    for s in (4, 6, 8, 9):
        hi, lo = oracle.matmul_split(A, X, s)
        w = 0.0
        for i in range(n):
            for j in range(k):
                err = abs(Fraction(float(hi[i, j])) + Fraction(float(lo[i, j])) - ex[i][j])
                bound = Fraction(n * (s + 2)) * Fraction(2) ** (int(EA[i]) + int(EX[j]) - 7 * s)
                assert err <= bound
                w = max(w, float(err / Fraction(2) ** (int(EA[i]) + int(EX[j]))))
        worst[s] = w
    assert worst[6] < worst[4] * 2.0 ** -10
    assert worst[8] < worst[6] * 2.0 ** -10
    assert worst[9] < worst[8] * 2.0 ** -4


def test_split_step_agrees_with_double_double_step():
    """A step whose line 1 comes from the split form (9 slices, error about
    2^-60 relative to the line scales) matches the Dot2 step to about u; with
    1 slice it must not (guards against the option being ignored)."""
    P = synth.dense_well_separated(256, 8)
    r_dd = oracle.refine_step(P.A, P.X0, norm_a=P.norm_a, dd=True)
    r_s9 = oracle.refine_step(P.A, P.X0, norm_a=P.norm_a, split=9)
    r_s1 = oracle.refine_step(P.A, P.X0, norm_a=P.norm_a, split=1)
    assert r_s9.status == 0 and r_dd.status == 0
    assert np.max(np.abs(r_s9.X - r_dd.X)) < 1e-15
    assert np.max(np.abs(r_s1.X - r_dd.X)) > 1e-6


# --------------------------------------------------------------------------
# Modular form of the product step (Sec. 3.1.3's accelerator direction by the
# integer route of Ozaki scheme II)
# --------------------------------------------------------------------------
def _greedy_moduli(count):
    """The largest pairwise coprime integers <= 256, taken greedily from 256
    down: the definition of the moduli, derived here independently."""
    ms = []
    m = 256
    while len(ms) < count:
        if all(math.gcd(m, q) == 1 for q in ms):
            ms.append(m)
        m -= 1
    return ms


@pytest.mark.parametrize("n", [1, 2, 3, 40, 1000, 16384, 65536])
def test_crt_bit_budget_against_the_exact_moduli_product(n):
    """bA + bX = L - 3 - ceil(log2 n), L the bit length of M (Python big
    integers), bA the larger half: then n 2^(bA+bX) < M/2, so the exact
    integer product is the one value in [-M/2, M/2) with its residues."""
    for N in range(oracle.CRT_MODULI_MIN, oracle.CRT_MODULI_MAX + 1):
        M = math.prod(_greedy_moduli(N))
        bA, bX = oracle.crt_bits(N, n)
        c = max(0, (n - 1).bit_length())
        assert bA + bX == M.bit_length() - 3 - c
        assert bA - bX in (0, 1)
        assert n * 2 ** (bA + bX) < M // 2
    with pytest.raises(ValueError):
        oracle.crt_bits(oracle.CRT_MODULI_MIN - 1, 100)
    with pytest.raises(ValueError):
        oracle.crt_bits(oracle.CRT_MODULI_MAX + 1, 100)


def _garner_balanced(res, ms):
    """Balanced mixed-radix digits of the integer with residues `res` modulo
    `ms` (Garner), evaluated back to an integer: the reconstruction the
    method uses, written in Python integers."""
    v = []
    for t, m in enumerate(ms):
        P = 1
        acc = 0
        for s_ in range(t):
            acc += v[s_] * P
            P *= ms[s_]
        d = ((res[t] - acc) * pow(P, -1, m)) % m
        if d >= (m + 1) // 2:
            d -= m
        v.append(d)
    x, P = 0, 1
    for t, m in enumerate(ms):
        x += v[t] * P
        P *= m
    return x


def test_crt_reconstruction_recovers_products_within_the_budget():
    """The reading of the method behind the modular form: with the budget of
    crt_bits, residue products modulo each m_t (each operand reduced to a
    balanced residue first) determine the exact integer sum through
    balanced Garner digits, also at the extremes +-n 2^(bA+bX); with one
    modulus fewer the same extremes wrap."""
    rng = np.random.default_rng(5)
    for N, n in ((8, 17), (12, 64), (16, 300)):
        ms = _greedy_moduli(N)
        bA, bX = oracle.crt_bits(N, n)
        cases = [([2 ** bA] * n, [2 ** bX] * n), ([2 ** bA] * n, [-(2 ** bX)] * n)]
        for _ in range(5):
            a = [int(v) for v in rng.integers(-(2 ** 62), 2 ** 62, n)]
            x = [int(v) for v in rng.integers(-(2 ** 62), 2 ** 62, n)]
            cases.append(([v >> (62 - bA) for v in a], [v >> (62 - bX) for v in x]))
        for a, x in cases:
            exact = sum(p * q for p, q in zip(a, x))
            def bal(v, m):
                r = v % m
                return r - m if r >= (m + 1) // 2 else r
            res = [sum(bal(p, m) * bal(q, m) for p, q in zip(a, x)) % m for m in ms]
            assert _garner_balanced(res, ms) == exact
        a, x = cases[0]
        exact = sum(p * q for p, q in zip(a, x))
        short = ms[:-1]
        res = [sum(p * q for p, q in zip(a, x)) % m for m in short]
        assert _garner_balanced(res, short) != exact


def _short_integer_matrix(rows, cols, bits, seed, by_row):
    """Integers below 2^bits in magnitude times a power of two per line: the
    scaled images rint(m 2^(b - E)) are exact when b >= bits + 1."""
    rng = np.random.default_rng(seed)
    m = rng.integers(-(2 ** bits) + 1, 2 ** bits, (rows, cols)).astype(np.float64)
    ex = rng.integers(-20, 20, rows if by_row else cols)
    scale = np.exp2(ex)
    return m * (scale[:, None] if by_row else scale[None, :])


@pytest.mark.parametrize("N,bits", [(12, 20), (16, 48)])
def test_crt_product_is_exact_when_nothing_is_truncated(N, bits):
    """Operands of at most `bits` significant bits per line scale are
    represented exactly by the scaled integers, so the modular form must
    return the exact product (Python integers) as its (hi, lo) pair: hi the
    nearest double, lo the nearest double to the rest.  A is not symmetric,
    so a transposed operand or a swapped scale fails."""
    n, k = 40, 6
    bA, bX = oracle.crt_bits(N, n)
    assert bX >= bits + 1
    A = _short_integer_matrix(n, n, bits, 91 + N, True)
    X = _short_integer_matrix(n, k, bits, 92 + N, False)
    assert not np.array_equal(A, A.T)
    hi, lo = oracle.matmul_crt(A, X, N)
    ex = _exact_product(A, X)
    for i in range(n):
        for j in range(k):
            rest = ex[i][j] - Fraction(float(hi[i, j]))
            assert Fraction(float(hi[i, j])) == Fraction(float(ex[i][j]))  # nearest double
            assert Fraction(float(lo[i, j])) == Fraction(float(rest))
    if bits > 30:
        assert np.any(lo != 0.0)                     # the pair is needed


def _offdiag_exponents(A):
    """E_i: the smallest integer with max_{l != i} |a_il| < 2^E_i (0 for a
    zero line), in exact arithmetic."""
    E = []
    for i, row in enumerate(A):
        mx = max((abs(float(v)) for l, v in enumerate(row) if l != i), default=0.0)
        E.append(math.frexp(mx)[1] if mx > 0.0 else 0)
    return E


def _crt_error_check(A, X, moduli):
    """Largest error of the modular product relative to the line scales, after
    checking every entry against the truncation bound 2^(E_i-bA-1) sum_{l!=i}
    |x_lj| + 2^(F_j-bX-1) sum_{l!=i} |a_il| + n 2^(E_i+F_j-bA-bX-2) (each scaled
    image off by at most half a unit; E_i from the off-diagonal maxima, the
    diagonal's part exact) plus the pair's own rounding."""
    n, k = X.shape
    ex = _exact_product(A, X)
    EA = _offdiag_exponents(A)
    _, EX = oracle.split_digits(X, 1, False)
    worst = {}
    for N in moduli:
        bA, bX = oracle.crt_bits(N, n)
        hi, lo = oracle.matmul_crt(A, X, N)
        w = 0.0
        for i in range(n):
            sa = sum(Fraction(abs(float(v))) for l, v in enumerate(A[i]) if l != i)
            for j in range(k):
                sx = sum(Fraction(abs(float(X[l, j]))) for l in range(n) if l != i)
                ua = Fraction(2) ** (EA[i] - bA - 1)
                ux = Fraction(2) ** (int(EX[j]) - bX - 1)
                bound = ua * sx + ux * sa + n * ua * ux + abs(ex[i][j]) * Fraction(2) ** -104
                err = abs(Fraction(float(hi[i, j])) + Fraction(float(lo[i, j])) - ex[i][j])
                assert err <= bound, (N, i, j, float(err), float(bound))
                w = max(w, float(err / Fraction(2) ** (EA[i] + int(EX[j]))))
        worst[N] = w
    return worst


def test_crt_product_truncation_bound_and_rate():
    """Full 53-bit operands: every entry within the truncation bound, and four
    more moduli (about 31 bits more budget) cut the error by at least 2^12."""
    n, k = 29, 4
    A = _wide_range_matrix(n, n, 83)
    X = _wide_range_matrix(n, k, 84)
    worst = _crt_error_check(A, X, (8, 12, 16))
    assert worst[12] < worst[8] * 2.0 ** -12
    assert worst[16] < worst[12] * 2.0 ** -12


def test_crt_product_keeps_the_diagonal_out_of_the_image():
    """A diagonal 2^30 times the off-diagonal entries: the scales come from the
    off-diagonal maxima, so the error stays within the off-diagonal bound
    (about 2^-30 of what a full-row scale would give), and the diagonal's
    part a_ii x_ij is present exactly (an image that drops it, or rounds it
    to the off-diagonal unit, fails the bound)."""
    n, k = 24, 3
    rng = np.random.default_rng(87)
    A = rng.standard_normal((n, n))
    A[np.arange(n), np.arange(n)] = 2.0 ** 30 * (1.0 + rng.random(n))
    X = rng.standard_normal((n, k))
    _crt_error_check(A, X, (12,))


def test_crt_step_agrees_with_double_double_step():
    """A step whose line 1 comes from the modular form with 16 moduli (about
    56 bits per operand at n = 256) matches the Dot2 step to about u; with 8
    moduli (about 24 bits) it must not."""
    P = synth.dense_well_separated(256, 8)
    r_dd = oracle.refine_step(P.A, P.X0, norm_a=P.norm_a, dd=True)
    r_16 = oracle.refine_step(P.A, P.X0, norm_a=P.norm_a, crt=16)
    r_8 = oracle.refine_step(P.A, P.X0, norm_a=P.norm_a, crt=8)
    assert r_16.status == 0 and r_dd.status == 0
    assert np.max(np.abs(r_16.X - r_dd.X)) < 1e-15
    assert np.max(np.abs(r_8.X - r_dd.X)) > 1e-9


def test_separable_laplacian_generator_eigenpairs():
    """The separable-diagonal Laplacian used for the largest sparse timing
    run: its Kronecker-product eigenvectors are eigenvectors of the CSR
    matrix it builds (checked densely at N = 6), they are the k smallest, and
    sigma is the Gershgorin upper bound."""
    import scipy.sparse as sp
    P, lam, Xt, X0 = synth.laplacian3d_separable(6, 8)
    M = sp.csr_matrix((P.val, P.col_idx, P.row_ptr), shape=(P.n, P.n)).toarray()
    assert np.array_equal(M, M.T)
    assert np.max(np.abs(M @ Xt - Xt * lam)) < 1e-13
    w = np.linalg.eigvalsh(M)
    assert np.allclose(w[:8], lam, atol=1e-13) and w[8] == pytest.approx(P.meta["lam_next"], abs=1e-13)
    off = np.abs(M).sum(1) - np.abs(np.diag(M))
    assert P.sigma == pytest.approx(np.max(np.diag(M) + off), abs=1e-14)
    # the same pattern as laplacian3d
    L = synth.laplacian3d(6)
    assert np.array_equal(L.row_ptr, P.row_ptr) and np.array_equal(L.col_idx, P.col_idx)


# --------------------------------------------------------------------------
# Rayleigh-Ritz preprocessing (Sec. 3.4, clustered eigenvalues)
# --------------------------------------------------------------------------
def test_rayleigh_ritz_on_an_invariant_subspace_returns_its_eigenpairs():
    """X spans an exact invariant subspace (6 eigenvectors mixed by a random
    nonsingular R): the Ritz pairs are those eigenpairs, ordered by |lambda|
    descending, with the sign convention z_jj <= 0."""
    n, k = 80, 6
    rng = np.random.default_rng(31)
    lam = np.concatenate([rng.uniform(-0.5, 0.5, n - k), [0.9, -0.85, 0.8, 0.75, -0.7, 0.65]])
    A, Q = _sym_problem(n, lam, 32)
    idx = np.arange(n - k, n)
    R = rng.standard_normal((k, k)) + 3.0 * np.eye(k)
    X = Q[:, idx] @ R
    Z, theta = oracle.rayleigh_ritz(A, X)
    want = lam[idx][np.argsort(-np.abs(lam[idx]))]
    assert np.allclose(theta, want, atol=1e-13)
    Qs = Q[:, idx][:, np.argsort(-np.abs(lam[idx]))]
    assert max_abs_diff_aligned(Z, Qs) < 1e-12
    assert np.all(np.diag(Z[:k]) <= 0.0)


def test_rayleigh_ritz_basis_properties_and_separation_theorem():
    """On a clustered problem from an fp32-accurate start: Z^T Z = I and
    Z^T A Z = diag(theta) to rounding, and the Ritz values obey the
    Poincare separation theorem lam_{n-k+i} <= theta_i <= lam_i (both sorted
    descending).  Shifted ordering: with mu above the spectrum the columns
    come in ascending theta."""
    P = synth.dense_clustered(300, 8, 71)
    A, X = P.A, P.X0
    Z, theta = oracle.rayleigh_ritz(A, X)
    k = X.shape[1]
    assert np.max(np.abs(Z.T @ Z - np.eye(k))) < 1e-13
    H = Z.T @ (A @ Z)
    assert np.max(np.abs(H - np.diag(theta))) < 1e-13
    lam = np.sort(np.linalg.eigvalsh(A))[::-1]
    th = np.sort(theta)[::-1]
    n = A.shape[0]
    assert np.all(th <= lam[:k] + 1e-13) and np.all(th >= lam[n - k:] - 1e-13)
    assert np.all(np.diff(np.abs(theta)) <= 0.0)
    Zs, ths = oracle.rayleigh_ritz(A, X, mu=2.0)
    assert np.all(np.diff(ths) >= 0.0)


def test_rr_zero_top_step_keeps_the_bottom_block():
    """The step after Rayleigh-Ritz with the leading k x k block of E_L set to
    zero: that block is exactly zero, the bottom rows equal those of the
    plain step on the same input (they do not depend on the option), and the
    plain step's leading block on a Ritz basis is only rounding-sized
    off the clusters."""
    P = synth.dense_clustered(200, 6, 91)
    Z, theta = oracle.rayleigh_ritz(P.A, P.X0)
    k = Z.shape[1]
    a = oracle.refine_step(P.A, Z, norm_a=1.0, rr_top=True, normalize=False)
    b = oracle.refine_step(P.A, Z, norm_a=1.0, normalize=False)
    assert a.status == 0 and b.status == 0
    assert np.all(a.E[:k] == 0.0)
    assert np.array_equal(a.E[k:], b.E[k:])
    assert np.max(np.abs(np.diag(b.E[:k]))) < 1e-14
    assert a.corr_fro <= b.corr_fro


# --------------------------------------------------------------------------
# Modified LU, compact WY from it, and the one-time sign flip (Sec. 3.1.1)
# --------------------------------------------------------------------------
def _x_with_singular_y1(n, k, seed):
    """Orthonormal columns whose first one is e_1 (so Y1 = X1 - I has a zero
    column and Algorithm 1 cannot run)."""
    Xo = _orthonormal(n - 1, k - 1, seed)
    X = np.zeros((n, k))
    X[0, 0] = 1.0
    X[1:, 1:] = Xo
    return X


@pytest.mark.parametrize("case", ["random", "singular_y1"])
def test_modified_lu_factorises_q_minus_sigma(case):
    n, k = 40, 6
    X = _orthonormal(n, k, 77) if case == "random" else _x_with_singular_y1(n, k, 78)
    Y, U, sigma = oracle.modified_lu(X)
    S = np.zeros((n, k))
    S[np.arange(k), np.arange(k)] = sigma
    assert np.max(np.abs(X - S - Y @ U)) < 1e-14
    assert np.all(np.abs(np.diag(U)) >= 1.0 - 1e-14)
    assert np.array_equal(np.abs(sigma), np.ones(k))
    assert np.allclose(np.tril(U, -1), 0.0) and np.allclose(np.diag(Y[:k]), 1.0)


@pytest.mark.parametrize("case", ["random", "singular_y1"])
def test_compact_wy_lu_is_orthogonal_and_maps_the_first_columns(case):
    """Algorithm 3 for any orthonormal Q, including one whose Y1 is singular
    for Algorithm 1: H = I - Y T Y^T is orthogonal and its first k columns are
    Q Sigma (I_{n,k} + Y U Sigma = I_{n,k} + (Q - Sigma) Sigma), i.e. Q up to
    the column signs that the one-time flip absorbs."""
    n, k = 30, 5
    X = _orthonormal(n, k, 81) if case == "random" else _x_with_singular_y1(n, k, 82)
    Y, T, sigma = oracle.compact_wy_lu(X)
    H = np.eye(n) - Y @ T @ Y.T
    assert np.max(np.abs(H.T @ H - np.eye(n))) < 1e-13
    assert np.max(np.abs(H[:, :k] - X * sigma)) < 1e-13
    # T is upper triangular, as a compact WY T factor is
    assert np.max(np.abs(np.tril(T, -1))) < 1e-13


def test_sign_flip_makes_compact_wy_applicable():
    """Algorithm 1 fails on X (Y1 singular) and succeeds on X Sigma, whose
    columns span the same space; the flip changes signs only."""
    n, k = 50, 5
    X = _x_with_singular_y1(n, k, 83)
    rc, _, _, _ = oracle.compact_wy(X)
    assert rc == oracle.SINGULAR
    Xf, sigma = oracle.sign_flip(X)
    assert np.array_equal(np.abs(Xf), np.abs(X))
    rc, Y, T, cond = oracle.compact_wy(Xf)
    assert rc == oracle.OK and cond < 1e3
    H = np.eye(n) - Y @ T @ Y.T
    assert np.max(np.abs(H[:, :k] - Xf)) < 1e-13


# --------------------------------------------------------------------------
# Squared shift for the smallest |lambda| (Sec. 5.2): B = A^2 - alpha I, with
# A^2 X formed as A (A X)
# --------------------------------------------------------------------------
def test_square_equals_the_step_on_an_explicit_square():
    """The step on B = A^2 - alpha I through two products equals the plain
    shifted step on the explicitly formed (and symmetrised) A^2."""
    n, k = 60, 4
    P = synth.dense_smallest_abs(n, k, 91)
    A = P.A
    alpha = 0.6
    r1 = oracle.refine_step(A, P.X0, mu=alpha, norm_a=1.0, square=True)
    A2 = A @ A
    A2 = 0.5 * (A2 + A2.T)
    r2 = oracle.refine_step(A2, P.X0, mu=alpha, norm_a=1.0)
    assert r1.status == 0 and r2.status == 0
    assert np.max(np.abs(r1.X - r2.X)) < 1e-14
    assert np.max(np.abs(r1.d - r2.d)) < 1e-14


def test_square_k1_is_the_power_method_on_b():
    """k = 1: one step is one power iteration x <- B x / ||B x|| on
    B = A^2 - alpha I."""
    n = 41
    A, Q = _sym_problem(n, np.linspace(-1.0, 0.9, n), 17)
    rng = np.random.default_rng(17)
    x = Q[:, 20:21] + 0.05 * rng.standard_normal((n, 1))
    x /= np.linalg.norm(x)
    alpha = 0.7
    r = oracle.refine_step(A, x, mu=alpha, norm_a=1.0, square=True)
    y = A @ (A @ x) - alpha * x
    y /= np.linalg.norm(y)
    assert max_abs_diff_aligned(r.X, y) < 1e-15


def test_square_converges_to_the_smallest_abs_eigenvectors():
    """With alpha = (||A||^2 + lambda_{k+1}^2) / 2 the targets of smallest
    |lambda| (both signs) satisfy the separation condition for B; the
    iterates converge to them and d~ to lambda^2.  The same step without the
    square (mu = 0) drifts away from them, as eq. (condition) predicts."""
    n, k = 80, 5
    P = synth.dense_smallest_abs(n, k, 93)
    lam_t = P.lam[P.targets]
    rest = np.delete(P.lam, P.targets)
    alpha = (1.0 + np.min(np.abs(rest)) ** 2) / 2
    X = P.X0
    for _ in range(20):
        r = oracle.refine_step(P.A, X, mu=alpha, norm_a=1.0, square=True)
        assert r.status == 0
        X = r.X
    assert max_abs_diff_aligned(X, P.X_true) < 1e-13
    assert np.max(np.abs(r.d - lam_t ** 2)) < 1e-14
    Xp = P.X0
    for _ in range(12):
        rp = oracle.refine_step(P.A, Xp, norm_a=1.0)
        if rp.status != 0:
            break
        Xp = rp.X
    assert rp.status != 0 or max_abs_diff_aligned(Xp, P.X_true) > 1e-3


def test_square_rayleigh_ritz_orders_by_distance_from_alpha():
    """Rayleigh-Ritz on the squared pencil: theta are lambda^2 of the
    targets, ascending (largest |theta - alpha| first)."""
    n, k = 70, 4
    P = synth.dense_smallest_abs(n, k, 95)
    Z, theta = oracle.rayleigh_ritz(P.A, P.X0, mu=0.6, square=True)
    assert np.all(np.diff(theta) >= 0.0)
    assert np.max(np.abs(theta - np.sort(P.lam[P.targets] ** 2))) < 1e-12
