"""Parity of the modular form of the product (Ozaki scheme II: residues of A
and X modulo N coprime moduli, one INT8 product per modulus on the matrix
cores, Chinese-remainder reconstruction into a double-double W) with the
oracle's modular product, which forms the same exact integer product of the
scaled images directly.

The GPU pair (W_hi, W_lo) carries the exact integer up to the rounding of its
double-double Horner evaluation (relative 2^-104 once the integer exceeds 106
bits), so the products are compared to 2^-100 max |W|; whole steps are
compared with the oracle's steps of the same form (1e-13), and with its Dot2
steps.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import align_signs

pytestmark = pytest.mark.gpu

TOL = 1e-13


def _lib():
    import paper_2602_23778_amd as rf
    rf.load_library()
    return rf


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def _say(msg):
    print(msg, flush=True)


def _product_check(A, X0, k, nmod):
    rf = _lib()
    n = A.shape[0]
    _say("case: modular product n=%d k=%d N=%d" % (n, k, nmod))
    ctx = rf.RefineContext(_dev(A), k, norm_a=1.0, precision="split_crt", slices=nmod)
    X = _dev(X0).clone()
    ctx.time_product(X, 1)           # the product alone, into the workspace's W
    wh, wl = ctx.debug_product()
    ctx.close()
    oh, ol = oracle.matmul_crt(A, X0, nmod)
    d = (wh.cpu().numpy() - oh) + (wl.cpu().numpy() - ol)
    scale = np.max(np.abs(oh))
    err = float(np.max(np.abs(d)))
    assert err <= 2.0 ** -100 * scale, "n=%d k=%d N=%d: |dW| = %.3e (max|W| %.3e)" % (
        n, k, nmod, err, scale)
    # the high parts agree exactly wherever the GPU's pair is the nearest one
    assert np.mean(wh.cpu().numpy() == oh) > 0.99


@pytest.mark.parametrize("n,k", [(777, 13), (1000, 64), (1280, 33), (640, 128), (300, 1),
                                 (513, 96), (150, 128), (30, 5), (2049, 40)])
def test_crt_product_matches_oracle(n, k):
    """Ragged n (not a multiple of the 32-wide chunks, of the chunk groups or
    of the 128-row blocks), every column-tile layout (k <= 32, 64, 96, 128)."""
    P = synth.dense_spectrum(n, k, 6000 + n)
    _product_check(P.A, P.X0, k, 16)


@pytest.mark.parametrize("nmod", [12, 13, 14, 15])
def test_crt_product_other_moduli_counts(nmod):
    P = synth.dense_spectrum(700, 40, 6100 + nmod)
    _product_check(P.A, P.X0, 40, nmod)


def test_crt_product_wide_dynamic_range():
    """Entries spanning many binades in every row and column, a zero row and
    column of A, a zero column of X: the scaled images use their whole bit
    budget and many are rounded, and the GPU still returns the oracle's exact
    integer product."""
    rng = np.random.default_rng(61)
    n, k = 520, 24
    A = rng.standard_normal((n, n)) * np.exp2(rng.integers(-30, 4, (n, n)))
    A = 0.5 * (A + A.T)
    A[7, :] = 0.0
    A[:, 7] = 0.0
    X = rng.standard_normal((n, k)) * np.exp2(rng.integers(-20, 2, (n, k)))
    X[:, 5] = 0.0
    _product_check(A, X, k, 16)


@pytest.mark.parametrize("n,k", [(777, 13), (640, 64), (513, 17)])
def test_crt_steps_match_oracle(n, k):
    """Whole modular-form steps against the oracle's modular-form steps (the
    same product definition) and against its Dot2 steps."""
    rf = _lib()
    P = synth.dense_spectrum(n, k, 6200 + n)
    ctx = rf.RefineContext(_dev(P.A), k, norm_a=1.0, precision="split_crt")
    Xg = _dev(P.X0).clone()
    Xo = np.array(P.X0, copy=True)
    for s in range(3):
        st = ctx.step(Xg)
        assert st.status == rf.OK, rf.status_string(st.status)
        r = oracle.refine_step(P.A, Xo, norm_a=1.0, crt=16)
        assert r.status == 0
        Xo = r.X
        got = Xg.cpu().numpy()
        err = float(np.max(np.abs(align_signs(got, Xo) - Xo)))
        assert err <= TOL, "step %d: max |dX| = %.3e" % (s, err)
        assert st.corr_fro == pytest.approx(r.corr_fro, rel=1e-6, abs=1e-15)
        assert st.resid_rel == pytest.approx(r.resid_rel, rel=1e-6, abs=1e-15)
        assert st.iters == s + 1
    ctx.close()
    Xd, _ = oracle.refine(P.A, P.X0, 3, norm_a=1.0, dd=True)
    assert np.max(np.abs(align_signs(Xg.cpu().numpy(), Xd) - Xd)) <= TOL


def test_crt_uniform_top_reduced():
    """The uniform spectrum with 128 targets 1e-3 apart (n = 2048, k = 128):
    two modular-form steps against the double-double oracle."""
    rf = _lib()
    P = synth.dense_uniform_top(2048, 128)
    ctx = rf.RefineContext(_dev(P.A), 128, norm_a=1.0, precision="split_crt")
    X = _dev(P.X0).clone()
    for _ in range(2):
        st = ctx.step(X)
        assert st.status == rf.OK, rf.status_string(st.status)
    ctx.close()
    Xd, _ = oracle.refine(P.A, P.X0, 2, norm_a=1.0, dd=True)
    err = float(np.max(np.abs(align_signs(X.cpu().numpy(), Xd) - Xd)))
    _say("uniform top 2048 x 128, two steps: %.3e vs the Dot2 oracle" % err)
    assert err <= TOL


def test_crt_shift_and_run():
    """A shifted target (the smallest eigenvalues through the Gershgorin
    bound) for one step, and refine_run's eight-step graphs with the modular
    product: sixteen steps against sixteen oracle steps of the same form."""
    rf = _lib()
    n, k = 600, 6
    P = synth.dense_spectrum(n, k, 6300)
    lam, Q = np.linalg.eigh(P.A)
    X0 = synth.fp32_round(Q[:, :k])
    ctx = rf.RefineContext(_dev(P.A), k, target="smallest", norm_a=1.0, precision="split_crt")
    mu = ctx.info()["mu"]
    Xg = _dev(X0).clone()
    st = ctx.step(Xg)
    assert st.status == rf.OK, rf.status_string(st.status)
    ctx.close()
    r = oracle.refine_step(P.A, X0, mu=mu, norm_a=1.0, crt=16)
    assert float(np.max(np.abs(align_signs(Xg.cpu().numpy(), r.X) - r.X))) <= TOL
    ctx = rf.RefineContext(_dev(P.A), k, norm_a=1.0, precision="split_crt")
    Xg = _dev(P.X0).clone()
    st = ctx.run(Xg, 16, stop="iters")
    assert st.status == rf.OK and st.iters == 16, rf.status_string(st.status)
    ctx.close()
    Xo, hist = oracle.refine(P.A, P.X0, 16, norm_a=1.0, crt=16)
    assert len(hist) == 16 and hist[-1].status == 0
    assert float(np.max(np.abs(align_signs(Xg.cpu().numpy(), Xo) - Xo))) <= TOL


def test_crt_step_is_deterministic():
    rf = _lib()
    P = synth.dense_spectrum(900, 32, 6400)
    out = []
    for _ in range(2):
        ctx = rf.RefineContext(_dev(P.A), 32, norm_a=1.0, precision="split_crt")
        X = _dev(P.X0).clone()
        for _ in range(3):
            ctx.step(X)
        ctx.close()
        out.append(X.cpu().numpy())
    assert np.array_equal(out[0], out[1])


def test_crt_invalid_arguments():
    rf = _lib()
    A = _dev(np.eye(64))
    for bad in (11, 17, -1):
        with pytest.raises(rf.RefineError) as e:
            rf.RefineContext(A, 4, precision="split_crt", slices=bad)
        assert e.value.status == rf.EINVAL
    L = synth.laplacian3d(4, seed=1)
    C = rf.CsrMatrix(L.n, _dev(L.row_ptr), _dev(L.col_idx), _dev(L.val))
    with pytest.raises(rf.RefineError) as e:
        rf.RefineContext(C, 4, precision="split_crt")
    assert e.value.status == rf.EINVAL
    with pytest.raises(rf.RefineError) as e:
        rf.RefineBatch([A, A], [4, 4], precision="split_crt")
    assert e.value.status == rf.EINVAL
