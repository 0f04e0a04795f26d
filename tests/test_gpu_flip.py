"""One-time column sign flip X <- X Sigma (Sec. 3.1.1; Sigma of the modified LU,
Algorithm 2) on the GPU against the oracle, through the C ABI.

Sigma is a sign decision taken in FP64 on both sides with the same operations
(one rounding for each division and each product and difference of the
elimination), so it is compared exactly, and the flipped X is compared bit for
bit.  On the singular case (an exact eigenvector e_1 as the first column, so
Y1 = X1 - I has a zero column) the step reports the singular status and keeps
X; after the flip the steps match the oracle's on its own flipped X.
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


@pytest.mark.parametrize("n,k", [(300, 12), (640, 128), (129, 1), (1000, 37), (70, 69)])
def test_sign_flip_matches_oracle(n, k):
    rf = _lib()
    P = synth.dense_spectrum(n, k, 7100 + n + k)
    ctx = rf.RefineContext(_dev(P.A), k, norm_a=1.0)
    X = _dev(P.X0).clone()
    sigma = ctx.sign_flip(X)
    ctx.close()
    Xo, so = oracle.sign_flip(P.X0)
    assert sigma == [int(v) for v in so]
    assert np.array_equal(X.cpu().numpy(), Xo)


def test_sign_flip_on_a_padded_leading_dimension():
    rf = _lib()
    n, k = 400, 20
    P = synth.dense_spectrum(n, k, 7150)
    ctx = rf.RefineContext(_dev(P.A), k, norm_a=1.0)
    buf = torch.full((n, k + 5), 7.0, dtype=torch.float64, device="cuda")
    buf[:, :k] = _dev(P.X0)
    X = buf[:, :k]
    ctx.sign_flip(X)
    ctx.close()
    Xo, _ = oracle.sign_flip(P.X0)
    assert np.array_equal(X.cpu().numpy(), Xo)
    assert bool((buf[:, k:] == 7.0).all())


@pytest.mark.parametrize("precision,slices", [("fp64", 0), ("split_int8", 9)])
def test_singular_y1_then_flip_then_steps_match_oracle(precision, slices):
    rf = _lib()
    n, k = 500, 10
    P = synth.dense_exact_first(n, k, 7200)
    ctx = rf.RefineContext(_dev(P.A), k, norm_a=1.0, precision=precision, slices=slices)
    X = _dev(P.X0).clone()
    st = ctx.step(X)
    assert st.status == rf.EWY_SINGULAR
    assert np.array_equal(X.cpu().numpy(), P.X0)
    sigma = ctx.sign_flip(X)
    Xo, so = oracle.sign_flip(P.X0)
    assert sigma == [int(v) for v in so] and sigma[0] == -1
    for s in range(3):
        st = ctx.step(X)
        assert st.status == rf.OK, rf.status_string(st.status)
        r = oracle.refine_step(P.A, Xo, norm_a=1.0)
        assert r.status == oracle.OK
        Xo = r.X
        err = float(np.max(np.abs(align_signs(X.cpu().numpy(), Xo) - Xo)))
        assert err <= TOL, "step %d: %.3e" % (s, err)
        assert st.corr_fro == pytest.approx(r.corr_fro, rel=1e-6, abs=1e-15)
    ctx.close()


def test_flip_after_rayleigh_ritz_keeps_the_zero_leading_block():
    """Flipping the signs of a Ritz basis leaves X^T A X diagonal, so the
    next step still takes E11 = 0 (oracle rr_top)."""
    rf = _lib()
    P = synth.dense_spectrum(600, 16, 7300)
    ctx = rf.RefineContext(_dev(P.A), 16, norm_a=1.0)
    X = _dev(P.X0).clone()
    ctx.rayleigh_ritz(X)
    Z = X.cpu().numpy()
    ctx.sign_flip(X)
    Zf, _ = oracle.sign_flip(Z)
    assert np.array_equal(X.cpu().numpy(), Zf)
    st = ctx.step(X)
    assert st.status == rf.OK
    r = oracle.refine_step(P.A, Zf, norm_a=1.0, rr_top=True)
    err = float(np.max(np.abs(align_signs(X.cpu().numpy(), r.X) - r.X)))
    assert err <= TOL
    ctx.close()


def test_sign_flip_rejects_non_finite_leading_block():
    rf = _lib()
    P = synth.dense_spectrum(200, 6, 7400)
    X0 = np.array(P.X0)
    X0[2, 4] = np.nan
    ctx = rf.RefineContext(_dev(P.A), 6, norm_a=1.0)
    X = _dev(X0).clone()
    with pytest.raises(rf.RefineError) as ei:
        ctx.sign_flip(X)
    assert ei.value.status == rf.ENONFINITE
    assert np.array_equal(np.isnan(X.cpu().numpy()), np.isnan(X0))
    assert np.array_equal(np.nan_to_num(X.cpu().numpy()), np.nan_to_num(X0))
    X2 = _dev(P.X0).clone()
    assert ctx.step(X2).status == rf.OK
    ctx.close()


def test_batched_sign_flip_matches_oracle_per_problem():
    """Grouped launch over uneven problems: one with an exact e_1 column,
    one with an Inf in its leading block (which alone reports the non-finite
    status and keeps its X); then a step of every other problem matches the
    oracle step on the oracle's flipped X."""
    rf = _lib()
    shapes = [(130, 4), (257, 9), (511, 32), (200, 17), (129, 31)]
    probs = [synth.dense_spectrum(n, k, 7500 + i) for i, (n, k) in enumerate(shapes)]
    probs[1] = synth.dense_exact_first(257, 9, 7511)
    X0s = [np.array(p.X0) for p in probs]
    X0s[3][5, 1] = np.inf
    b = rf.RefineBatch([_dev(p.A) for p in probs], [k for _, k in shapes], norm_a=1.0)
    Xs = [_dev(x).clone() for x in X0s]
    rc, st = b.sign_flip(Xs)
    assert rc == rf.ENONFINITE and st == [0, 0, 0, rf.ENONFINITE, 0]
    assert np.array_equal(Xs[3].cpu().numpy(), X0s[3])
    for i in (0, 1, 2, 4):
        Xo, _ = oracle.sign_flip(X0s[i])
        assert np.array_equal(Xs[i].cpu().numpy(), Xo), "problem %d" % i
    Xs[3] = _dev(probs[3].X0).clone()
    rc, per = b.run(Xs, 1)
    assert rc == rf.OK
    for i in (0, 1, 2, 4):
        Xo, _ = oracle.sign_flip(X0s[i])
        r = oracle.refine_step(probs[i].A, Xo, norm_a=1.0)
        err = float(np.max(np.abs(align_signs(Xs[i].cpu().numpy(), r.X) - r.X)))
        assert err <= TOL, "problem %d: %.3e" % (i, err)
    b.close()
