"""Squared-shift variant for the eigenvectors of smallest |lambda| (Sec. 5.2)
on the GPU against the oracle, through the C ABI.

The method runs on B = A^2 - alpha I with the product step of Algorithm 4 as A (A X)
(two products; A^2 is never formed) and alpha = (||A||^2 + lhat^2) / 2.  The
GPU takes the Rayleigh quotient of A^2 as ||A x||^2 / x^T x (the second
product's input norm), the oracle as x^T (A (A x)) / x^T x; for symmetric A
the two agree to rounding, and the step is compared entry by entry.  Targets
of both signs sit at |lambda| <= 0.3 with lambda^2 gaps >= 4e-3, so the
comparison is not limited by the squared gaps (u / gap_B ~ 3e-14).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._util import align_signs

pytestmark = pytest.mark.gpu

TOL = 1e-13
LHAT = 0.7          # estimate of the (k+1)-th smallest |lambda| (the rest lie in [0.7, 1])


def _lib():
    import paper_2602_23778_amd as rf
    rf.load_library()
    return rf


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def _err(g, o):
    return float(np.max(np.abs(align_signs(g, o) - o)))


@pytest.mark.parametrize("n,k", [(500, 8), (333, 13), (640, 64), (257, 1)])
def test_square_steps_match_oracle(n, k):
    rf = _lib()
    P = synth.dense_smallest_abs(n, k, 8100 + n + k)
    ctx = rf.RefineContext(_dev(P.A), k, norm_a=1.0, target="smallest_abs", shift=LHAT)
    alpha = 0.5 * (1.0 + LHAT ** 2)
    info = ctx.info()
    assert info["mu"] == pytest.approx(alpha, rel=1e-15)
    assert info["norm_used"] == pytest.approx(1.0, rel=1e-15)
    X = _dev(P.X0).clone()
    Xo = P.X0
    for s in range(3):
        st = ctx.step(X)
        assert st.status == rf.OK, rf.status_string(st.status)
        r = oracle.refine_step(P.A, Xo, mu=alpha, norm_a=1.0, square=True)
        assert r.status == oracle.OK
        Xo = r.X
        err = _err(X.cpu().numpy(), Xo)
        assert err <= TOL, "step %d: %.3e" % (s, err)
        assert st.corr_fro == pytest.approx(r.corr_fro, rel=1e-6, abs=1e-15)
        assert st.resid_rel == pytest.approx(r.resid_rel, rel=1e-6, abs=1e-16)
    ctx.close()


def test_square_converges_to_the_smallest_abs_eigenvectors():
    rf = _lib()
    n, k = 600, 6
    P = synth.dense_smallest_abs(n, k, 8200)
    ctx = rf.RefineContext(_dev(P.A), k, norm_a=1.0, target="smallest_abs", shift=LHAT)
    X = _dev(P.X0).clone()
    st = ctx.run(X, 25)
    ctx.close()
    assert st.status == rf.OK
    assert _err(X.cpu().numpy(), P.X_true) < 1e-12


def test_square_default_alpha_without_estimate():
    """shift <= 0: alpha = ||A||^2 (here the caller's norm_a = 1)."""
    rf = _lib()
    P = synth.dense_smallest_abs(300, 5, 8250)
    ctx = rf.RefineContext(_dev(P.A), 5, norm_a=1.0, target="smallest_abs")
    assert ctx.info()["mu"] == pytest.approx(1.0, rel=1e-15)
    X = _dev(P.X0).clone()
    st = ctx.step(X)
    ctx.close()
    r = oracle.refine_step(P.A, P.X0, mu=1.0, norm_a=1.0, square=True)
    assert st.status == rf.OK
    assert _err(X.cpu().numpy(), r.X) <= TOL


def _dense_as_csr(A):
    n = A.shape[0]
    rp = np.arange(0, n * n + 1, n, dtype=np.int32)
    ci = np.tile(np.arange(n, dtype=np.int32), n)
    return rp, ci, np.ascontiguousarray(A).reshape(-1)


def test_square_csr_matches_oracle():
    """CSR product twice per step, on the well-separated dense spectrum
    stored as CSR (every entry)."""
    rf = _lib()
    n, k = 300, 7
    P = synth.dense_smallest_abs(n, k, 8260)
    rp, ci, av = _dense_as_csr(P.A)
    C = rf.CsrMatrix(n, _dev(rp), _dev(ci), _dev(av))
    ctx = rf.RefineContext(C, k, target="smallest_abs", shift=LHAT, norm_a=1.0)
    alpha = 0.5 * (1.0 + LHAT ** 2)
    Ao = oracle.Csr(n, rp, ci, av)
    X = _dev(P.X0).clone()
    Xo = P.X0
    for s in range(3):
        st = ctx.step(X)
        assert st.status == rf.OK, rf.status_string(st.status)
        Xo = oracle.refine_step(Ao, Xo, mu=alpha, norm_a=1.0, square=True).X
        err = _err(X.cpu().numpy(), Xo)
        assert err <= TOL, "step %d: %.3e" % (s, err)
    ctx.close()


def test_square_csr_laplacian():
    """The 3-D Laplacian's smallest eigenvalues through the squared variant.
    Their squares lie 0.04 apart against ||B|| <= sigma^2 = 167, so rounding
    differences between two correct FP64 products grow by ||B|| / gap ~ 4e3
    in the correction; the bound is 32 u ||B|| / gap (1.5e-11)."""
    rf = _lib()
    L, lam, Xt, X0 = synth.laplacian3d_separable(12, 8)
    lhat = 1.2
    C = rf.CsrMatrix(L.n, _dev(L.row_ptr), _dev(L.col_idx), _dev(L.val))
    ctx = rf.RefineContext(C, 8, target="smallest_abs", shift=lhat, norm_a=L.sigma)
    alpha = 0.5 * (L.sigma ** 2 + lhat ** 2)
    assert ctx.info()["mu"] == pytest.approx(alpha, rel=1e-15)
    sq = np.sort(lam ** 2)
    tol = 32 * 2.0 ** -53 * L.sigma ** 2 / float(np.min(np.diff(sq)))
    X = _dev(X0).clone()
    Ao = oracle.Csr(L.n, L.row_ptr, L.col_idx, L.val)
    Xo = X0
    for s in range(2):
        st = ctx.step(X)
        assert st.status == rf.OK, rf.status_string(st.status)
        Xo = oracle.refine_step(Ao, Xo, mu=alpha, norm_a=L.sigma ** 2, square=True).X
        err = _err(X.cpu().numpy(), Xo)
        assert err <= tol, "step %d: %.3e (bound %.1e)" % (s, err, tol)
    ctx.close()


def test_square_rayleigh_ritz_then_step():
    rf = _lib()
    n, k = 500, 8
    P = synth.dense_smallest_abs(n, k, 8300)
    alpha = 0.5 * (1.0 + LHAT ** 2)
    ctx = rf.RefineContext(_dev(P.A), k, norm_a=1.0, target="smallest_abs", shift=LHAT)
    X = _dev(P.X0).clone()
    ctx.rayleigh_ritz(X)
    Zo, theta = oracle.rayleigh_ritz(P.A, P.X0, mu=alpha, square=True)
    assert np.all(np.diff(theta) >= 0.0)
    assert float(np.max(np.abs(X.cpu().numpy() - Zo))) <= TOL
    st = ctx.step(X)
    assert st.status == rf.OK
    r = oracle.refine_step(P.A, Zo, mu=alpha, norm_a=1.0, square=True, rr_top=True)
    assert _err(X.cpu().numpy(), r.X) <= TOL
    ctx.close()


def test_square_batch_matches_oracle_per_problem():
    rf = _lib()
    shapes = [(130, 4), (257, 9), (511, 32), (200, 17)]
    probs = [synth.dense_smallest_abs(n, k, 8400 + i) for i, (n, k) in enumerate(shapes)]
    alpha = 0.5 * (1.0 + LHAT ** 2)
    b = rf.RefineBatch([_dev(p.A) for p in probs], [k for _, k in shapes], norm_a=1.0,
                       target="smallest_abs", shift=LHAT)
    Xs = [_dev(p.X0).clone() for p in probs]
    rc, per = b.run(Xs, 2)
    b.close()
    assert rc == rf.OK
    for i, p in enumerate(probs):
        Xo, _ = oracle.refine(p.A, p.X0, 2, mu=alpha, norm_a=1.0, square=True)
        assert _err(Xs[i].cpu().numpy(), Xo) <= TOL, "problem %d" % i


def test_square_rejects_the_split_form():
    rf = _lib()
    P = synth.dense_smallest_abs(200, 4, 8500)
    with pytest.raises(rf.RefineError) as ei:
        rf.RefineContext(_dev(P.A), 4, norm_a=1.0, target="smallest_abs", shift=LHAT,
                         precision="split_int8", slices=9)
    assert ei.value.status == rf.EINVAL
