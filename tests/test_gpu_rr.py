"""Rayleigh-Ritz preprocessing (Sec. 3.4, clustered eigenvalues) on the GPU
against the oracle, through the C ABI.

On well-separated spectra the Ritz vectors are unique up to sign, and both
sides fix the sign (z_jj <= 0) and the order (|theta - mu| descending), so
the comparison is entry by entry.  Inside a cluster of gap 1e-6 only the
cluster's subspace is determined to rounding (a vector inside it only to
about u / gap), so there the subspaces are compared, together with the
properties Z^T Z = I and Z^T A Z diagonal that hold for any valid answer.
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


@pytest.mark.parametrize("precision,slices", [("fp64", 0), ("split_int8", 9)])
@pytest.mark.parametrize("n,k", [(500, 12), (333, 13), (640, 64), (300, 1)])
def test_rayleigh_ritz_matches_oracle(n, k, precision, slices):
    rf = _lib()
    P = synth.dense_spectrum(n, k, 6100 + n + k)
    ctx = rf.RefineContext(_dev(P.A), k, norm_a=1.0, precision=precision, slices=slices)
    X = _dev(P.X0).clone()
    ctx.rayleigh_ritz(X)
    ctx.close()
    Zo, theta = oracle.rayleigh_ritz(P.A, P.X0)
    Z = X.cpu().numpy()
    err = float(np.max(np.abs(Z - Zo)))
    assert err <= TOL, "max |Z - Z_oracle| = %.3e" % err
    assert np.all(np.diag(Z[:k]) <= 0.0)


def test_rayleigh_ritz_csr_smallest():
    """CSR product and the shifted order (targets the smallest eigenvalues,
    mu = Gershgorin bound, so the columns come in ascending theta)."""
    rf = _lib()
    L, lam, Xt, X0 = synth.laplacian3d_separable(12, 8)
    C = rf.CsrMatrix(L.n, _dev(L.row_ptr), _dev(L.col_idx), _dev(L.val))
    ctx = rf.RefineContext(C, 8, target="smallest", norm_a=L.sigma)
    X = _dev(X0).clone()
    ctx.rayleigh_ritz(X)
    ctx.close()
    Zo, theta = oracle.rayleigh_ritz(oracle.Csr(L.n, L.row_ptr, L.col_idx, L.val), X0, mu=L.sigma)
    assert np.all(np.diff(theta) >= 0.0)
    assert float(np.max(np.abs(X.cpu().numpy() - Zo))) <= TOL


def test_rayleigh_ritz_then_steps_match_oracle():
    """The step after Rayleigh-Ritz takes E11 = 0 (oracle rr_top), the next one
    is plain again; iterates and statistics match the oracle's."""
    rf = _lib()
    P = synth.dense_spectrum(700, 16, 6200)
    ctx = rf.RefineContext(_dev(P.A), 16, norm_a=1.0)
    X = _dev(P.X0).clone()
    ctx.rayleigh_ritz(X)
    Xo, _ = oracle.rayleigh_ritz(P.A, P.X0)
    for s in range(3):
        st = ctx.step(X)
        assert st.status == rf.OK
        r = oracle.refine_step(P.A, Xo, norm_a=1.0, rr_top=(s == 0))
        Xo = r.X
        err = float(np.max(np.abs(align_signs(X.cpu().numpy(), Xo) - Xo)))
        assert err <= TOL, "step %d: %.3e" % (s, err)
        assert st.corr_fro == pytest.approx(r.corr_fro, rel=1e-6, abs=1e-15)
    ctx.close()


def test_rayleigh_ritz_on_clusters_then_refinement():
    """Two clusters with internal gaps of 1e-6 (split form, 10 slices): the
    Ritz basis is orthonormal and diagonalises A to rounding and spans the
    oracle's cluster subspaces.  Inside a cluster the Ritz vectors are fixed
    only to about u / gap, so the refinement that follows is compared by its
    distance to the exact eigenvectors: it falls as the oracle's does on the
    same path (Rayleigh-Ritz, then steps with a double-double product; the
    targets sit 0.98-0.99 over a rest below 0.97, so the rate is slow)."""
    rf = _lib()
    P = synth.dense_clustered(300, 8, 6300)
    A, k = P.A, 8
    ctx = rf.RefineContext(_dev(A), k, norm_a=1.0, precision="split_int8", slices=10)
    X = _dev(P.X0).clone()
    ctx.rayleigh_ritz(X)
    Z = X.cpu().numpy()
    Zl = Z.astype(np.longdouble)
    assert float(np.max(np.abs(Zl.T @ Zl - np.eye(k)))) < 1e-13
    H = Zl.T @ (A.astype(np.longdouble) @ Zl)
    assert float(np.max(np.abs(H - np.diag(np.diag(H))))) < 1e-13
    assert np.all(np.diff(np.abs(np.diag(H).astype(float))) <= 1e-15)
    assert np.all(np.diag(Z[:k]) <= 0.0)
    Zo, theta = oracle.rayleigh_ritz(A, P.X0)
    for cl in (slice(0, 4), slice(4, 8)):
        Pg = Z[:, cl] @ Z[:, cl].T
        Po = Zo[:, cl] @ Zo[:, cl].T
        assert float(np.max(np.abs(Pg - Po))) < 1e-12
    st = ctx.run(X, 12)
    assert st.status in (rf.OK, rf.NOT_CONVERGED)
    ctx.close()

    def dist(Y):
        return float(np.max(np.abs(align_signs(Y, P.X_true) - P.X_true)))

    Xo = Zo
    for s in range(12):
        Xo = oracle.refine_step(A, Xo, norm_a=1.0, dd=True, rr_top=(s == 0)).X
    e0, eg, eo = dist(Z), dist(X.cpu().numpy()), dist(Xo)
    assert eg < 0.2 * e0, "distance %.3e after Rayleigh-Ritz, %.3e after 12 steps" % (e0, eg)
    assert abs(eg - eo) < 0.05 * eo, "GPU %.3e, oracle %.3e" % (eg, eo)


def test_rayleigh_ritz_rejects_dependent_columns():
    rf = _lib()
    P = synth.dense_spectrum(200, 6, 6400)
    X0 = np.array(P.X0)
    X0[:, 3] = X0[:, 2]
    ctx = rf.RefineContext(_dev(P.A), 6, norm_a=1.0)
    X = _dev(X0).clone()
    with pytest.raises(rf.RefineError) as ei:
        ctx.rayleigh_ritz(X)
    assert ei.value.status == rf.ERANK
    assert np.array_equal(X.cpu().numpy(), X0)
    # the context still steps afterwards
    X2 = _dev(P.X0).clone()
    assert ctx.step(X2).status == rf.OK
    ctx.close()


def test_batched_rayleigh_ritz_matches_oracle_per_problem():
    """Grouped launches over uneven problems (one of them with dependent
    columns, which alone reports REFINE_ERANK and keeps its X), then a step
    with the zero leading block, against the oracle problem by problem."""
    rf = _lib()
    shapes = [(130, 4), (257, 9), (511, 32), (200, 17), (129, 31)]
    probs = [synth.dense_spectrum(n, k, 6500 + i) for i, (n, k) in enumerate(shapes)]
    X0s = [np.array(p.X0) for p in probs]
    X0s[3][:, 5] = X0s[3][:, 4]
    b = rf.RefineBatch([_dev(p.A) for p in probs], [k for _, k in shapes], norm_a=1.0)
    Xs = [_dev(x).clone() for x in X0s]
    rc, st = b.rayleigh_ritz(Xs)
    assert rc == rf.ERANK and st == [0, 0, 0, rf.ERANK, 0]
    assert np.array_equal(Xs[3].cpu().numpy(), X0s[3])
    rc, per = b.run(Xs, 1)
    for i, ((n, k), p) in enumerate(zip(shapes, probs)):
        if i == 3:
            continue
        Zo, _ = oracle.rayleigh_ritz(p.A, X0s[i])
        r = oracle.refine_step(p.A, Zo, norm_a=1.0, rr_top=True)
        err = float(np.max(np.abs(align_signs(Xs[i].cpu().numpy(), r.X) - r.X)))
        assert err <= TOL, "problem %d: %.3e" % (i, err)
    b.close()
