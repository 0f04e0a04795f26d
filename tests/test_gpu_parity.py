"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every case feeds the same seeded inputs to librefine.so and to the oracle and
compares the iterates element by element after per-column sign alignment
(eigenvectors are defined up to sign), together with the step statistics.
Tolerance: max |X_gpu - X_oracle| <= 1e-13 (the accuracy target of the refined vectors),
for well-separated spectra where two correct FP64 implementations agree to a
few ulps of the vector entries (about u / (gap * sqrt(n))).
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


def _compare_steps(A_np, X0, steps, *, norm_a, mu=0.0, target="largest_abs", shift=0.0,
                   A_dev=None, csr=None, tol=TOL, dd=False, split=0, **opts):
    rf = _lib()
    A_host = oracle.Csr(csr.n, csr.row_ptr, csr.col_idx, csr.val) if csr is not None else A_np
    if csr is not None:
        Ad = rf.CsrMatrix(csr.n, _dev(csr.row_ptr), _dev(csr.col_idx), _dev(csr.val))
    else:
        Ad = A_dev if A_dev is not None else _dev(A_np)
    ctx = rf.RefineContext(Ad, X0.shape[1], target=target, shift=shift, norm_a=norm_a, **opts)
    info = ctx.info()
    assert info["mu"] == pytest.approx(mu, abs=1e-12)
    Xg = _dev(X0).clone()
    Xo = np.array(X0, copy=True)
    worst = 0.0
    for s in range(steps):
        st = ctx.step(Xg)
        assert st.status == rf.OK, rf.status_string(st.status)
        r = oracle.refine_step(A_host, Xo, mu=info["mu"], norm_a=norm_a, dd=dd, split=split,
                               normalize=opts.get("normalize", True))
        assert r.status == 0
        Xo = r.X
        got = Xg.cpu().numpy()
        err = float(np.max(np.abs(align_signs(got, Xo) - Xo)))
        worst = max(worst, err)
        assert err <= tol, "step %d: max |dX| = %.3e" % (s, err)
        assert st.corr_fro == pytest.approx(r.corr_fro, rel=1e-6, abs=1e-15)
        assert st.resid_rel == pytest.approx(r.resid_rel, rel=1e-6, abs=1e-15)
        assert st.iters == s + 1
    ctx.close()
    return worst, Xg.cpu().numpy()


def test_dense_n256_k8_five_steps():
    """Dense well-separated case (n = 256, k = 8, lam_i = i/256), 5 steps."""
    P = synth.dense_well_separated(256, 8)
    worst, X = _compare_steps(P.A, P.X0, 5, norm_a=P.norm_a)
    # and the iterate approaches the true eigenvectors
    assert np.max(np.abs(align_signs(X, P.X_true) - P.X_true)) < np.max(np.abs(P.X0 - P.X_true))


@pytest.mark.parametrize("n,k", [(1000, 13), (777, 5), (300, 1), (640, 64), (513, 17), (701, 37),
                                 (900, 99)])
def test_dense_ragged_shapes(n, k):
    """Ragged n (not a multiple of the 128-row tiles, odd leading dimension)
    and ragged k (not a multiple of 16), including k = 1; odd k above 32 takes
    the statistics after the update, whose partials (stride 5k) are then
    summed one slot per thread instead of in pairs."""
    lam = np.concatenate([np.linspace(0.01, 0.6, n - k), np.linspace(0.8, 1.0, k)])
    Q = synth.householder_q(n, n, 123 + n).numpy()
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    Xt = Q[:, ::-1][:, :k]
    _compare_steps(A, synth.fp32_round(Xt), 3, norm_a=1.0)


def test_dense_logspace_reduced():
    """The log-spaced spectrum (separation ratio 1.05) at n = 2048, k = 64."""
    P = synth.dense_logspace(2048, 64)
    _compare_steps(P.A, P.X0, 3, norm_a=P.norm_a)


def test_dense_shift_smallest():
    """Sec. 5.1: the k smallest eigenpairs through mu = Gershgorin upper bound."""
    n, k = 400, 6
    lam = np.concatenate([np.linspace(0.1, 0.35, k), np.linspace(1.0, 2.0, n - k)])
    Q = synth.householder_q(n, n, 77).numpy()
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    D = np.abs(A).sum(1) - np.abs(np.diag(A))
    mu = float(np.max(np.diag(A) + D))
    X0 = synth.fp32_round(Q[:, :k])
    _compare_steps(A, X0, 4, norm_a=2.0, mu=mu, target="smallest")


def test_csr_laplacian_16():
    """CSR path: 16^3 Laplacian with a random diagonal, k = 8 smallest through
    mu = sigma (Gershgorin upper bound)."""
    L = synth.laplacian3d(16, seed=synth.SEED_BASE + 4)
    X0 = synth.laplacian_start(L, 8, seed=5, noise=1e-6, exact=True)
    _compare_steps(None, X0, 3, norm_a=L.sigma, mu=L.sigma, target="smallest", csr=L)


def test_csr_laplacian_32_iid_diagonal_k32():
    """The sparse workload's parity size: the 32^3 Laplacian (n = 32768) with
    the iid U[0, 1) diagonal, the k = 32 smallest through mu = sigma, from
    shift-invert Lanczos vectors plus N(0, (1e-6)^2) noise; three steps."""
    L = synth.laplacian3d(32, seed=synth.SEED_BASE + 4)
    X0 = synth.laplacian_start(L, 32, seed=5, noise=1e-6, exact=True)
    _compare_steps(None, X0, 3, norm_a=L.sigma, mu=L.sigma, target="smallest", csr=L)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 6, 13, 20, 32, 64, 100, 128])
def test_csr_every_row_width(k):
    """CSR product widths: k picks the lanes per row (1 to 32); for odd k the
    per-column loads, for even k not a power of two the lanes whose second
    column pair lies past k (k = 2, 6, 20, 100).
    Separable Laplacian on a 12^3 grid (exact eigenvectors + 1e-6 noise)."""
    L, lam, Xt, X0 = synth.laplacian3d_separable(12, k)
    _compare_steps(None, X0, 2, norm_a=L.sigma, mu=L.sigma, target="smallest", csr=L)


@pytest.mark.parametrize("k,lanes", [(12, None), (5, "8"), (5, "32"), (8, "16")])
def test_csr_irregular_rows(k, lanes, monkeypatch):
    """Rows of 0 to ~2000 nonzeros: empty rows, rows longer than one gather
    round, and a chunk whose nonzeros exceed the block's LDS copy (read from
    memory instead).  The k largest |lambda| of a random sparse symmetric
    matrix, X0 = fl32 of its eigenvectors.  k <= 8 runs the row form (lanes
    over a row's nonzeros) with the lane count forced."""
    if lanes is not None:
        monkeypatch.setenv("REFINE_SPMM_L", lanes)
    n = 1500
    rng = np.random.default_rng(4242)
    M = np.zeros((n, n))
    for i in range(n):
        cols = rng.choice(n, size=int(rng.integers(0, 4)), replace=False)
        M[i, cols] = rng.standard_normal(len(cols))
    M[5, :] = 0.05 * rng.standard_normal(n)
    M = M + M.T
    M[np.arange(n), np.arange(n)] += np.linspace(0.0, 3.0, n)
    for e in (17, 300, 301):
        M[e, :] = 0.0
        M[:, e] = 0.0
    lam, V = np.linalg.eigh(M)
    order = np.argsort(-np.abs(lam))[:k]
    X0 = synth.fp32_round(V[:, order])
    rp = np.zeros(n + 1, dtype=np.int32)
    nz = M != 0.0
    rp[1:] = np.cumsum(nz.sum(1))
    ci = np.nonzero(nz)[1].astype(np.int32)
    val = M[nz]
    assert rp[256] - rp[0] > 2048 and rp[1] - rp[0] > 0 and rp[18] == rp[17]

    class Csr:
        pass

    C = Csr()
    C.n, C.row_ptr, C.col_idx, C.val = n, rp, ci, val
    norm = float(np.max(np.abs(M).sum(1)))
    _compare_steps(None, X0, 2, norm_a=norm, csr=C)


@pytest.mark.parametrize("m,bands,k,lanes", [
    (14, (2, 2, 1), 5, None), (14, (2, 2, 1), 5, "8"), (14, (2, 2, 1), 5, "32"),
    (13, (1, 1, 1), 3, None), (12, (3, 3, 3), 5, None), (12, (3, 3, 3), 8, "32"),
    (15, (2, 2, 1), 1, None), (14, (2, 2, 1), 6, "16")])
def test_csr_kron_banded(m, bands, k, lanes, monkeypatch):
    """The Kronecker-banded sparse workload (27 to 343-point stencils, the
    paper's 25-364 nonzeros per row), k largest |lambda| of an indefinite
    spectrum, through the row form of the CSR product (k <= 8) with its lane
    count chosen from the mean row length or forced."""
    if lanes is not None:
        monkeypatch.setenv("REFINE_SPMM_L", lanes)
    K, lam, Xt, X0 = synth.kron_banded(m=m, bands=bands, k=k)
    _compare_steps(None, X0, 3, norm_a=K.sigma, csr=K)


@pytest.mark.parametrize("k,pad,kron", [(20, 5, False), (20, 6, False), (32, 1, False), (32, 2, False),
                                        (3, 1, False), (5, 3, True), (5, 4, True)])
def test_csr_x_inside_wider_buffer(k, pad, kron):
    """X held inside a wider buffer (ldx = k + pad): an odd ldx leaves X rows
    without 16-byte alignment (single-double loads in the vector form), an
    even one keeps the paired loads at a stride other than k; the row form
    (Kronecker workload, k = 5) loads X rows as 8-byte-aligned pairs at any
    ldx.  The step touches only the (n, k) view."""
    rf = _lib()
    if kron:
        C, lam, Xt, X0 = synth.kron_banded(m=14, bands=(2, 2, 1), k=k)
        mu, target = 0.0, "largest_abs"
    else:
        C, lam, Xt, X0 = synth.laplacian3d_separable(12, k)
        mu, target = C.sigma, "smallest"
    Ad = rf.CsrMatrix(C.n, _dev(C.row_ptr), _dev(C.col_idx), _dev(C.val))
    Xbuf = torch.full((C.n, k + pad), 7.0, dtype=torch.float64, device="cuda")
    Xbuf[:, :k] = _dev(X0)
    X = Xbuf[:, :k]
    assert X.stride(0) == k + pad
    ctx = rf.RefineContext(Ad, k, target=target, norm_a=C.sigma)
    assert ctx.info()["mu"] == pytest.approx(mu, abs=1e-12)
    A_host = oracle.Csr(C.n, C.row_ptr, C.col_idx, C.val)
    Xo = np.array(X0, copy=True)
    for s in range(2):
        st = ctx.step(X)
        assert st.status == rf.OK, rf.status_string(st.status)
        r = oracle.refine_step(A_host, Xo, mu=mu, norm_a=C.sigma)
        Xo = r.X
        err = float(np.max(np.abs(align_signs(X.cpu().numpy(), Xo) - Xo)))
        assert err <= TOL, "step %d: max |dX| = %.3e" % (s, err)
    ctx.close()
    assert bool(torch.all(Xbuf[:, k:] == 7.0))


def test_new_iterate_starts_a_new_divergence_history():
    """Steps on one X, then a restart from the start block in another buffer:
    the first step of the restart has a larger correction than the last steps
    before it, which is no divergence (the history begins anew)."""
    rf = _lib()
    P = synth.dense_logspace(1024, 16)
    ctx = rf.RefineContext(_dev(P.A), 16, norm_a=P.norm_a)
    X = _dev(P.X0).clone()
    for _ in range(6):
        assert ctx.step(X).status == rf.OK
    X2 = _dev(P.X0).clone()
    for _ in range(3):
        st = ctx.step(X2)
        assert st.status == rf.OK, rf.status_string(st.status)
    ctx.close()


@pytest.mark.parametrize("k,pipe", [(5, "1"), (64, "0")])
def test_kxk_forms_single_problem(k, pipe, monkeypatch):
    """Both forms of the k x k stage for one problem: the panel pipeline
    forced at small k and the one-workgroup kernel forced at k = 64."""
    monkeypatch.setenv("REFINE_KXK_PIPE", pipe)
    P = synth.dense_logspace(1024, k)
    _compare_steps(P.A, P.X0, 3, norm_a=P.norm_a)


def test_refine_run_converges_and_counts():
    """refine_run with the correction-size stopping rule (Sec. 3.1.3)."""
    rf = _lib()
    P = synth.dense_well_separated(256, 8)
    ctx = rf.RefineContext(_dev(P.A), 8, norm_a=P.norm_a)
    X = _dev(P.X0)
    st = ctx.run(X, 500, stop="correction", tol=1e-12)
    assert st.status == rf.OK
    Xo, hist = oracle.refine(P.A, P.X0, st.iters, norm_a=P.norm_a)
    assert hist[-1].corr_fro <= 1e-12 < hist[-2].corr_fro
    err = np.max(np.abs(align_signs(X.cpu().numpy(), Xo) - Xo))
    assert err < 1e-12
    st2 = ctx.run(X, 3, stop="iters")
    assert st2.status == rf.OK and st2.iters == 3
    ctx.close()


def test_singular_y1_and_nonfinite_are_reported():
    rf = _lib()
    n, k = 64, 4
    A = np.diag(np.linspace(1.0, 2.0, n))
    ctx = rf.RefineContext(_dev(A), k, norm_a=2.0)
    X = torch.zeros((n, k), dtype=torch.float64, device="cuda")
    X[:k, :k] = torch.eye(k)
    X0 = X.clone()
    st = ctx.step(X)
    assert st.status == rf.EWY_SINGULAR
    assert torch.equal(X, X0)          # the rejected step leaves X unchanged
    Xn = _dev(synth.householder_q(n, n, 3).numpy()[:, :k]).contiguous()
    Xn[5, 2] = float("nan")
    st = ctx.step(Xn)
    assert st.status == rf.ENONFINITE
    ctx.close()


def test_error_of_an_unsynchronised_step_is_reported_not_reset():
    """A step enqueued without statistics that fails (a NaN in X) keeps its
    status; the next reporting call returns it instead of resetting it away:
    refine_run on the same X, refine_time_product, and a batch call after an
    unsynchronised batch run.  A good start then steps normally again."""
    rf = _lib()
    P = synth.dense_spectrum(200, 6, 9300)
    ctx = rf.RefineContext(_dev(P.A), 6, norm_a=1.0)
    X = _dev(P.X0).clone()
    X[7, 3] = float("nan")
    ctx.step(X, sync=False)
    ctx.step(X, sync=False)
    st = ctx.run(X, 3)
    assert st.status == rf.ENONFINITE
    ctx.step(X, sync=False)
    with pytest.raises(rf.RefineError) as ei:
        ctx.time_product(X, 2)
    assert ei.value.status == rf.ENONFINITE
    Xg = _dev(P.X0).clone()
    st = ctx.run(Xg, 3)
    assert st.status == rf.OK and st.iters == 3
    ctx.close()
    shapes = [(150, 4), (200, 6)]
    probs = [synth.dense_spectrum(n, k, 9310 + i) for i, (n, k) in enumerate(shapes)]
    b = rf.RefineBatch([_dev(p.A) for p in probs], [k for _, k in shapes], norm_a=1.0)
    Xs = [_dev(p.X0).clone() for p in probs]
    Xs[1][3, 2] = float("nan")
    b.run(Xs, 2, sync=False)
    with pytest.raises(rf.RefineError) as ei:
        b.time_product(2)
    assert ei.value.status == rf.ENONFINITE
    Xs[1] = _dev(probs[1].X0).clone()
    rc, per = b.run(Xs, 2)
    assert rc == rf.OK and [s.iters for s in per] == [2, 2]
    b.close()


@pytest.mark.parametrize("k", [8, 40])
def test_diverged_step_is_rejected_and_x_unchanged(k):
    """||E_L||_F >= 1 (a random orthonormal start) is reported as divergence
    and the rejected step leaves X unchanged, both where the statistics are
    formed before the update (k <= 32) and after it (k > 32)."""
    rf = _lib()
    P = synth.dense_spectrum(300, k, 9100 + k)
    rng = np.random.default_rng(5)
    q, r = np.linalg.qr(rng.standard_normal((300, k)))
    X0 = q * np.sign(np.diag(r))
    assert oracle.refine_step(P.A, X0, norm_a=1.0).corr_fro > 1.0
    ctx = rf.RefineContext(_dev(P.A), k, norm_a=1.0)
    X = _dev(X0).clone()
    st = ctx.step(X)
    assert st.status == rf.EDIVERGED
    assert np.array_equal(X.cpu().numpy(), X0)
    # the context recovers with a good start
    Xg = _dev(P.X0).clone()
    assert ctx.step(Xg).status == rf.OK
    ctx.close()


@pytest.mark.parametrize("k", [8, 40])
def test_normalization_off_matches_oracle(k):
    """normalize = 0 (Sec. 3.1.3 makes normalisation a choice): columns 0.1 %
    longer than unit length stay unnormalised, as in the oracle."""
    P = synth.dense_spectrum(300, k, 9200 + k)
    X0 = P.X0 * 1.001
    _compare_steps(P.A, X0, 3, norm_a=1.0, normalize=False)


def test_invalid_arguments():
    rf = _lib()
    A = _dev(np.eye(16))
    with pytest.raises(rf.RefineError) as e:
        rf.RefineContext(A, 16)
    assert e.value.status == rf.EINVAL
    with pytest.raises(rf.RefineError):
        rf.RefineContext(A, 0)


def test_batched_matches_oracle_per_problem():
    """Batched dense problems with uneven n and k (one grouped launch per
    kernel): every problem matches its own oracle run."""
    rf = _lib()
    shapes = [(130, 4), (257, 9), (511, 32), (200, 17), (129, 31), (384, 16)]
    probs = [synth.dense_spectrum(n, k, 900 + i) for i, (n, k) in enumerate(shapes)]
    As = [_dev(p.A) for p in probs]
    Xs = [_dev(p.X0).clone() for p in probs]
    b = rf.RefineBatch(As, [k for _, k in shapes], norm_a=1.0)
    rc, per = b.run(Xs, 3)
    assert rc == rf.OK
    for (n, k), p, X, s in zip(shapes, probs, Xs, per):
        Xo, hist = oracle.refine(p.A, p.X0, 3, norm_a=1.0)
        err = np.max(np.abs(align_signs(X.cpu().numpy(), Xo) - Xo))
        assert err <= TOL, "problem n=%d k=%d: max |dX| = %.3e" % (n, k, err)
        assert s.iters == 3
        assert s.corr_fro == pytest.approx(hist[-1].corr_fro, rel=1e-6)
    b.close()


def test_batched_multi_step_graph():
    """Seven batched steps: one five-step graph and two single-step graphs
    give the oracle's seven steps for every problem."""
    rf = _lib()
    shapes = [(300, 8), (150, 4), (420, 20)]
    probs = [synth.dense_spectrum(n, k, 950 + i) for i, (n, k) in enumerate(shapes)]
    b = rf.RefineBatch([_dev(p.A) for p in probs], [k for _, k in shapes], norm_a=1.0)
    Xs = [_dev(p.X0).clone() for p in probs]
    rc, per = b.run(Xs, 7)
    assert rc == rf.OK
    for p, X, s in zip(probs, Xs, per):
        Xo, hist = oracle.refine(p.A, p.X0, 7, norm_a=1.0)
        assert np.max(np.abs(align_signs(X.cpu().numpy(), Xo) - Xo)) <= TOL
        assert s.iters == 7
    b.close()


def test_step_is_deterministic():
    rf = _lib()
    P = synth.dense_logspace(1024, 32)
    outs = []
    for _ in range(2):
        ctx = rf.RefineContext(_dev(P.A), 32, norm_a=1.0)
        X = _dev(P.X0).clone()
        for _ in range(3):
            ctx.step(X)
        outs.append(X.cpu().numpy())
        ctx.close()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("cfg", list(range(8)))
def test_every_product_configuration(cfg, monkeypatch):
    """Every launch configuration of the dense product (the tuner may pick
    any of them) gives the oracle's step, on ragged shapes, with and without
    a K split."""
    for (n, k), ks in (((777, 13), 1), ((1000, 64), 2), ((1280, 33), 4)):
        monkeypatch.setenv("REFINE_GEMM", "%d,%d" % (cfg, ks))
        P = synth.dense_spectrum(n, k, 4000 + n)
        _compare_steps(P.A, P.X0, 1, norm_a=1.0)


@pytest.mark.parametrize("cfg", list(range(8)))
def test_batched_mixed_k_every_product_configuration(cfg, monkeypatch):
    """A batch whose largest k (72) sets five 16-column tiles for every
    problem, so most problems run with zero-padded X columns (k = 1 .. 49):
    every launch configuration gives each problem its own oracle steps."""
    rf = _lib()
    monkeypatch.setenv("REFINE_GEMM", "%d,1" % cfg)
    shapes = [(200, 5), (333, 48), (150, 49), (260, 72), (180, 16), (97, 1)]
    probs = [synth.dense_spectrum(n, k, 4500 + 7 * i + n) for i, (n, k) in enumerate(shapes)]
    b = rf.RefineBatch([_dev(p.A) for p in probs], [k for _, k in shapes], norm_a=1.0)
    Xs = [_dev(p.X0).clone() for p in probs]
    rc, per = b.run(Xs, 2)
    b.close()
    assert rc == rf.OK
    for (n, k), p, X in zip(shapes, probs, Xs):
        Xo, _ = oracle.refine(p.A, p.X0, 2, norm_a=1.0)
        err = np.max(np.abs(align_signs(X.cpu().numpy(), Xo) - Xo))
        assert err <= TOL, "cfg %d, problem n=%d k=%d: max |dX| = %.3e" % (cfg, n, k, err)


# --------------------------------------------------------------------------
# Split form of the product (INT8 slices on the matrix cores)
# --------------------------------------------------------------------------
def _split_product_check(P, n, k, slices, ks, monkeypatch, variant=0):
    """One split-mode step: the product W = A X of the step's input, read
    back as (W_hi, W_lo), equals the oracle's split product (exact binned
    digit products) up to the double-double rounding of the recombination.
    variant 0 stages the tiles through registers, 1 loads them straight
    into LDS, 2 through direct-to-LDS rings (A several chunks ahead)."""
    rf = _lib()
    monkeypatch.setenv("REFINE_SPLIT_KS", "%d,%d" % (ks, variant))
    ctx = rf.RefineContext(_dev(P.A), k, norm_a=1.0, precision="split_int8", slices=slices)
    X = _dev(P.X0).clone()
    st = ctx.step(X)
    assert st.status == rf.OK, rf.status_string(st.status)
    wh, wl = ctx.debug_product()
    ctx.close()
    oh, ol = oracle.matmul_split(P.A, P.X0, slices)
    d = (wh.cpu().numpy() - oh) + (wl.cpu().numpy() - ol)
    scale = np.max(np.abs(oh))
    err = float(np.max(np.abs(d)))
    assert err <= 2.0 ** -100 * scale, "n=%d k=%d s=%d ks=%d: |dW| = %.3e (max|W| %.3e)" % (
        n, k, slices, ks, err, scale)


@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("n,k,ks", [(777, 13, 1), (1000, 64, 2), (1280, 33, 4), (640, 128, 1),
                                    (300, 1, 1), (513, 96, 8), (150, 128, 1), (30, 5, 1)])
def test_split_product_matches_oracle(n, k, ks, variant, monkeypatch):
    """Ragged n (not a multiple of the 32-wide chunks or of the row blocks),
    every column-tile layout (k <= 32, 64, 96, 128), K splits 1-8 (K ranges
    down to two chunks, fewer than the ring's prefetch depth), the three
    tile-loading variants."""
    P = synth.dense_spectrum(n, k, 5000 + n)
    _split_product_check(P, n, k, 9, ks, monkeypatch, variant)


@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("slices", [7, 8, 10])
def test_split_product_other_slice_counts(slices, variant, monkeypatch):
    P = synth.dense_spectrum(700, 40, 5100 + slices)
    _split_product_check(P, 700, 40, slices, 2, monkeypatch, variant)


@pytest.mark.parametrize("n,k", [(777, 13), (640, 64), (513, 17)])
def test_split_steps_match_oracle(n, k):
    """Whole split-mode steps against the oracle's split-mode steps (the same
    product definition), and against its Dot2 steps."""
    P = synth.dense_spectrum(n, k, 5200 + n)
    worst, X = _compare_steps(P.A, P.X0, 3, norm_a=1.0, split=9, precision="split_int8")
    Xd, _ = oracle.refine(P.A, P.X0, 3, norm_a=1.0, dd=True)
    assert np.max(np.abs(align_signs(X, Xd) - Xd)) <= TOL


def test_split_uniform_top_reduced():
    """The uniform spectrum with 128 targets 1e-3 apart (n = 2048, k = 128):
    two split-mode steps against the double-double oracle."""
    P = synth.dense_uniform_top(2048, 128)
    worst, X = _compare_steps(P.A, P.X0, 2, norm_a=1.0, split=9, precision="split_int8")
    Xd, _ = oracle.refine(P.A, P.X0, 2, norm_a=1.0, dd=True)
    assert np.max(np.abs(align_signs(X, Xd) - Xd)) <= TOL


def test_split_invalid_arguments():
    rf = _lib()
    A = _dev(np.eye(64))
    for bad in (6, 11, -1):
        with pytest.raises(rf.RefineError) as e:
            rf.RefineContext(A, 4, precision="split_int8", slices=bad)
        assert e.value.status == rf.EINVAL
    L = synth.laplacian3d(4, seed=1)
    C = rf.CsrMatrix(L.n, _dev(L.row_ptr), _dev(L.col_idx), _dev(L.val))
    with pytest.raises(rf.RefineError) as e:
        rf.RefineContext(C, 4, precision="split_int8")
    assert e.value.status == rf.EINVAL


# --------------------------------------------------------------------------
# k-by-k stage: the panel pipeline (warm-started Newton-Schulz) and its
# one-workgroup fallback
# --------------------------------------------------------------------------
def _ctrl_fallback_flag(ctx):
    """Reads the control word's fallback flag (int32 after the fixed
    fields: 6 int32, 1 + 2 + 4 doubles)."""
    import ctypes
    rf = _lib()
    ptrs = (ctypes.c_void_p * 6)()
    assert rf.load_library().refine_debug_workspace(ctx._ctx, ptrs, 6) == 0
    torch.cuda.synchronize()
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    buf = (ctypes.c_int32 * 2)()
    off = 6 * 4 + 7 * 8
    assert hip.hipMemcpy(ctypes.addressof(buf), ptrs[5] + off, 8, 2) == 0
    return buf[0]


@pytest.mark.parametrize("n,k", [(1500, 128), (1100, 100), (900, 48)])
def test_kxk_panel_pipeline_steps(n, k, monkeypatch):
    """Several FP64 steps at k up to 128 through the panel pipeline (forced
    for k <= 48, where one workgroup is the default): the first step has no
    warm start and takes the one-workgroup solver, the later ones the
    pipeline; every step matches the oracle."""
    monkeypatch.setenv("REFINE_KXK_PIPE", "1")
    P = synth.dense_spectrum(n, k, 6000 + n)
    rf = _lib()
    ctx = rf.RefineContext(_dev(P.A), k, norm_a=1.0)
    Xg = _dev(P.X0).clone()
    Xo = np.array(P.X0, copy=True)
    flags = []
    for s in range(4):
        st = ctx.step(Xg)
        assert st.status == rf.OK
        flags.append(_ctrl_fallback_flag(ctx))
        r = oracle.refine_step(P.A, Xo, norm_a=1.0)
        Xo = r.X
        err = float(np.max(np.abs(align_signs(Xg.cpu().numpy(), Xo) - Xo)))
        assert err <= TOL, "step %d: %.3e" % (s, err)
        assert st.corr_fro == pytest.approx(r.corr_fro, rel=1e-6)
    ctx.close()
    assert flags[0] == 1 and flags[-1] == 0, flags


@pytest.mark.parametrize("fused", ["1", "0"])
@pytest.mark.parametrize("n,k,prec", [(1500, 128, "fp64"), (1100, 100, "split_crt"),
                                      (900, 64, "fp64"), (700, 53, "split_int8")])
def test_pipeline_update_orders_match_oracle(n, k, prec, fused, monkeypatch):
    """One problem through the k x k panel pipeline, with the statistics
    formed from k x k quadratic forms before an update that writes the
    normalised iterate (REFINE_FUSED_PIPE=1, the default) and in the order
    update, statistics, normalisation (0): both match the oracle's steps,
    and the step statistics agree with the oracle's."""
    monkeypatch.setenv("REFINE_FUSED_PIPE", fused)
    P = synth.dense_spectrum(n, k, 7100 + n)
    rf = _lib()
    ctx = rf.RefineContext(_dev(P.A), k, norm_a=1.0, precision=prec)
    form = {"fp64": {}, "split_int8": {"split": 9}, "split_crt": {"crt": 16}}[prec]
    Xg = _dev(P.X0).clone()
    Xo = np.array(P.X0, copy=True)
    for s in range(3):
        st = ctx.step(Xg)
        assert st.status == rf.OK
        r = oracle.refine_step(P.A, Xo, norm_a=1.0, **form)
        Xo = r.X
        err = float(np.max(np.abs(align_signs(Xg.cpu().numpy(), Xo) - Xo)))
        assert err <= TOL, "step %d: %.3e" % (s, err)
        assert st.corr_fro == pytest.approx(r.corr_fro, rel=1e-6)
    ctx.close()


@pytest.mark.parametrize("variant", [None, 2])
def test_split_batched_matches_oracle_per_problem(variant, monkeypatch):
    """Batched split-mode steps (uneven n and k, one grouped launch per
    kernel): every problem matches the oracle's split-mode steps (the tuned
    tile-loading variant, and the ring variant forced)."""
    rf = _lib()
    if variant is not None:
        monkeypatch.setenv("REFINE_SPLIT_KS", "1,%d" % variant)
    shapes = [(130, 4), (257, 9), (511, 32), (200, 17), (129, 31)]
    probs = [synth.dense_spectrum(n, k, 970 + i) for i, (n, k) in enumerate(shapes)]
    b = rf.RefineBatch([_dev(p.A) for p in probs], [k for _, k in shapes], norm_a=1.0,
                       precision="split_int8")
    Xs = [_dev(p.X0).clone() for p in probs]
    rc, per = b.run(Xs, 6)
    assert rc == rf.OK
    for (n, k), p, X, s in zip(shapes, probs, Xs, per):
        Xo, hist = oracle.refine(p.A, p.X0, 6, norm_a=1.0, split=9)
        err = np.max(np.abs(align_signs(X.cpu().numpy(), Xo) - Xo))
        assert err <= TOL, "problem n=%d k=%d: max |dX| = %.3e" % (n, k, err)
        assert s.iters == 6
    b.close()


def test_split_batched_clusters_reach_double_double_accuracy():
    """Two target clusters with internal gaps of 1e-6 (the batched workload's
    spectrum): after 30 steps the split form with 10 slices (W within about
    2^-70 of the row and column scales) matches the Dot2 oracle to 1e-13, the
    FP64 form only to about u / gap."""
    rf = _lib()
    shapes = [(256, 8), (300, 6)]
    probs = [synth.dense_clustered(n, k, 990 + i) for i, (n, k) in enumerate(shapes)]
    res = {}
    for prec in ("fp64", "split_int8"):
        b = rf.RefineBatch([_dev(p.A) for p in probs], [k for _, k in shapes], norm_a=1.0,
                           precision=prec, slices=10 if prec == "split_int8" else 0)
        Xs = [_dev(p.X0).clone() for p in probs]
        rc, _ = b.run(Xs, 30)
        assert rc == rf.OK
        res[prec] = [X.cpu().numpy() for X in Xs]
        b.close()
    for i, p in enumerate(probs):
        Xd, _ = oracle.refine(p.A, p.X0, 30, norm_a=1.0, dd=True)
        es = np.max(np.abs(align_signs(res["split_int8"][i], Xd) - Xd))
        ef = np.max(np.abs(align_signs(res["fp64"][i], Xd) - Xd))
        print("problem %d: split %.3e, fp64 %.3e" % (i, es, ef))
        assert es <= TOL, "split: %.3e (fp64 %.3e)" % (es, ef)
        assert es < ef


def test_split_residual_keeps_the_low_part_on_clusters():
    """One split-mode step on a spectrum with clusters of gap 1e-6: the
    correction divides residual inner products of about 1e-17 by the gap, so
    the step matches the oracle's split step only if R = (W_hi - x d) + W_lo
    is formed with an exact product (no fused multiply-add folding x d into
    the subtraction)."""
    rf = _lib()
    p = synth.dense_clustered(256, 8, 990)
    ctx = rf.RefineContext(_dev(p.A), 8, norm_a=1.0, precision="split_int8", slices=10)
    X = _dev(p.X0).clone()
    Xo = np.array(p.X0, copy=True)
    for s in range(4):
        Xin = X.cpu().numpy()
        assert ctx.step(X).status == rf.OK
        r = oracle.refine_step(p.A, Xin, norm_a=1.0, split=10)
        err = float(np.max(np.abs(align_signs(X.cpu().numpy(), r.X) - r.X)))
        assert err <= 1e-14, "step %d: %.3e" % (s, err)
    ctx.close()
