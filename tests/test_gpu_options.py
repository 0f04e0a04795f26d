"""Options and layouts of the C ABI on the GPU against the oracle: the
targets "largest" (mu = Gershgorin lower bound) and "shift" (mu given;
Sec. 5.1), beta = 0 and a caller's delta constant for close Rayleigh
quotients (the diagonal-block rule of eq. E_L), the residual stopping rule,
a caller's HIP stream, and A and X held inside wider buffers (lda > n,
ldx > k).  Tolerance as in the other parity tests: max |X_gpu - X_oracle|
<= 1e-13 after sign alignment."""
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


def _err(g, o):
    return float(np.max(np.abs(align_signs(g, o) - o)))


def _spectral(lam, seed):
    """A = Q diag(lam) Q^T with a seeded Householder Q; returns (A, Q)."""
    n = len(lam)
    Q = synth.householder_q(n, n, seed).numpy()
    A = (Q * lam) @ Q.T
    return 0.5 * (A + A.T), Q


def _steps(rf, A_dev, A_host, X0, steps, *, norm_a, mu_expect=None, X_dev=None, corr_abs=1e-15,
           **opts):
    ctx = rf.RefineContext(A_dev, X0.shape[1], norm_a=norm_a, **opts)
    mu = ctx.info()["mu"]
    if mu_expect is not None:
        assert mu == pytest.approx(mu_expect, rel=1e-13, abs=1e-15)
    X = X_dev if X_dev is not None else _dev(X0).clone()
    Xo = np.array(X0, copy=True)
    okw = {"delta_c": opts.get("delta_c", 10.0), "beta_zero": opts.get("beta", "") == "zero"}
    for s in range(steps):
        st = ctx.step(X)
        assert st.status == rf.OK, rf.status_string(st.status)
        r = oracle.refine_step(A_host, Xo, mu=mu, norm_a=norm_a, **okw)
        assert r.status == oracle.OK
        Xo = r.X
        err = _err(X.cpu().numpy(), Xo)
        assert err <= TOL, "step %d: %.3e" % (s, err)
        assert st.corr_fro == pytest.approx(r.corr_fro, rel=1e-6, abs=corr_abs)
    ctx.close()
    return X


def test_target_largest_uses_the_gershgorin_lower_bound():
    """The k largest eigenvalues of an indefinite A whose largest |lambda|
    are negative: mu is the Gershgorin lower bound, so the targets are the
    eigenvalues farthest above it."""
    rf = _lib()
    n, k = 400, 6
    lam = np.concatenate([np.linspace(0.9, 1.0, k), np.linspace(-2.0, 0.5, n - k)])
    A, Q = _spectral(lam, 301)
    lo = float(np.min(np.diag(A) - (np.abs(A).sum(1) - np.abs(np.diag(A)))))
    assert lo < -2.0
    X0 = synth.fp32_round(Q[:, :k])
    _steps(rf, _dev(A), A, X0, 3, norm_a=2.0, mu_expect=lo, target="largest")


def test_target_shift_takes_both_ends_of_the_spectrum():
    """A given shift inside the spectrum: the targets are the eigenvalues
    farthest from it on both sides, so d - mu has both signs in the bottom
    rows' denominators."""
    rf = _lib()
    n, k, mu = 360, 6, 0.45
    lam = np.concatenate([np.linspace(0.0, 0.02, 3), np.linspace(0.98, 1.0, 3),
                          np.linspace(0.3, 0.6, n - k)])
    A, Q = _spectral(lam, 302)
    X0 = synth.fp32_round(Q[:, :k])
    _steps(rf, _dev(A), A, X0, 3, norm_a=1.0, mu_expect=mu, target="shift", shift=mu)


@pytest.mark.parametrize("beta", ["half_gram", "zero"])
def test_close_pair_takes_the_diagonal_block_rule(beta):
    """Two targets 1e-9 apart with delta = c ||A|| u raised to about 1e-7 by
    the caller's constant c = 1e9: that pair's off-diagonal entries use beta
    (-x_i^T x_j / 2, or 0) instead of dividing by the gap."""
    rf = _lib()
    n, k, c = 300, 5, 1e9
    lam = np.concatenate([[1.0, 1.0 - 1e-9, 0.95, 0.9, 0.85], np.linspace(0.0, 0.7, n - k)])
    A, Q = _spectral(lam, 303)
    X0 = synth.fp32_round(Q[:, :k])
    ctx = rf.RefineContext(_dev(A), k, norm_a=1.0, delta_c=c)
    assert ctx.info()["delta"] == pytest.approx(c * 2.0 ** -53, rel=1e-12)
    ctx.close()
    _steps(rf, _dev(A), A, X0, 3, norm_a=1.0, delta_c=c, beta=beta)


@pytest.mark.parametrize("k", [24, 40, 80])
def test_close_group_across_column_tiles(k):
    """Four targets 1e-9 apart at columns 14-17 (and 30-33 from k = 40 on),
    across the 16-column tiles of the Gram pass, with delta raised to about
    1e-7: those pairs take -x_i^T x_j / 2, which needs X^T X in full, the
    leading rows' part of the tiles below the diagonal included (k = 24: the
    one-wavefront Gram pass; 40: the per-tile Gram pass; 80: that and the
    panel pipeline of the k x k stage)."""
    rf = _lib()
    n, c = 400, 1e9
    top = np.linspace(1.0, 0.85, k)
    for g0 in (14, 30):
        if g0 + 4 <= k:
            top[g0:g0 + 4] = top[g0] - 1e-9 * np.arange(4)
    lam = np.concatenate([top, np.linspace(0.0, 0.7, n - k)])
    A, Q = _spectral(lam, 304 + k)
    X0 = synth.fp32_round(Q[:, :k])
    _steps(rf, _dev(A), A, X0, 3, norm_a=1.0, delta_c=c)


def test_residual_stopping_rule():
    """refine_run stops at the first step whose input has ||R||_F / ||A||
    <= tol; the tolerance is the geometric mean of two of the oracle's
    successive residuals at least 10 % apart (the GPU's agree with them to
    about 1e-6), so the step count is fixed."""
    rf = _lib()
    P = synth.dense_well_separated(256, 8)
    _, hist = oracle.refine(P.A, P.X0, 12, norm_a=P.norm_a)
    res = [h.resid_rel for h in hist]
    stop_at = next(i for i in range(2, len(res)) if res[i] < 0.9 * res[i - 1])
    tol = float(np.sqrt(res[stop_at] * res[stop_at - 1]))
    ctx = rf.RefineContext(_dev(P.A), 8, norm_a=P.norm_a)
    X = _dev(P.X0).clone()
    st = ctx.run(X, 50, stop="residual", tol=tol)
    ctx.close()
    assert st.status == rf.OK
    assert st.iters == stop_at + 1
    Xo, _ = oracle.refine(P.A, P.X0, stop_at + 1, norm_a=P.norm_a)
    assert _err(X.cpu().numpy(), Xo) <= TOL


def test_steps_on_a_callers_stream():
    """A context bound to a stream of the caller's: steps enqueued without a
    host sync, then the stream is synchronised."""
    rf = _lib()
    P = synth.dense_spectrum(500, 12, 304)
    s = torch.cuda.Stream()
    A = _dev(P.A)
    X = _dev(P.X0).clone()
    torch.cuda.synchronize()
    ctx = rf.RefineContext(A, 12, stream=s, norm_a=1.0)
    for _ in range(3):
        ctx.step(X, sync=False)
    s.synchronize()
    ctx.close()
    Xo, _ = oracle.refine(P.A, P.X0, 3, norm_a=1.0)
    assert _err(X.cpu().numpy(), Xo) <= TOL


@pytest.mark.parametrize("k", [12, 40])
def test_a_and_x_inside_wider_buffers(k):
    """lda = n + 37 (odd, so A rows are not 16-byte aligned) and ldx = k + 5:
    the step reads and writes only the (n, k) view, for the statistics
    formed before the update (k <= 32) and after it (k > 32)."""
    rf = _lib()
    n = 600
    P = synth.dense_spectrum(n, k, 305 + k)
    Abuf = torch.full((n, n + 37), 3.0, dtype=torch.float64, device="cuda")
    Abuf[:, :n] = _dev(P.A)
    Xbuf = torch.full((n, k + 5), 7.0, dtype=torch.float64, device="cuda")
    Xbuf[:, :k] = _dev(P.X0)
    A = Abuf[:, :n]
    X = Xbuf[:, :k]
    assert A.stride(0) == n + 37 and X.stride(0) == k + 5
    _steps(rf, A, P.A, P.X0, 3, norm_a=1.0, X_dev=X)
    assert bool(torch.all(Xbuf[:, k:] == 7.0))
    assert bool(torch.all(Abuf[:, n:] == 3.0))


@pytest.mark.parametrize("k", [8, 16, 40, 64, 128])
def test_one_bottom_row(k):
    """n = k + 1: a single row below the leading k x k block, for the k x k
    stage in one workgroup (k <= 48) and in the panel pipeline (k = 64, 128),
    with the statistics before (k <= 32) or after the update."""
    rf = _lib()
    n = k + 1
    P = synth.dense_spectrum(n, k, 400 + k)
    _steps(rf, _dev(P.A), P.A, P.X0, 2, norm_a=1.0)


@pytest.mark.parametrize("k", [8, 40])
def test_exact_start_is_a_fixed_point(k):
    """X = Q's columns for the targets: R is rounding noise and the steps
    move X only by the distance between Q and the eigenvectors of the
    rounded A (about u / gap), where the oracle moves it.  ||E_L||_F is then
    rounding noise itself (1e-14 to 1e-12 here), so the two sides' values
    are held to that level rather than to each other's digits."""
    rf = _lib()
    n = 300
    lam = np.concatenate([np.linspace(0.9, 1.0, k)[::-1], np.linspace(0.0, 0.8, n - k)])
    A, Q = _spectral(lam, 410 + k)
    X0 = np.ascontiguousarray(Q[:, :k])
    X = _steps(rf, _dev(A), A, X0, 2, norm_a=1.0, corr_abs=1e-11)
    gap = 0.1 / (k - 1)
    assert float(np.max(np.abs(X.cpu().numpy() - X0))) < 16 * 2.0 ** -53 / gap


@pytest.mark.parametrize("n,k", [(9, 8), (65, 64), (500, 20)])
def test_split_form_shifted_in_wider_buffers(n, k):
    """The split form (INT8 slices of A and X, nine each) on the smallest
    eigenvalues through mu = the Gershgorin upper bound, with A and X inside
    wider buffers (lda = n + 37, ldx = k + 5) and down to one bottom row,
    against the oracle's split-mode steps (the same product definition)."""
    rf = _lib()
    lam = np.concatenate([np.linspace(0.0, 0.1, k), np.linspace(0.2, 1.0, n - k)])
    A, Q = _spectral(lam, 420 + n)
    hi = float(np.max(np.diag(A) + (np.abs(A).sum(1) - np.abs(np.diag(A)))))
    X0 = synth.fp32_round(Q[:, :k])
    Abuf = torch.full((n, n + 37), 3.0, dtype=torch.float64, device="cuda")
    Abuf[:, :n] = _dev(A)
    Xbuf = torch.full((n, k + 5), 7.0, dtype=torch.float64, device="cuda")
    Xbuf[:, :k] = _dev(X0)
    X = Xbuf[:, :k]
    ctx = rf.RefineContext(Abuf[:, :n], k, norm_a=1.0, target="smallest", precision="split_int8",
                           slices=9)
    mu = ctx.info()["mu"]
    assert mu == pytest.approx(hi, rel=1e-13)
    Xo = X0
    for s in range(2):
        st = ctx.step(X)
        assert st.status == rf.OK, rf.status_string(st.status)
        r = oracle.refine_step(A, Xo, mu=mu, norm_a=1.0, split=9)
        assert r.status == oracle.OK
        Xo = r.X
        err = _err(X.cpu().numpy(), Xo)
        assert err <= TOL, "step %d: %.3e" % (s, err)
    ctx.close()
    assert bool(torch.all(Xbuf[:, k:] == 7.0))
