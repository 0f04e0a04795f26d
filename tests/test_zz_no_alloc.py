"""The entry point that allocates nothing (refine_step_static): one step with
all of its device memory beyond A and X in the library's static per-GPU
array, against refine_step on a context (the existing entry point) on the
same input, two calls in a row with the second on a smaller problem (the
array keeps the first call's contents, which the second must not see)."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from tests._util import align_signs

pytestmark = pytest.mark.gpu

TOL = 1e-13


def _lib():
    import paper_2602_23778_amd as rf
    rf.load_library()
    return rf


def _static_step(rf, A, X, k, norm_a, **opts):
    return rf.step_static(A, X, k, norm_a=norm_a, **opts)


def _case(rf, n, k, seed):
    print("case: refine_step_static n=%d k=%d" % (n, k), flush=True)
    P = synth.dense_spectrum(n, k, seed)
    A = torch.as_tensor(P.A).cuda()
    X0 = torch.as_tensor(P.X0).cuda()
    Xs = X0.clone()
    rc, st = _static_step(rf, A, Xs, k, 1.0)
    assert rc == rf.OK and st.status == rf.OK and st.iters == 1, rf.status_string(rc)
    ctx = rf.RefineContext(A, k, norm_a=1.0)
    Xc = X0.clone()
    sc = ctx.step(Xc)
    ctx.close()
    assert sc.status == rf.OK
    a, b = Xs.cpu().numpy(), Xc.cpu().numpy()
    err = float(np.max(np.abs(align_signs(a, b) - b)))
    print("  max |dX| against refine_step: %.3e" % err, flush=True)
    assert err <= TOL
    assert st.corr_fro == pytest.approx(sc.corr_fro, rel=1e-9)
    assert st.resid_rel == pytest.approx(sc.resid_rel, rel=1e-9)


def test_static_step_matches_refine_step_twice():
    rf = _lib()
    _case(rf, 3000, 64, 7100)     # unfused tail, k x k panel pipeline
    _case(rf, 700, 16, 7101)      # smaller: fused tail, one-workgroup k x k stage


def test_static_step_rejects_what_it_cannot_hold():
    rf = _lib()
    A = torch.eye(64, dtype=torch.float64, device="cuda")
    X = torch.zeros(64, 4, dtype=torch.float64, device="cuda")
    rc, _ = _static_step(rf, A, X, 4, 0.0)                 # norm_a must be given
    assert rc == rf.EINVAL
    rc, _ = _static_step(rf, A, X, 4, 1.0, target="smallest")
    assert rc == rf.EINVAL
    rc, _ = _static_step(rf, A, X, 4, 1.0, precision="split_crt")
    assert rc == rf.EINVAL
    # a workspace far beyond the array is rejected on the host, before any
    # device access (the 1-element buffers are never read)
    big = torch.zeros(1, dtype=torch.float64, device="cuda")
    m_n = 1 << 20
    m = rf.refine_matrix()
    m.kind, m.n, m.a, m.lda = rf.DENSE, m_n, big.data_ptr(), m_n
    o = rf.make_options(norm_a=1.0)
    st = rf.refine_stats()
    rc = rf.load_library().refine_step_static(ctypes.byref(m), 128, ctypes.byref(o),
                                              big.data_ptr(), 128, None, ctypes.byref(st))
    assert rc == rf.EINVAL
