"""Argument checks of the C ABI that run on the host before any device work,
as include/refine.h states them: 1 <= k <= 128, k < n, n < 2^31, lda >= n,
non-null matrix pointers, CSR nnz in [0, 2^31) and FP64 only, split mode with
n <= 65536 and 7..10 slices, delta_c >= 0, a known target, the squared
variant in FP64 only, and a null context or batch handle.  Every case below
returns REFINE_EINVAL, so the library makes no HIP call and dereferences no
pointer.  The matrix pointers are placeholders: the module is skipped where
a GPU is visible, so a case that the checks let through could never reach a
kernel."""
import ctypes

import pytest

PH = 0x100000  # placeholder device address (never dereferenced in these cases)


@pytest.fixture(scope="module")
def rf():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("host-only argument checks with placeholder pointers")
    import paper_2602_23778_amd as m
    m.load_library()
    return m


def _dense(rf, n=100, lda=None, a=PH):
    m = rf.refine_matrix()
    m.kind, m.n, m.a, m.lda = rf.DENSE, n, a, n if lda is None else lda
    return m


def _csr(rf, n=100, nnz=500, rp=PH, ci=PH, val=PH):
    m = rf.refine_matrix()
    m.kind, m.n, m.row_ptr, m.col_idx, m.val, m.nnz = rf.CSR, n, rp, ci, val, nnz
    return m


def _opt(rf, **kw):
    o = rf.refine_options()
    rf.refine_options_default(o)
    for key, v in kw.items():
        setattr(o, key, v)
    return o


_INIT_CASES = {
    "n = 0": (lambda rf: _dense(rf, n=0), 1, {}),
    "n < 0": (lambda rf: _dense(rf, n=-5, lda=5), 1, {}),
    "n = 2^31": (lambda rf: _dense(rf, n=1 << 31), 4, {}),
    "k = 0": (lambda rf: _dense(rf), 0, {}),
    "k < 0": (lambda rf: _dense(rf), -3, {}),
    "k = 129": (lambda rf: _dense(rf, n=1000), 129, {}),
    "k = n": (lambda rf: _dense(rf, n=100), 100, {}),
    "dense a = NULL": (lambda rf: _dense(rf, a=None), 4, {}),
    "lda < n": (lambda rf: _dense(rf, lda=99), 4, {}),
    "unknown kind": (lambda rf: _dense(rf), 4, {"kind": 2}),
    "CSR row_ptr = NULL": (lambda rf: _csr(rf, rp=None), 4, {}),
    "CSR col_idx = NULL": (lambda rf: _csr(rf, ci=None), 4, {}),
    "CSR val = NULL": (lambda rf: _csr(rf, val=None), 4, {}),
    "CSR nnz < 0": (lambda rf: _csr(rf, nnz=-1), 4, {}),
    "CSR nnz = 2^31": (lambda rf: _csr(rf, nnz=1 << 31), 4, {}),
    "CSR in split mode": (lambda rf: _csr(rf), 4, {"precision": 1}),
    "unknown precision 2": (lambda rf: _dense(rf), 4, {"precision": 2}),
    "unknown precision -1": (lambda rf: _dense(rf), 4, {"precision": -1}),
    "split, 6 slices": (lambda rf: _dense(rf), 4, {"precision": 1, "slices": 6}),
    "split, 11 slices": (lambda rf: _dense(rf), 4, {"precision": 1, "slices": 11}),
    "split, n = 65537": (lambda rf: _dense(rf, n=65537), 4, {"precision": 1}),
    "delta_c < 0": (lambda rf: _dense(rf), 4, {"delta_c": -1.0}),
    "delta_c NaN": (lambda rf: _dense(rf), 4, {"delta_c": float("nan")}),
    "target -1": (lambda rf: _dense(rf), 4, {"target": -1}),
    "target 5": (lambda rf: _dense(rf), 4, {"target": 5}),
    "smallest |lambda| in split mode": (lambda rf: _dense(rf), 4, {"target": 4, "precision": 1}),
}


@pytest.mark.parametrize("case", list(_INIT_CASES))
def test_init_rejects(rf, case):
    make, k, fields = _INIT_CASES[case]
    A = make(rf)
    if "kind" in fields:
        A.kind = fields["kind"]
    opt = _opt(rf, **{f: v for f, v in fields.items() if f != "kind"})
    ctx = ctypes.c_void_p()
    assert rf.refine_init(ctx, A, k, opt, None) == rf.EINVAL
    assert ctx.value is None
    # the same matrix as the only member of a batch (dense members only)
    b = ctypes.c_void_p()
    As = (rf.refine_matrix * 1)(A)
    ks = (ctypes.c_int32 * 1)(k)
    assert rf.refine_batch_init(b, 1, As, ks, opt, None) == rf.EINVAL
    assert b.value is None


def test_init_rejects_null_arguments(rf):
    lib = rf.load_library()
    A = _dense(rf)
    ctx = ctypes.c_void_p()
    assert lib.refine_init(None, ctypes.byref(A), 4, None, None) == rf.EINVAL
    assert lib.refine_init(ctypes.byref(ctx), None, 4, None, None) == rf.EINVAL
    assert ctx.value is None


def test_batch_init_rejects(rf):
    lib = rf.load_library()
    good = _dense(rf, n=300)
    b = ctypes.c_void_p()
    As = (rf.refine_matrix * 3)(good, good, _dense(rf, n=50))
    ks = (ctypes.c_int32 * 3)(4, 8, 50)  # the third has k = n
    assert rf.refine_batch_init(b, 3, As, ks, None, None) == rf.EINVAL
    As2 = (rf.refine_matrix * 2)(good, _csr(rf, n=300))  # batches take dense problems
    ks2 = (ctypes.c_int32 * 2)(4, 4)
    assert rf.refine_batch_init(b, 2, As2, ks2, None, None) == rf.EINVAL
    assert rf.refine_batch_init(b, 0, As2, ks2, None, None) == rf.EINVAL
    assert rf.refine_batch_init(b, -1, As2, ks2, None, None) == rf.EINVAL
    assert lib.refine_batch_init(ctypes.byref(b), 2, None, ks2, None, None) == rf.EINVAL
    assert lib.refine_batch_init(ctypes.byref(b), 2, As2, None, None, None) == rf.EINVAL
    assert lib.refine_batch_init(None, 2, As2, ks2, None, None) == rf.EINVAL
    assert b.value is None


def test_null_handles(rf):
    st = rf.refine_stats()
    assert rf.refine_step(None, PH, 4, st) == rf.EINVAL
    assert rf.refine_run(None, PH, 4, 5, rf.STOPS["iters"], 0.0, st) == rf.EINVAL
    assert rf.refine_rayleigh_ritz(None, PH, 4) == rf.EINVAL
    assert rf.refine_sign_flip(None, PH, 4, None) == rf.EINVAL
    assert rf.refine_get_info(None)[0] == rf.EINVAL
    assert rf.refine_time_product(None, PH, 4, 3)[0] == rf.EINVAL
    assert rf.refine_destroy(None) == rf.EINVAL
    assert rf.refine_batch_run(None, None, None, 1, None) == rf.EINVAL
    assert rf.refine_batch_rayleigh_ritz(None, None, None, None) == rf.EINVAL
    assert rf.refine_batch_sign_flip(None, None, None, None) == rf.EINVAL
    assert rf.refine_batch_time_product(None, 2)[0] == rf.EINVAL
    assert rf.refine_batch_destroy(None) == rf.EINVAL


def test_option_defaults_and_status_strings(rf):
    o = rf.refine_options()
    rf.refine_options_default(o)
    assert (o.precision, o.target, o.beta, o.normalize, o.slices) == (rf.FP64, 0, 0, 1, 0)
    assert o.delta_c == 10.0 and o.shift == 0.0 and o.norm_a <= 0.0
    codes = (rf.OK, rf.NOT_CONVERGED, rf.EINVAL, rf.ENOMEM, rf.EHIP, rf.EWY_SINGULAR,
             rf.EDIVERGED, rf.ENONFINITE, rf.ERANK)
    texts = [rf.refine_status_string(c) for c in codes]
    assert len(set(texts)) == len(codes)
    assert "unknown" not in " ".join(texts)
    assert rf.refine_status_string(12345) == "unknown status"
