"""Python binding of librefine.so, the MI355X (gfx950) library for iterative
refinement of a subset of eigenvectors of a real symmetric matrix (Terao,
Ozaki, Imamura and Ogita, arXiv 2602.23778; Algorithm 4 with Algorithm 1).

This module only marshals arguments: every step of the refinement runs in the
library's HIP kernels.  PyTorch provides device memory and streams.  The
functions named like the C ABI (refine_init, refine_step, refine_run,
refine_destroy, refine_batch_init, refine_batch_run, refine_batch_destroy,
refine_status_string, refine_get_info) take the same arguments as their C
counterparts; RefineContext and RefineBatch wrap them for torch tensors.

There is no CPU fallback: importing the binding without the built library,
or calling it without a GPU, raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch  # loads the HIP runtime that librefine.so then shares

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librefine.so")

# status codes (include/refine.h)
OK = 0
NOT_CONVERGED = 1
EINVAL = -1
ENOMEM = -2
EHIP = -3
EWY_SINGULAR = -4
EDIVERGED = -5
ENONFINITE = -6
ERANK = -7

DENSE, CSR = 0, 1
FP64, SPLIT_INT8, SPLIT_FP8, SPLIT_CRT = 0, 1, 2, 3
TARGETS = {"largest_abs": 0, "smallest": 1, "largest": 2, "shift": 3, "smallest_abs": 4}
BETAS = {"half_gram": 0, "zero": 1}
STOPS = {"iters": 0, "correction": 1, "residual": 2}


class refine_matrix(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("n", ctypes.c_int64), ("a", ctypes.c_void_p),
                ("lda", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p), ("nnz", ctypes.c_int64)]


class refine_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("target", ctypes.c_int), ("shift", ctypes.c_double),
                ("delta_c", ctypes.c_double), ("norm_a", ctypes.c_double), ("beta", ctypes.c_int),
                ("normalize", ctypes.c_int32), ("slices", ctypes.c_int32)]


class refine_stats(ctypes.Structure):
    _fields_ = [("corr_fro", ctypes.c_double), ("resid_rel", ctypes.c_double),
                ("iters", ctypes.c_int32), ("status", ctypes.c_int32)]


EXPORTS = ("refine_options_default", "refine_init", "refine_step", "refine_run",
           "refine_get_info", "refine_destroy", "refine_batch_init", "refine_batch_run",
           "refine_batch_destroy", "refine_status_string", "refine_time_product",
           "refine_batch_time_product", "refine_rayleigh_ritz", "refine_batch_rayleigh_ritz",
           "refine_sign_flip", "refine_batch_sign_flip", "refine_time_product_parts",
           "refine_step_static")

_lib = None


class RefineError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__("%s: %s (status %d)" % (what or "refine", status_string(status), status))


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads librefine.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("librefine.so not found at %s; build it with "
                          "`python -m paper_2602_23778_amd.build`" % path)
    lib = ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    lib.refine_options_default.argtypes = [P(refine_options)]
    lib.refine_options_default.restype = None
    lib.refine_init.argtypes = [P(vp), P(refine_matrix), i32, P(refine_options), vp]
    lib.refine_step.argtypes = [vp, vp, i64, P(refine_stats)]
    lib.refine_run.argtypes = [vp, vp, i64, i32, ctypes.c_int, dbl, P(refine_stats)]
    lib.refine_get_info.argtypes = [vp, P(dbl), P(dbl), P(dbl), P(dbl)]
    lib.refine_destroy.argtypes = [vp]
    lib.refine_batch_init.argtypes = [P(vp), i32, P(refine_matrix), P(i32), P(refine_options), vp]
    lib.refine_batch_run.argtypes = [vp, P(vp), P(i64), i32, P(refine_stats)]
    lib.refine_batch_destroy.argtypes = [vp]
    lib.refine_time_product.argtypes = [vp, vp, i64, i32, P(ctypes.c_float)]
    lib.refine_time_product_parts.argtypes = [vp, vp, i64, i32, P(ctypes.c_float), i32, P(i32)]
    lib.refine_step_static.argtypes = [P(refine_matrix), i32, P(refine_options), vp, i64, vp,
                                       P(refine_stats)]
    lib.refine_rayleigh_ritz.argtypes = [vp, vp, i64]
    lib.refine_batch_rayleigh_ritz.argtypes = [vp, P(vp), P(i64), P(i32)]
    lib.refine_sign_flip.argtypes = [vp, vp, i64, P(i32)]
    lib.refine_batch_sign_flip.argtypes = [vp, P(vp), P(i64), P(i32)]
    lib.refine_batch_time_product.argtypes = [vp, i32, P(ctypes.c_float)]
    lib.refine_debug_workspace.argtypes = [vp, P(vp), i32]
    lib.refine_debug_workspace.restype = ctypes.c_int
    lib.refine_status_string.argtypes = [ctypes.c_int]
    lib.refine_status_string.restype = ctypes.c_char_p
    for name in ("refine_init", "refine_step", "refine_run", "refine_get_info", "refine_destroy",
                 "refine_batch_init", "refine_batch_run", "refine_batch_destroy",
                 "refine_batch_time_product", "refine_rayleigh_ritz",
                 "refine_batch_rayleigh_ritz", "refine_time_product", "refine_sign_flip",
                 "refine_batch_sign_flip", "refine_time_product_parts", "refine_step_static"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _l():
    return load_library()


# ---------------------------------------------------------------------------
# Functions with the C names and C arguments.
# ---------------------------------------------------------------------------
def refine_options_default(opt: refine_options) -> None:
    _l().refine_options_default(ctypes.byref(opt))


def refine_init(ctx: ctypes.c_void_p, A: refine_matrix, k: int, opt: refine_options | None,
                hip_stream: int | None) -> int:
    return _l().refine_init(ctypes.byref(ctx), ctypes.byref(A), k,
                            ctypes.byref(opt) if opt is not None else None, hip_stream)


def refine_step(ctx, X_ptr: int, ldx: int, stats: refine_stats | None) -> int:
    return _l().refine_step(ctx, X_ptr, ldx, ctypes.byref(stats) if stats is not None else None)


def refine_run(ctx, X_ptr: int, ldx: int, max_iters: int, stop: int, tol: float,
               stats: refine_stats | None) -> int:
    return _l().refine_run(ctx, X_ptr, ldx, max_iters, stop, tol,
                           ctypes.byref(stats) if stats is not None else None)


def refine_rayleigh_ritz(ctx, X_ptr: int, ldx: int) -> int:
    return _l().refine_rayleigh_ritz(ctx, X_ptr, ldx)


def refine_sign_flip(ctx, X_ptr: int, ldx: int, sigma) -> int:
    return _l().refine_sign_flip(ctx, X_ptr, ldx, sigma)


def refine_get_info(ctx):
    v = [ctypes.c_double() for _ in range(4)]
    rc = _l().refine_get_info(ctx, *[ctypes.byref(x) for x in v])
    return rc, tuple(x.value for x in v)


def refine_time_product(ctx, X_ptr: int, ldx: int, reps: int):
    ms = ctypes.c_float()
    rc = _l().refine_time_product(ctx, X_ptr, ldx, reps, ctypes.byref(ms))
    return rc, ms.value


def refine_time_product_parts(ctx, X_ptr: int, ldx: int, reps: int, max_parts: int = 8):
    ms = (ctypes.c_float * max_parts)()
    n = ctypes.c_int32()
    rc = _l().refine_time_product_parts(ctx, X_ptr, ldx, reps, ms, max_parts, ctypes.byref(n))
    return rc, [ms[i] for i in range(min(n.value, max_parts))]


def refine_batch_time_product(b, reps: int):
    ms = ctypes.c_float()
    rc = _l().refine_batch_time_product(b, reps, ctypes.byref(ms))
    return rc, ms.value


def refine_destroy(ctx) -> int:
    return _l().refine_destroy(ctx)


def refine_batch_init(b: ctypes.c_void_p, count: int, As, ks, opt, hip_stream) -> int:
    return _l().refine_batch_init(ctypes.byref(b), count, As, ks,
                                  ctypes.byref(opt) if opt is not None else None, hip_stream)


def refine_batch_run(b, Xs, ldxs, iters: int, per_problem) -> int:
    return _l().refine_batch_run(b, Xs, ldxs, iters, per_problem)


def refine_batch_rayleigh_ritz(b, Xs, ldxs, status) -> int:
    return _l().refine_batch_rayleigh_ritz(b, Xs, ldxs, status)


def refine_batch_sign_flip(b, Xs, ldxs, status) -> int:
    return _l().refine_batch_sign_flip(b, Xs, ldxs, status)


def refine_batch_destroy(b) -> int:
    return _l().refine_batch_destroy(b)


def refine_status_string(status: int) -> str:
    return _l().refine_status_string(status).decode()


status_string = refine_status_string


# ---------------------------------------------------------------------------
# torch-facing wrappers
# ---------------------------------------------------------------------------
@dataclass
class Stats:
    corr_fro: float
    resid_rel: float
    iters: int
    status: int


def _require_cuda(t: torch.Tensor, dtype, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s" % (name, dtype))


def _stream_handle(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def make_options(precision="fp64", target="largest_abs", shift=0.0, delta_c=10.0, norm_a=0.0,
                 beta="half_gram", normalize=True, slices=0) -> refine_options:
    o = refine_options()
    refine_options_default(o)
    o.precision = {"fp64": FP64, "split_int8": SPLIT_INT8, "split_crt": SPLIT_CRT}[precision]
    o.target = TARGETS[target]
    o.shift = float(shift)
    o.delta_c = float(delta_c)
    o.norm_a = float(norm_a)
    o.beta = BETAS[beta]
    o.normalize = 1 if normalize else 0
    o.slices = int(slices)
    return o


def step_static(A: torch.Tensor, X: torch.Tensor, k: int, stream=None, sync: bool = True,
                **options):
    """One step through refine_step_static (no allocation, no context): A
    dense (n, n) float64 on the GPU, X (n, k) float64 updated in place;
    options as make_options (norm_a required).  Returns (status, Stats or
    None)."""
    _require_cuda(A, torch.float64, "A")
    _require_cuda(X, torch.float64, "X")
    m = refine_matrix()
    m.kind, m.n, m.a, m.lda = DENSE, A.shape[0], A.data_ptr(), A.stride(0)
    o = make_options(**options)
    st = refine_stats()
    rc = _l().refine_step_static(ctypes.byref(m), k, ctypes.byref(o), X.data_ptr(), X.stride(0),
                                 _stream_handle(stream), ctypes.byref(st) if sync else None)
    return rc, (Stats(st.corr_fro, st.resid_rel, st.iters, st.status) if sync else None)


@dataclass
class CsrMatrix:
    """Symmetric matrix in CSR form on the GPU (int32 indices, float64 values)."""
    n: int
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    val: torch.Tensor


def _matrix_struct(A) -> refine_matrix:
    m = refine_matrix()
    if isinstance(A, CsrMatrix):
        _require_cuda(A.row_ptr, torch.int32, "row_ptr")
        _require_cuda(A.col_idx, torch.int32, "col_idx")
        _require_cuda(A.val, torch.float64, "val")
        m.kind, m.n = CSR, A.n
        m.row_ptr, m.col_idx, m.val = A.row_ptr.data_ptr(), A.col_idx.data_ptr(), A.val.data_ptr()
        m.nnz = A.val.numel()
        m.a, m.lda = None, 0
    else:
        _require_cuda(A, torch.float64, "A")
        if A.dim() != 2 or A.shape[0] != A.shape[1] or A.stride(1) != 1:
            raise ValueError("A must be a square row-major float64 matrix")
        m.kind, m.n = DENSE, A.shape[0]
        m.a, m.lda = A.data_ptr(), A.stride(0)
    return m


class RefineContext:
    """One problem: refine k approximate eigenvectors X (n x k, float64, GPU)."""

    def __init__(self, A, k: int, stream=None, **options):
        self._A = A   # borrowed by the library: keep it alive
        self.k = k
        self.stream = stream
        self.n = A.n if isinstance(A, CsrMatrix) else A.shape[0]
        self._opt = make_options(**options)
        self._ctx = ctypes.c_void_p()
        rc = refine_init(self._ctx, _matrix_struct(A), k, self._opt, _stream_handle(stream))
        if rc != OK:
            raise RefineError(rc, "refine_init")

    def _check_x(self, X):
        _require_cuda(X, torch.float64, "X")
        if X.dim() != 2 or X.shape[0] != self.n or X.shape[1] != self.k or X.stride(1) != 1:
            raise ValueError("X must be (n, k) float64 with unit column stride")

    def step(self, X: torch.Tensor, sync: bool = True) -> Stats | None:
        """One refinement step on X in place.  sync=False only enqueues it."""
        self._check_x(X)
        if not sync:
            rc = refine_step(self._ctx, X.data_ptr(), X.stride(0), None)
            if rc != OK:
                raise RefineError(rc, "refine_step")
            return None
        st = refine_stats()
        rc = refine_step(self._ctx, X.data_ptr(), X.stride(0), st)
        s = Stats(st.corr_fro, st.resid_rel, st.iters, rc)
        return s

    def run(self, X: torch.Tensor, max_iters: int, stop: str = "iters", tol: float = 0.0) -> Stats:
        self._check_x(X)
        st = refine_stats()
        rc = refine_run(self._ctx, X.data_ptr(), X.stride(0), max_iters, STOPS[stop], tol, st)
        return Stats(st.corr_fro, st.resid_rel, st.iters, rc)

    def rayleigh_ritz(self, X: torch.Tensor) -> None:
        """Rayleigh-Ritz preprocessing of X in place (Sec. 3.4, clustered
        eigenvalues); the next applied step takes the leading block of E_L as
        zero.  Raises RefineError (ERANK when X^T X is not positive definite)."""
        self._check_x(X)
        rc = refine_rayleigh_ritz(self._ctx, X.data_ptr(), X.stride(0))
        if rc != OK:
            raise RefineError(rc, "refine_rayleigh_ritz")

    def sign_flip(self, X: torch.Tensor) -> list:
        """One-time column sign flip X <- X Sigma in place (Sec. 3.1.1, Sigma of
        the modified LU, Algorithm 2), for an X whose compact WY factor is
        singular; returns sigma as a list of +1 / -1."""
        self._check_x(X)
        k = X.shape[1]
        sg = (ctypes.c_int32 * k)()
        rc = refine_sign_flip(self._ctx, X.data_ptr(), X.stride(0), sg)
        if rc != OK:
            raise RefineError(rc, "refine_sign_flip")
        return list(sg)

    def time_product(self, X: torch.Tensor, reps: int) -> float:
        """Mean milliseconds of one launch of the product W = A X alone."""
        self._check_x(X)
        rc, ms = refine_time_product(self._ctx, X.data_ptr(), X.stride(0), reps)
        if rc != OK:
            raise RefineError(rc, "refine_time_product")
        return ms

    def time_product_parts(self, X: torch.Tensor, reps: int):
        """Mean milliseconds of each kernel of the product W = A X, in launch
        order (include/refine.h lists the kernels of each form)."""
        self._check_x(X)
        rc, ms = refine_time_product_parts(self._ctx, X.data_ptr(), X.stride(0), reps)
        if rc != OK:
            raise RefineError(rc, "refine_time_product_parts")
        return ms

    def debug_product(self):
        """Test hook: device copies (W_hi, W_lo) of the last step's product
        W = A X of its input X (W_lo is None outside split mode), read from
        the context's workspace after synchronising its stream."""
        ptrs = (ctypes.c_void_p * 2)()
        rc = _l().refine_debug_workspace(self._ctx, ptrs, 2)
        if rc != OK:
            raise RefineError(rc, "refine_debug_workspace")
        (self.stream or torch.cuda.current_stream()).synchronize()
        hip = ctypes.CDLL("libamdhip64.so.7")
        hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        out = []
        for p in ptrs:
            if not p:
                out.append(None)
                continue
            t = torch.empty((self.n, self.k), dtype=torch.float64, device="cuda")
            if hip.hipMemcpy(t.data_ptr(), p, 8 * self.n * self.k, 3) != 0:  # device to device
                raise RefineError(EHIP, "hipMemcpy")
            out.append(t)
        return out[0], out[1]

    def info(self) -> dict:
        rc, (mu, ninf, nused, delta) = refine_get_info(self._ctx)
        if rc != OK:
            raise RefineError(rc, "refine_get_info")
        return {"mu": mu, "norm_inf": ninf, "norm_used": nused, "delta": delta}

    def close(self):
        if self._ctx:
            refine_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RefineBatch:
    """Independent dense problems refined together (one grouped launch per kernel)."""

    def __init__(self, As, ks, stream=None, **options):
        self._As = list(As)
        self.ks = [int(k) for k in ks]
        self.stream = stream
        self._opt = make_options(**options)
        n = len(self._As)
        arr = (refine_matrix * n)(*[_matrix_struct(A) for A in self._As])
        karr = (ctypes.c_int32 * n)(*self.ks)
        self._b = ctypes.c_void_p()
        rc = refine_batch_init(self._b, n, arr, karr, self._opt, _stream_handle(stream))
        if rc != OK:
            raise RefineError(rc, "refine_batch_init")

    def run(self, Xs, iters: int, sync: bool = True):
        n = len(self._As)
        ptrs = (ctypes.c_void_p * n)(*[X.data_ptr() for X in Xs])
        lds = (ctypes.c_int64 * n)(*[X.stride(0) for X in Xs])
        if not sync:
            rc = refine_batch_run(self._b, ptrs, lds, iters, None)
            if rc != OK:
                raise RefineError(rc, "refine_batch_run")
            return None
        per = (refine_stats * n)()
        rc = refine_batch_run(self._b, ptrs, lds, iters, per)
        return rc, [Stats(p.corr_fro, p.resid_rel, p.iters, p.status) for p in per]

    def rayleigh_ritz(self, Xs):
        """Rayleigh-Ritz preprocessing of every problem in place (Sec. 3.4);
        returns (status, per-problem statuses)."""
        n = len(self._As)
        ptrs = (ctypes.c_void_p * n)(*[X.data_ptr() for X in Xs])
        lds = (ctypes.c_int64 * n)(*[X.stride(0) for X in Xs])
        st = (ctypes.c_int32 * n)()
        rc = refine_batch_rayleigh_ritz(self._b, ptrs, lds, st)
        return rc, list(st)

    def sign_flip(self, Xs):
        """Column sign flip X <- X Sigma of every problem in place (Sec. 3.1.1);
        returns (status, per-problem statuses)."""
        n = len(self._As)
        ptrs = (ctypes.c_void_p * n)(*[X.data_ptr() for X in Xs])
        lds = (ctypes.c_int64 * n)(*[X.stride(0) for X in Xs])
        st = (ctypes.c_int32 * n)()
        rc = refine_batch_sign_flip(self._b, ptrs, lds, st)
        return rc, list(st)

    def time_product(self, reps: int) -> float:
        """Mean milliseconds of one grouped product launch (X of the last run)."""
        rc, ms = refine_batch_time_product(self._b, reps)
        if rc != OK:
            raise RefineError(rc, "refine_batch_time_product")
        return ms

    def close(self):
        if self._b:
            refine_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
