"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws and assembles inputs: symmetric matrices with a known
eigen-decomposition, a 3-D Laplacian in CSR form, batches of independent
problems, and starting approximations X0.  It holds none of the refinement
method's arithmetic, and neither the GPU library nor the CPU oracle depends on
anything here except the arrays it returns.

Dense test matrices are A = Q diag(lam) Q^T, where Q is the product of m
seeded Householder reflectors H_i = I - 2 v v^T / v^T v with v ~ N(0, I_n),
accumulated 64 at a time in compact WY form (this accumulation is generic
linear algebra, unrelated to the paper's Algorithm 1).  The refined targets are
columns of Q, so the exact answer is known up to the rounding of A.

Shapes and spectra follow the paper's dense and sparse workloads: randsvd-like
dense matrices with ||A|| about 1 (Sec. 4.2) and sparse SPD matrices (Sec. 4.3,
replaced here by a 7-point Laplacian with a random diagonal, because the
SuiteSparse matrices are not available).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2026_0000


def _torch():
    import torch
    return torch


def householder_q(n: int, m: int | None = None, seed: int = 0, device: str = "cpu",
                  block: int = 64):
    """Q = H_1 H_2 ... H_m (float64 torch tensor on `device`)."""
    torch = _torch()
    m = n if m is None else m
    rng = np.random.default_rng(seed)
    Q = torch.eye(n, dtype=torch.float64, device=device)
    for b0 in range(0, m, block):
        b = min(block, m - b0)
        V = torch.from_numpy(rng.standard_normal((b, n)).T.copy()).to(device)  # n x b
        tau = 2.0 / (V * V).sum(0)
        # forward, columnwise T (upper triangular) so that H_1..H_b = I - V T V^T
        VtV = (V.T @ V).cpu()
        T = torch.zeros((b, b), dtype=torch.float64)
        tau_c = tau.cpu()
        for j in range(b):
            T[j, j] = tau_c[j]
            if j:
                T[:j, j] = -tau_c[j] * (T[:j, :j] @ VtV[:j, j])
        T = T.to(device)
        Q = Q - ((Q @ V) @ T) @ V.T
    return Q


@dataclass
class DenseProblem:
    A: object                 # n x n float64 (numpy or torch)
    lam: np.ndarray           # eigenvalues, lam[i] belongs to column i of Q
    targets: np.ndarray       # indices of the refined eigenpairs, in X0's column order
    X_true: object            # n x k, the columns of Q at `targets`
    X0: object                # n x k starting approximation
    mu: float = 0.0
    norm_a: float = 1.0
    meta: dict = field(default_factory=dict)


def _assemble(Q, lam, targets, torch_out: bool):
    torch = _torch()
    lam_t = torch.from_numpy(lam).to(Q.device)
    A = (Q * lam_t) @ Q.T
    A = 0.5 * (A + A.T)
    Xt = Q[:, torch.from_numpy(np.asarray(targets)).to(Q.device)].contiguous()
    if torch_out:
        return A.contiguous(), Xt
    return A.cpu().numpy(), Xt.cpu().numpy()


def fp32_round(X):
    """X rounded to single precision and back (the paper's single-precision
    starting vectors)."""
    if isinstance(X, np.ndarray):
        return X.astype(np.float32).astype(np.float64)
    return X.float().double()


def dense_well_separated(n=256, k=8, seed=SEED_BASE + 1, device="cpu", torch_out=False):
    """Small dense case: lam_i = i/n, the k largest are refined, X0 = fl32(Q_top)."""
    lam = np.arange(1, n + 1, dtype=np.float64) / n
    targets = np.arange(n - 1, n - 1 - k, -1)
    Q = householder_q(n, n, seed, device)
    A, Xt = _assemble(Q, lam, targets, torch_out)
    return DenseProblem(A, lam, targets, Xt, fp32_round(Xt), 0.0, float(lam.max()),
                        {"workload": "dense_well_separated", "n": n, "k": k, "seed": seed})


def dense_logspace(n=8192, k=64, seed=SEED_BASE + 2, device="cpu", torch_out=False,
                   noise=1e-7):
    """Log-spaced spectrum in [1e-3, 1]: the k largest of logspace(-3, 0, n) are the
    targets; the remaining n-k are log-spaced from 1e-3 up to lam_target_min/1.05,
    so the separation ratio is exactly 1.05.  X0 = Q_top + N(0, noise^2),
    re-orthonormalised by QR with a positive diagonal."""
    top = np.logspace(-3, 0, n)[n - k:]
    bottom = np.logspace(-3, math.log10(top[0] / 1.05), n - k)
    lam = np.concatenate([bottom, top])
    targets = np.arange(n - 1, n - 1 - k, -1)
    Q = householder_q(n, n, seed, device)
    A, Xt = _assemble(Q, lam, targets, torch_out)
    rng = np.random.default_rng(seed + 7)
    E = rng.standard_normal((n, k)) * noise
    torch = _torch()
    X0 = torch.as_tensor(np.asarray(Xt.cpu() if hasattr(Xt, "cpu") else Xt)) + torch.from_numpy(E)
    q, r = torch.linalg.qr(X0)
    q = q * torch.sign(torch.diagonal(r))
    X0 = q.numpy() if not torch_out else q.to(Xt.device)
    return DenseProblem(A, lam, targets, Xt, X0, 0.0, float(lam.max()),
                        {"workload": "dense_logspace", "n": n, "k": k, "seed": seed})


def dense_uniform_top(n=16384, k=128, seed=SEED_BASE + 3, device="cpu", torch_out=False):
    """Bottom n-k eigenvalues iid U[0, 0.871); the k targets at 0.872 + 1e-3 j,
    j = 0..k-1 (mutual gaps and gap to the rest >= 1e-3).  X0 = fl32(Q_top)."""
    rng = np.random.default_rng(seed)
    bottom = rng.uniform(0.0, 0.871, n - k)
    top = 0.872 + 1e-3 * np.arange(k)
    lam = np.concatenate([bottom, top])
    targets = np.arange(n - 1, n - 1 - k, -1)
    Q = householder_q(n, n, seed + 1, device)
    A, Xt = _assemble(Q, lam, targets, torch_out)
    return DenseProblem(A, lam, targets, Xt, fp32_round(Xt), 0.0, float(lam.max()),
                        {"workload": "dense_uniform_top", "n": n, "k": k, "seed": seed})


def dense_clustered(n, k, seed, device="cpu", torch_out=False, gap=1e-6):
    """Targets in two clusters of ceil(k/2) and floor(k/2) eigenvalues at
    0.98 + j*gap and 0.99 + j*gap; the rest iid U[0, 0.97).  X0 = fl32(Q_top)."""
    rng = np.random.default_rng(seed)
    k1 = (k + 1) // 2
    k2 = k // 2
    rest = rng.uniform(0.0, 0.97, n - k)
    c1 = 0.98 + gap * np.arange(k1)
    c2 = 0.99 + gap * np.arange(k2)
    lam = np.concatenate([rest, c1, c2])
    order = np.argsort(-lam[n - k:]) + (n - k)
    targets = order
    Q = householder_q(n, n, seed + 1, device)
    A, Xt = _assemble(Q, lam, targets, torch_out)
    return DenseProblem(A, lam, targets, Xt, fp32_round(Xt), 0.0, float(lam.max()),
                        {"workload": "dense_clustered", "n": n, "k": k, "seed": seed})


def dense_spectrum(n, k, seed, top_lo=0.9, top_hi=1.0, rest_hi=0.8, device="cpu",
                   torch_out=False):
    """k targets evenly spaced in [top_lo, top_hi] (descending in X0's column
    order), the rest iid U[0, rest_hi).  X0 = fl32(Q_top)."""
    rng = np.random.default_rng(seed)
    rest = rng.uniform(0.0, rest_hi, n - k)
    top = np.linspace(top_lo, top_hi, k) if k > 1 else np.array([top_hi])
    lam = np.concatenate([rest, top])
    targets = np.arange(n - 1, n - 1 - k, -1)
    Q = householder_q(n, n, seed + 1, device)
    A, Xt = _assemble(Q, lam, targets, torch_out)
    return DenseProblem(A, lam, targets, Xt, fp32_round(Xt), 0.0, float(lam.max()),
                        {"workload": "dense_spectrum", "n": n, "k": k, "seed": seed})


def dense_exact_first(n, k, seed, device="cpu", torch_out=False):
    """As dense_spectrum, except that the largest target's eigenvector is e_1
    exactly: Q = diag(1, Q') with Q' seeded Householder of order n - 1.  X0 =
    fl32(Q_top) then has e_1 as its first column, so X0(1:k,:) - I_k has a zero
    first column (the singular case of the compact WY form)."""
    torch = _torch()
    rng = np.random.default_rng(seed)
    rest = rng.uniform(0.0, 0.8, n - k)
    top = np.linspace(0.9, 1.0, k) if k > 1 else np.array([1.0])
    lam = np.concatenate([[top[-1]], rest, top[:-1]])
    targets = np.concatenate([[0], np.arange(n - 1, n - k, -1)]).astype(np.int64)
    Q = torch.zeros((n, n), dtype=torch.float64, device=device)
    Q[0, 0] = 1.0
    Q[1:, 1:] = householder_q(n - 1, n - 1, seed + 1, device)
    A, Xt = _assemble(Q, lam, targets, torch_out)
    return DenseProblem(A, lam, targets, Xt, fp32_round(Xt), 0.0, float(lam.max()),
                        {"workload": "dense_exact_first", "n": n, "k": k, "seed": seed})


def dense_smallest_abs(n, k, seed, device="cpu", torch_out=False, top=0.3, rest_lo=0.7):
    """Targets of small magnitude and both signs, +-top * (j + 1) / k with
    alternating signs (distinct |lambda|); the rest have |lambda| iid
    U[rest_lo, 1] with random signs.  The targets are the k smallest |lambda|
    (the squared-shift variant).  X0 = fl32(Q_top), in ascending |lambda|."""
    rng = np.random.default_rng(seed)
    mag = rng.uniform(rest_lo, 1.0, n - k)
    rest = mag * np.where(rng.uniform(size=n - k) < 0.5, -1.0, 1.0)
    tgt = top * np.arange(1, k + 1) / k * np.where(np.arange(k) % 2 == 0, 1.0, -1.0)
    lam = np.concatenate([rest, tgt])
    targets = np.arange(n - k, n)
    Q = householder_q(n, n, seed + 1, device)
    A, Xt = _assemble(Q, lam, targets, torch_out)
    return DenseProblem(A, lam, targets, Xt, fp32_round(Xt), 0.0, 1.0,
                        {"workload": "dense_smallest_abs", "n": n, "k": k, "seed": seed})


def batch_shapes(count=512, seed=SEED_BASE + 5, n_lo=128, n_hi=2048, k_lo=4, k_hi=32):
    """Sizes of the batched workload: n ~ U_int[n_lo, n_hi], k ~ U_int[k_lo, k_hi]."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, count)
    ks = rng.integers(k_lo, k_hi + 1, count)
    return [(int(a), int(b)) for a, b in zip(ns, ks)]


def batch_problems(count=512, seed=SEED_BASE + 5, device="cpu", torch_out=False,
                   shapes=None):
    """Independent clustered dense problems; problem p uses seed + 1000 p."""
    shapes = batch_shapes(count, seed) if shapes is None else shapes
    return [dense_clustered(n, k, seed + 1000 * (p + 1), device, torch_out)
            for p, (n, k) in enumerate(shapes)]


# ----------------------------------------------------------------------------
# Sparse: 3-D 7-point Dirichlet Laplacian with a random diagonal.
# ----------------------------------------------------------------------------
@dataclass
class CsrProblem:
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray
    sigma: float
    meta: dict = field(default_factory=dict)


def laplacian3d(N: int, seed: int = SEED_BASE + 4) -> CsrProblem:
    """Lexicographic N^3 grid (x fastest), diagonal 6 + U[0,1), off-diagonals -1
    for the grid neighbours; full symmetric pattern, columns sorted.
    sigma = max_i (a_ii + sum_{j != i} |a_ij|), the Gershgorin upper bound."""
    n = N ** 3
    rng = np.random.default_rng(seed)
    diag = 6.0 + rng.uniform(0.0, 1.0, n)
    idx = np.arange(n, dtype=np.int64)
    x = idx % N
    y = (idx // N) % N
    z = idx // (N * N)
    cols = []
    vals = []
    # neighbours in increasing column order: -z, -y, -x, self, +x, +y, +z
    for off, ok in ((-N * N, z > 0), (-N, y > 0), (-1, x > 0)):
        cols.append(np.where(ok, idx + off, -1))
        vals.append(np.where(ok, -1.0, 0.0))
    cols.append(idx)
    vals.append(diag)
    for off, ok in ((1, x < N - 1), (N, y < N - 1), (N * N, z < N - 1)):
        cols.append(np.where(ok, idx + off, -1))
        vals.append(np.where(ok, -1.0, 0.0))
    C = np.stack(cols, 1)
    Vv = np.stack(vals, 1)
    mask = C >= 0
    counts = mask.sum(1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = C[mask].astype(np.int32)
    val = Vv[mask].astype(np.float64)
    offsum = np.abs(Vv).sum(1) - diag
    sigma = float(np.max(diag + offsum))
    return CsrProblem(n, row_ptr.astype(np.int32), col_idx, val, sigma,
                      {"workload": "laplacian3d", "N": N, "seed": seed})


def laplacian_start(P: CsrProblem, k: int, seed: int, noise: float = 1e-6,
                    exact: bool = True):
    """Starting vectors for the k smallest eigenpairs.  exact=True: scipy's
    shift-invert Lanczos vectors (tight tolerance) plus N(0, noise^2), then
    orthonormalised; exact=False (large grids): the k smoothest sine modes of
    the unperturbed Dirichlet Laplacian, which are only rough approximations."""
    rng = np.random.default_rng(seed)
    n = P.n
    if exact:
        import scipy.sparse as sp
        import scipy.sparse.linalg as spl
        M = sp.csr_matrix((P.val, P.col_idx, P.row_ptr), shape=(n, n))
        w, V = spl.eigsh(M, k=k, sigma=0.0, which="LM", tol=0.0)
        order = np.argsort(w)
        V = V[:, order]
        X = V + noise * rng.standard_normal(V.shape)
    else:
        N = round(n ** (1.0 / 3.0))
        modes = sorted(((a, b, c) for a in range(1, 8) for b in range(1, 8) for c in range(1, 8)),
                       key=lambda t: (sum(1 - math.cos(math.pi * s / (N + 1)) for s in t), t))[:k]
        g = np.arange(1, N + 1)
        X = np.empty((n, k))
        for j, (a, b, c) in enumerate(modes):
            sx = np.sin(math.pi * a * g / (N + 1))
            sy = np.sin(math.pi * b * g / (N + 1))
            sz = np.sin(math.pi * c * g / (N + 1))
            X[:, j] = (sz[:, None, None] * sy[None, :, None] * sx[None, None, :]).reshape(-1)
        X += noise * rng.standard_normal(X.shape)
    q, r = np.linalg.qr(X)
    return q * np.sign(np.diag(r))



def laplacian3d_separable(N: int, k: int, seed: int = SEED_BASE + 4, noise: float = 1e-6,
                          start_seed: int = 7):
    """The 7-point Dirichlet Laplacian of laplacian3d with the diagonal
    perturbation split by axis: a_ii = 6 + dx[x] + dy[y] + dz[z] with
    dx, dy, dz iid U[0, 1/3) (so a_ii in [6, 7), the same pattern and nnz).
    A is then the Kronecker sum Tz + Ty + Tx of three tridiagonal N x N
    matrices T = tridiag(-1, 2 + d, -1), whose eigenpairs give those of A
    exactly: lambda = mu_x[a] + mu_y[b] + mu_z[c], v = vz[:, c] (x) vy[:, b] (x)
    vx[:, a].  Returns (CsrProblem, lam_k, X_true, X0) for the k smallest
    eigenpairs, X0 = X_true + N(0, noise^2) orthonormalised; used where the
    grid is too large for a sparse eigensolver here."""
    rng = np.random.default_rng(seed)
    d = [rng.uniform(0.0, 1.0 / 3.0, N) for _ in range(3)]  # x, y, z
    n = N ** 3
    idx = np.arange(n, dtype=np.int64)
    x = idx % N
    y = (idx // N) % N
    z = idx // (N * N)
    diag = 6.0 + d[0][x] + d[1][y] + d[2][z]
    cols = []
    vals = []
    for off, ok in ((-N * N, z > 0), (-N, y > 0), (-1, x > 0)):
        cols.append(np.where(ok, idx + off, -1))
        vals.append(np.where(ok, -1.0, 0.0))
    cols.append(idx)
    vals.append(diag)
    for off, ok in ((1, x < N - 1), (N, y < N - 1), (N * N, z < N - 1)):
        cols.append(np.where(ok, idx + off, -1))
        vals.append(np.where(ok, -1.0, 0.0))
    C = np.stack(cols, 1)
    Vv = np.stack(vals, 1)
    mask = C >= 0
    counts = mask.sum(1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = C[mask].astype(np.int32)
    val = Vv[mask].astype(np.float64)
    del C, Vv, mask
    sigma = float(np.max(diag + (counts - 1)))  # Gershgorin: off-diagonal entries are -1
    P = CsrProblem(n, row_ptr.astype(np.int32), col_idx, val, sigma,
                   {"workload": "laplacian3d_separable", "N": N, "seed": seed})
    eig = []
    for a in range(3):
        T = np.diag(2.0 + d[a]) - np.eye(N, k=1) - np.eye(N, k=-1)
        mu, V = np.linalg.eigh(T)
        eig.append((mu, V))
    m = min(N, 16)
    cand = sorted((eig[0][0][a] + eig[1][0][b] + eig[2][0][c], a, b, c)
                  for a in range(m) for b in range(m) for c in range(m))
    top = cand[:k + 1]
    lam = np.array([t[0] for t in top[:k]])
    Xt = np.empty((n, k))
    for j, (_, a, b, c) in enumerate(top[:k]):
        vx, vy, vz = eig[0][1][:, a], eig[1][1][:, b], eig[2][1][:, c]
        Xt[:, j] = (vz[:, None, None] * vy[None, :, None] * vx[None, None, :]).reshape(-1)
    r = np.random.default_rng(start_seed)
    X = Xt + noise * r.standard_normal(Xt.shape)
    q, rr = np.linalg.qr(X)
    X0 = q * np.sign(np.diag(rr))
    P.meta["lam_next"] = float(top[k][0])
    return P, lam, Xt, X0


def _banded_symmetric(m: int, b: int, rng) -> np.ndarray:
    """m x m symmetric with iid N(0, 1) entries on the 2b + 1 central diagonals."""
    T = np.zeros((m, m))
    for o in range(b + 1):
        v = rng.standard_normal(m - o)
        T += np.diag(v, o)
        if o:
            T += np.diag(v, -o)
    return T


def kron_banded(m=53, bands=(2, 2, 1), k=5, seed=SEED_BASE + 265, noise=1e-6, start_seed=11):
    """Sparse symmetric A = T1 (x) T2 (x) T3 of three banded m x m factors with
    iid N(0, 1) entries (half-bandwidths `bands`): a 3-D stencil of
    prod(2 b + 1) points (75 for (2, 2, 1); about 70.7 nonzeros per row with
    the boundary rows), indefinite, with eigenpairs known exactly from the
    factors: lambda = t1[a] t2[b] t3[c], v = u1[:, a] (x) u2[:, b] (x) u3[:, c].
    At m = 53 it has the size and density of the paper's larger SuiteSparse
    cases (148,877 rows, 10.5M nonzeros).  The targets are the k largest
    |lambda| (the paper's sparse runs: k = 5, largest magnitude); the default
    seed gives relative gaps >= 2.4e-2 among them and 4e-2 to the next.
    Returns (CsrProblem, lam_k, X_true, X0) with X0 = X_true + N(0, noise^2)
    orthonormalised; CsrProblem.sigma is max |lambda| (= ||A||_2)."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    facs = [_banded_symmetric(m, b, rng) for b in bands]
    eig = [np.linalg.eigh(T) for T in facs]
    A = sp.kron(sp.kron(sp.csr_matrix(facs[0]), sp.csr_matrix(facs[1]), format="csr"),
                sp.csr_matrix(facs[2]), format="csr")
    A.eliminate_zeros()
    A.sort_indices()
    n = A.shape[0]
    t = [e[0] for e in eig]
    lam_all = (t[0][:, None, None] * t[1][None, :, None] * t[2][None, None, :]).reshape(-1)
    order = np.argsort(-np.abs(lam_all), kind="stable")[:k + 1]
    Xt = np.empty((n, k))
    for j, flat in enumerate(order[:k]):
        a, b, c = np.unravel_index(flat, (m, m, m))
        u1, u2, u3 = eig[0][1][:, a], eig[1][1][:, b], eig[2][1][:, c]
        Xt[:, j] = (u1[:, None, None] * u2[None, :, None] * u3[None, None, :]).reshape(-1)
    lam = lam_all[order[:k]]
    P = CsrProblem(n, A.indptr.astype(np.int32), A.indices.astype(np.int32),
                   A.data.astype(np.float64), float(np.abs(lam_all).max()),
                   {"workload": "kron_banded", "m": m, "bands": list(bands), "seed": seed})
    P.meta["lam_next"] = float(lam_all[order[k]])
    r = np.random.default_rng(start_seed)
    X = Xt + noise * r.standard_normal(Xt.shape)
    q, rr = np.linalg.qr(X)
    X0 = q * np.sign(np.diag(rr))
    return P, lam, Xt, X0

