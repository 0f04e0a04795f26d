"""Benchmark of the refinement step (Algorithm 4 with Algorithm 1) on one MI355X.

Default workload (uniform_top): dense, n = 16384, k = 128, A = Q diag(lam)
Q^T with Q a product of 16384 seeded Householder reflectors, lam iid U[0,
0.871) for the rest and 0.872 + 1e-3 j (j = 0..127) for the targets, X0 =
the true eigenvectors rounded to FP32.  A step is the whole hot path: W = A X,
Rayleigh quotients, residual, compact-WY factors, correction matrix, WY
update and normalisation, replayed as one HIP graph.  `value` is the main
form's refined eigenvectors per second (k / seconds per step).  The main form
(--precision, default crt) is the modular split form: W = A X through 16
INT8 residue products on the matrix cores and a Chinese-remainder
reconstruction into a double-double W (Ozaki scheme II).  The other two forms
run on the same input and are reported beside it: FP64 (config.fp64) and the
slice split form (INT8 digit slices, config.split), each with its speed ratio
against FP64.  The first step of every form is compared with the
double-double oracle step and the FP64 oracle step, and orthogonality is
measured in extended precision after all timed steps; meets_targets says
whether a form reached both accuracy targets (1e-13 and 1e-14).

Other workloads (--workload):
  logspace     dense n = 8192, k = 64, log-spaced spectrum, gap ratio 1.05;
  laplacian    CSR 3-D Laplacian on a 128^3 grid (separable random diagonal),
               k = 32 smallest through the Gershgorin shift;
  batch        512 dense problems, n ~ U[128, 2048], k ~ U[4, 32], two target
               clusters of gap 1e-6 each; 5 steps per graph; FP64 and split;
  kron         CSR Kronecker product of three banded 53 x 53 factors (148,877
               rows, 70.7 nonzeros per row, the size and density of the
               paper's larger sparse cases), k = 5 largest |lambda|;
  smallest_abs dense n = 8192, k = 64, targets the smallest |lambda| of both
               signs through B = A^2 - alpha I (Sec. 5.2), two products per step.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("refined eigvecs/sec and A·X̂ eff. GFLOP/s at ≤1e-13 err, split vs FP64")
FP64_PEAK_TFLOPS = 78.6
INT8_PEAK_TOPS = 5000.0
HBM_PEAK_GBS = 8000.0


def _cores() -> int:
    """Threads the oracle's OpenMP products run on: OMP_NUM_THREADS when set,
    bounded by the CPUs this process may use."""
    try:
        avail = len(os.sched_getaffinity(0))
    except Exception:
        avail = os.cpu_count() or 1
    try:
        omp = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        omp = 0
    return min(avail, omp) if omp > 0 else avail


def _aligned_err(g, o):
    import numpy as np
    s = np.sign(np.sum(g * o, 0))
    s[s == 0] = 1.0
    return float(np.max(np.abs(g * s - o)))


def _orthogonality(X):
    """max |X^T X - I| in extended precision on the host."""
    import numpy as np
    Xl = np.asarray(X, dtype=np.longdouble)
    G = Xl.T @ Xl
    return float(np.max(np.abs(G - np.eye(G.shape[0], dtype=np.longdouble))))


def _time_steps(ctx, X, steps, warmup, torch):
    st1 = ctx.step(X)
    X_first = X.clone()
    for _ in range(warmup):
        ctx.step(X, sync=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.step(X, sync=False)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    st_last = ctx.step(X)
    # every timed step was applied: a step that failed would have stopped the
    # context, and the later ones would have been no-ops
    _check_applied(st1.status, 1, st1.iters, "first step")
    _check_applied(st_last.status, warmup + steps + 2, st_last.iters, "timed steps")
    return sec, st1, st_last, X_first


def _meets(d):
    """Both accuracy targets met (None when the double-double check did not run)."""
    e = d.get("err_vs_dd_oracle_first_step")
    if e is None:
        return None
    return bool(e <= 1e-13 and d["orthogonality_last"] <= 1e-14)


def _progress(msg):
    print("bench: %s" % msg, file=sys.stderr, flush=True)


def _check_applied(status, want_iters, iters, what):
    if status != 0 or iters != want_iters:
        raise RuntimeError("%s: status %d, %d steps applied (expected %d): the timing is void"
                           % (what, status, iters, want_iters))


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def kernel_source_key(files):
    """SHA-256 of the named sources under paper_2602_23778_amd/csrc with their
    comments and blank space removed: it changes when the code of a kernel
    changes, not when its comments do."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in files:
        with open(os.path.join(ROOT, "paper_2602_23778_amd", "csrc", name)) as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(("%s\n%s\n" % (name, " ".join(src.split()))).encode())
    return h.hexdigest()


def _traffic_for(kernel_file, n, k):
    """HBM bytes per launch of the product from the committed counter summary
    profiles/traffic_<kernel>_n<n>_k<k>.json, when it was taken on this
    workload and on the present code of the kernel (else None)."""
    tpath = os.path.join(ROOT, "profiles", "traffic_%s_n%d_k%d.json" % (kernel_file, n, k))
    if not os.path.exists(tpath):
        return None
    try:
        with open(tpath) as f:
            tj = json.load(f)
        if tj.get("kernel_source_key") != kernel_source_key(tj["sources"]):
            return None
        return tj.get("bytes_per_launch")
    except Exception:
        return None


def _time_rayleigh_ritz(ctx, X0, torch, reps=3):
    """Milliseconds of one Rayleigh-Ritz preprocessing call (Sec. 3.4) on a copy
    of the start block, host-synchronised (the call reads its status back)."""
    best = None
    for _ in range(reps):
        Xr = X0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.rayleigh_ritz(Xr)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) * 1e3
        best = t if best is None else min(best, t)
    return best


FORMS = {"fp64": ("fp64", "FP64 plain"), "split": ("split_int8", "split INT8 slices"),
         "crt": ("split_crt", "modular INT8 (Ozaki scheme II)")}


def _form_slices(args, prec):
    return {"fp64": 0, "split_int8": args.slices, "split_crt": args.moduli}[prec]


# The dominant kernel of each form's product (index in the launch order that
# refine_time_product_parts reports) and the roofline it is held to.
DOMINANT = {"fp64": 0, "split_int8": 2, "split_crt": 2}


def _kpad(k):
    return (k + 31) // 32 * 32


def _product_roofline(prec, n, k, s, ms_kernel):
    """Roofline of the dominant kernel of the form's product, from its mean
    launch time (HIP events on the context's stream): the FP64 GEMM against
    the FP64 matrix peak (2 n^2 k flops; AI = k/4 flop/B is past the ridge);
    the slice products against the INT8 peak (s(s+1)/2 products of 2 n^2 k
    operations); the residue products of the modular form against HBM: they
    read the s residue planes of A (n^2 bytes each) and of X (n kpad bytes
    each) and write the s residue planes of the products (n kpad bytes each),
    at 2 kpad operations per byte of A, below the INT8 ridge of 625."""
    flops = 2.0 * n * n * k
    if prec == "fp64":
        eff = flops / (ms_kernel * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": eff, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": eff / FP64_PEAK_TFLOPS, "traffic": _traffic_for("gemm_f64_dense", n, k)}
    if prec == "split_int8":
        tops = s * (s + 1) / 2 * flops / (ms_kernel * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": tops, "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
                "frac": tops / INT8_PEAK_TOPS, "traffic": None}
    byts = _crt_gemm_bytes(n, k, s)
    gbs = byts / (ms_kernel * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": _traffic_for("crt_gemm", n, k)}


def _crt_gemm_bytes(n, k, nmod):
    """Algorithmic bytes of one launch of the modular form's residue products."""
    return nmod * (float(n) * n + 2.0 * n * _kpad(k))


def _product_only(ctx, X0, args, torch, info):
    """Counter runs: one plain copy of 2 GiB (a kernel of known size, for
    calibrating byte counters), then --product-reps launches of the product
    alone; prints their mean time."""
    buf = torch.empty(1 << 28, dtype=torch.float64, device=X0.device)
    cp = buf.clone()           # reads and writes 2 GiB
    torch.cuda.synchronize()
    del cp, buf
    ms = ctx.time_product(X0.clone(), args.product_reps)
    info.update({"product_ms": ms, "copy_bytes": 1 << 31})
    print(json.dumps(info), flush=True)


def bench_dense(args, rf, torch, np):
    import synth
    dev = "cuda:0"
    if args.workload == "logspace":
        n, k = args.n or 8192, args.k or 64
        P = synth.dense_logspace(n, k, device=dev, torch_out=True)
        desc = ("dense, n=%d, k=%d, log-spaced spectrum in [1e-3, 1], separation ratio 1.05, "
                "Householder Q" % (n, k))
    else:
        n, k = args.n or 16384, args.k or 128
        P = synth.dense_uniform_top(n, k, device=dev, torch_out=True)
        desc = ("dense, n=%d, k=%d, rest U[0, 0.871), targets 0.872 + 1e-3 j, Householder Q"
                % (n, k))
    A = P.A
    X0 = P.X0.to(dev).contiguous()
    torch.cuda.synchronize()

    main_prec = FORMS[args.precision][0]
    if args.product_only:
        ctx = rf.RefineContext(A, k, norm_a=P.norm_a, precision=main_prec,
                               slices=_form_slices(args, main_prec))
        _product_only(ctx, X0, args, torch, {"n": n, "k": k, "precision": main_prec,
                                             "slices": _form_slices(args, main_prec)})
        ctx.close()
        return None

    forms = [main_prec]
    if not args.no_split:
        forms += [FORMS[f][0] for f in ("fp64", "split", "crt") if FORMS[f][0] != main_prec]
    res = {}
    for prec in forms:
        s = _form_slices(args, prec)
        ctx = rf.RefineContext(A, k, norm_a=P.norm_a, precision=prec, slices=s)
        X = X0.clone()
        sec, st1, st_last, X_first = _time_steps(ctx, X, args.steps, args.warmup, torch)
        _progress("%s form timed: %.4f ms per step" % (prec, sec * 1e3))
        # the product W = A X alone, and each of its kernels, timed with HIP
        # events on the context's stream, same launch configuration as
        # inside the step
        ms_prod = ctx.time_product(X0.clone(), args.product_reps)
        parts = ctx.time_product_parts(X0.clone(), args.product_reps)
        rr_ms = _time_rayleigh_ritz(ctx, X0, torch) if prec == main_prec else None
        ctx.close()
        res[prec] = {"slices": s, "sec": sec, "st1": st1, "st_last": st_last,
                     "X_first": X_first.cpu().numpy(), "ms_prod": ms_prod, "rr_ms": rr_ms,
                     "parts": parts, "orth": _orthogonality(X.cpu().numpy())}

    errs = {p: {} for p in forms}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        A_h = A.cpu().numpy()
        X0_h = X0.cpu().numpy()
        # FP64 oracle steps from the same start until about 10 s have passed
        ts = time.perf_counter()
        reps = 0
        while reps == 0 or time.perf_counter() - ts < 10.0:
            r = oracle.refine_step(A_h, X0_h, norm_a=P.norm_a)
            reps += 1
        t_cpu = (time.perf_counter() - ts) / reps
        _progress("FP64 oracle: %d steps, %.2f s each" % (reps, t_cpu))
        for p in forms:
            errs[p]["err_vs_fp64_oracle_first_step"] = _aligned_err(res[p]["X_first"], r.X)
        cpu = {"value": k / t_cpu, "unit": "eigvecs/s", "cores": _cores(), "kind": "oracle",
               "cpu": _cpu_model(),
               "sample": "%d full FP64 oracle steps of the same workload (n=%d, k=%d), %.2f s each"
                         % (reps, n, k, t_cpu)}
        if not args.no_dd_check:
            _progress("double-double oracle step")
            rd = oracle.refine_step(A_h, X0_h, norm_a=P.norm_a, dd=True)
            for p in forms:
                errs[p]["err_vs_dd_oracle_first_step"] = _aligned_err(res[p]["X_first"], rd.X)

    flops = 2.0 * n * n * k

    def block(p):
        r = res[p]
        dom = r["parts"][DOMINANT[p]]
        b = {"precision": p, "slices": r["slices"], "eigvecs_per_s": k / r["sec"],
             "ms_per_step": r["sec"] * 1e3, "product_us": r["ms_prod"] * 1e3,
             "product_kernels_us": [t * 1e3 for t in r["parts"]],
             "product_eff_gflops": flops / (r["ms_prod"] * 1e-3) / 1e9,
             "product_roofline": _product_roofline(p, n, k, r["slices"], dom),
             "corr_fro_first": r["st1"].corr_fro, "corr_fro_last": r["st_last"].corr_fro,
             "resid_rel_last": r["st_last"].resid_rel, "orthogonality_last": r["orth"]}
        b.update(errs[p])
        if p != main_prec:
            b["max_dx_first_step_vs_main"] = _aligned_err(r["X_first"], res[main_prec]["X_first"])
        b["meets_targets"] = _meets(b)
        return b

    blocks = {p: block(p) for p in forms}
    main = res[main_prec]
    value = k / main["sec"]
    roof = blocks[main_prec].pop("product_roofline")
    cfg = {"workload": "%s form, " % FORMS[args.precision][1] + desc,
           "n": n, "k": k, "precision": main_prec, "slices": main["slices"],
           "rayleigh_ritz_ms": main["rr_ms"]}
    cfg.update({kk: vv for kk, vv in blocks[main_prec].items() if kk not in ("precision", "slices")})
    # the other forms on the same input, each with its speed against FP64
    t64 = res["fp64"]["sec"] if "fp64" in res else None
    for p in forms:
        if p == main_prec:
            continue
        b = blocks[p]
        if t64 is not None and p != "fp64":
            b["speed_ratio_split_over_fp64"] = t64 / res[p]["sec"]
        cfg[{"fp64": "fp64", "split_int8": "split", "split_crt": "split_crt"}[p]] = b
    if main_prec != "fp64" and t64 is not None:
        cfg["speed_ratio_split_over_fp64"] = t64 / main["sec"]
    # the accuracy targets: max |dX| <= 1e-13 against the double-double oracle
    # step, orthogonality max |X^T X - I| <= 1e-14 after all steps
    cfg["targets"] = {"err_vs_dd_oracle": 1e-13, "orthogonality": 1e-14}
    return {"value": value, "ms_per_step": main["sec"] * 1e3, "unit": "eigvecs/s",
            "dtype": "f64" if main_prec == "fp64" else "i8", "config": cfg, "roofline": roof,
            "cpu_baseline": cpu}


def bench_laplacian(args, rf, torch, np):
    import synth
    N = args.n or 128
    k = args.k or 32
    L, lam, Xt, X0h = synth.laplacian3d_separable(N, k)
    n, nnz = L.n, len(L.val)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    C = rf.CsrMatrix(n, dev(L.row_ptr), dev(L.col_idx), dev(L.val))
    ctx = rf.RefineContext(C, k, target="smallest", norm_a=L.sigma)
    X0 = dev(X0h)
    if args.product_only:
        _product_only(ctx, X0, args, torch, {"n": n, "k": k, "nnz": nnz})
        ctx.close()
        return None
    X = X0.clone()
    sec, st1, st_last, X_first = _time_steps(ctx, X, args.steps, args.warmup, torch)
    ms_prod = ctx.time_product(X0.clone(), args.product_reps)
    rr_ms = _time_rayleigh_ritz(ctx, X0, torch)
    ctx.close()
    byts = 12.0 * nnz + 4.0 * (n + 1) + 16.0 * n * k
    gbs = byts / (ms_prod * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": _traffic_for("spmm_csr", n, k)}
    Xg = X.cpu().numpy()
    cfg = {"workload": "CSR FP64, 3-D 7-point Laplacian %d^3 (n=%d, nnz=%d), diagonal 6 + "
                       "dx+dy+dz with d* iid U[0, 1/3), k=%d smallest via the Gershgorin shift"
                       % (N, n, nnz, k),
           "n": n, "k": k, "nnz": nnz, "precision": "fp64",
           "product_us": ms_prod * 1e3,
           "product_eff_gflops": 2.0 * nnz * k / (ms_prod * 1e-3) / 1e9,
           "corr_fro_first": st1.corr_fro, "corr_fro_last": st_last.corr_fro,
           "resid_rel_last": st_last.resid_rel,
           "err_vs_exact_eigvecs_last": _aligned_err(Xg, Xt),
           "err_vs_exact_eigvecs_start": _aligned_err(X0h, Xt),
           "rayleigh_ritz_ms": rr_ms}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        Co = oracle.Csr(n, L.row_ptr, L.col_idx, L.val)
        ts = time.perf_counter()
        # the library's shift for target="smallest" is the Gershgorin upper bound
        r = oracle.refine_step(Co, X0h, mu=L.sigma, norm_a=L.sigma)
        t_cpu = time.perf_counter() - ts
        cfg["err_vs_fp64_oracle_first_step"] = _aligned_err(X_first.cpu().numpy(), r.X)
        cpu = {"value": k / t_cpu, "unit": "eigvecs/s", "cores": _cores(), "kind": "oracle",
               "cpu": _cpu_model(), "sample": "one full FP64 oracle step of the same workload, %.1f s" % t_cpu}
    return {"value": k / sec, "ms_per_step": sec * 1e3, "unit": "eigvecs/s", "dtype": "f64",
            "config": cfg, "roofline": roof, "cpu_baseline": cpu}


def bench_kron(args, rf, torch, np):
    import synth
    m = args.n or 53
    k = args.k or 5
    K, lam, Xt, X0h = synth.kron_banded(m=m, k=k)
    n, nnz = K.n, len(K.val)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    C = rf.CsrMatrix(n, dev(K.row_ptr), dev(K.col_idx), dev(K.val))
    ctx = rf.RefineContext(C, k, norm_a=K.sigma)
    X0 = dev(X0h)
    if args.product_only:
        _product_only(ctx, X0, args, torch, {"n": n, "k": k, "nnz": nnz})
        ctx.close()
        return None
    X = X0.clone()
    sec, st1, st_last, X_first = _time_steps(ctx, X, args.steps, args.warmup, torch)
    ms_prod = ctx.time_product(X0.clone(), args.product_reps)
    rr_ms = _time_rayleigh_ritz(ctx, X0, torch)
    ctx.close()
    byts = 12.0 * nnz + 4.0 * (n + 1) + 16.0 * n * k
    gbs = byts / (ms_prod * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": _traffic_for("spmm_csr", n, k)}
    Xg = X.cpu().numpy()
    cfg = {"workload": "CSR FP64, Kronecker product of three banded %d x %d factors "
                       "(half-bandwidths 2, 2, 1; n=%d, nnz=%d, %.1f per row), k=%d largest |lambda|"
                       % (m, m, n, nnz, nnz / n, k),
           "n": n, "k": k, "nnz": nnz, "precision": "fp64",
           "product_us": ms_prod * 1e3,
           "product_eff_gflops": 2.0 * nnz * k / (ms_prod * 1e-3) / 1e9,
           "corr_fro_first": st1.corr_fro, "corr_fro_last": st_last.corr_fro,
           "resid_rel_last": st_last.resid_rel,
           "err_vs_exact_eigvecs_last": _aligned_err(Xg, Xt),
           "err_vs_exact_eigvecs_start": _aligned_err(X0h, Xt),
           "rayleigh_ritz_ms": rr_ms}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        Co = oracle.Csr(n, K.row_ptr, K.col_idx, K.val)
        ts = time.perf_counter()
        reps = 0
        while reps == 0 or time.perf_counter() - ts < 10.0:
            r = oracle.refine_step(Co, X0h, norm_a=K.sigma)
            reps += 1
        t_cpu = (time.perf_counter() - ts) / reps
        cfg["err_vs_fp64_oracle_first_step"] = _aligned_err(X_first.cpu().numpy(), r.X)
        cpu = {"value": k / t_cpu, "unit": "eigvecs/s", "cores": _cores(), "kind": "oracle",
               "cpu": _cpu_model(), "sample": "%d FP64 oracle steps of the same workload, %.3f s each" % (reps, t_cpu)}
    return {"value": k / sec, "ms_per_step": sec * 1e3, "unit": "eigvecs/s", "dtype": "f64",
            "config": cfg, "roofline": roof, "cpu_baseline": cpu}


def bench_smallest_abs(args, rf, torch, np):
    import synth
    n = args.n or 8192
    k = args.k or 64
    P = synth.dense_smallest_abs(n, k, synth.SEED_BASE + 12, device="cuda", torch_out=True)
    torch.cuda.synchronize()
    lhat = 0.7  # the rest of the spectrum has |lambda| >= 0.7
    ctx = rf.RefineContext(P.A, k, norm_a=1.0, target="smallest_abs", shift=lhat)
    alpha = ctx.info()["mu"]
    X0 = P.X0.cuda().contiguous()
    X = X0.clone()
    sec, st1, st_last, X_first = _time_steps(ctx, X, args.steps, args.warmup, torch)
    ms_prod = ctx.time_product(X0.clone(), args.product_reps)
    ctx.close()
    flops = 2.0 * n * n * k
    tf = flops / (ms_prod * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": tf / FP64_PEAK_TFLOPS, "traffic": None}
    Xt = P.X_true.cpu().numpy()
    cfg = {"workload": "dense FP64 n=%d, k=%d smallest |lambda| (targets +-0.3(j+1)/k, rest "
                       "|lambda| in [0.7, 1]) through B = A^2 - alpha I, alpha=%.4f, two products "
                       "per step" % (n, k, alpha),
           "n": n, "k": k, "precision": "fp64", "alpha": alpha,
           "product_us_one_of_two": ms_prod * 1e3,
           "corr_fro_first": st1.corr_fro, "corr_fro_last": st_last.corr_fro,
           "err_vs_exact_eigvecs_last": _aligned_err(X.cpu().numpy(), Xt),
           "err_vs_exact_eigvecs_start": _aligned_err(X0.cpu().numpy(), Xt)}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        A_h = P.A.cpu().numpy()
        X0h = X0.cpu().numpy()
        ts = time.perf_counter()
        r = oracle.refine_step(A_h, X0h, mu=alpha, norm_a=1.0, square=True)
        t_cpu = time.perf_counter() - ts
        cfg["err_vs_fp64_oracle_first_step"] = _aligned_err(X_first.cpu().numpy(), r.X)
        cpu = {"value": k / t_cpu, "unit": "eigvecs/s", "cores": _cores(), "kind": "oracle",
               "cpu": _cpu_model(), "sample": "one full FP64 oracle step of the same workload, %.1f s" % t_cpu}
    return {"value": k / sec, "ms_per_step": sec * 1e3, "unit": "eigvecs/s", "dtype": "f64",
            "config": cfg, "roofline": roof, "cpu_baseline": cpu}


def bench_batch(args, rf, torch, np):
    import synth
    count = args.count
    probs = synth.batch_problems(count, device="cuda", torch_out=True)
    torch.cuda.synchronize()
    As = [p.A for p in probs]
    ks = [int(p.X0.shape[1]) for p in probs]
    ns = [int(p.A.shape[0]) for p in probs]
    X0s = [p.X0.cuda().contiguous() for p in probs]
    ksum = sum(ks)
    steps_per_graph = 5
    reps = max(1, args.steps // steps_per_graph)
    res = {}
    for prec in ("fp64", "split_int8"):
        b = rf.RefineBatch(As, ks, norm_a=1.0, precision=prec,
                           slices=args.slices if prec == "split_int8" else 0)
        Xs = [x.clone() for x in X0s]
        rc, _ = b.run(Xs, steps_per_graph)
        first = [x.clone() for x in Xs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            b.run(Xs, steps_per_graph, sync=False)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / (reps * steps_per_graph)
        # every timed step of every problem was applied
        rc2, per = b.run(Xs, 0)
        for p, st in enumerate(per):
            _check_applied(st.status, steps_per_graph * (reps + 1), st.iters,
                           "%s batch, problem %d" % (prec, p))
        _progress("%s batch timed" % prec)
        ms_prod = b.time_product(args.product_reps)
        Xr = [x.clone() for x in X0s]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.rayleigh_ritz(Xr)
        torch.cuda.synchronize()
        rr_ms = (time.perf_counter() - t0) * 1e3
        b.close()
        res[prec] = {"sec": sec, "first": first, "rc": rc, "ms_prod": ms_prod, "rr_ms": rr_ms}
    byts = sum(8.0 * n * n for n in ns)
    main = res["fp64"]
    gbs = byts / (main["ms_prod"] * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": None}
    sample = list(range(min(args.sample, count)))
    cfg = {"workload": "batch of %d dense problems, n ~ U[128, 2048], k ~ U[4, 32], two target "
                       "clusters of internal gap 1e-6, 5 steps per graph, FP64 form" % count,
           "problems": count, "sum_k": ksum, "mean_n2": float(np.mean(np.array(ns, float) ** 2)),
           "precision": "fp64", "product_us": main["ms_prod"] * 1e3,
           "rayleigh_ritz_ms": main["rr_ms"],
           "split": {"slices": args.slices, "eigvecs_per_s": ksum / res["split_int8"]["sec"],
                     "ms_per_step": res["split_int8"]["sec"] * 1e3,
                     "product_us": res["split_int8"]["ms_prod"] * 1e3,
                     "speed_ratio_split_over_fp64": main["sec"] / res["split_int8"]["sec"]}}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        e64, esp = [], []
        ts = time.perf_counter()
        tcpu = 0.0
        for p in sample:
            A_h = probs[p].A.cpu().numpy()
            X_h = probs[p].X0.cpu().numpy()
            t1 = time.perf_counter()
            Xd, _ = oracle.refine(A_h, X_h, steps_per_graph, norm_a=1.0, dd=True)
            tcpu += time.perf_counter() - t1
            e64.append(_aligned_err(res["fp64"]["first"][p].cpu().numpy(), Xd))
            esp.append(_aligned_err(res["split_int8"]["first"][p].cpu().numpy(), Xd))
        cfg["err_vs_dd_oracle_5_steps_fp64_max"] = max(e64)
        cfg["split"]["err_vs_dd_oracle_5_steps_max"] = max(esp)
        cfg["err_sample"] = "problems 0..%d, 5 steps each, double-double oracle" % (len(sample) - 1)
        kk = sum(ks[p] for p in sample) * steps_per_graph
        cpu = {"value": kk / tcpu, "unit": "eigvecs/s", "cores": _cores(), "kind": "oracle",
               "cpu": _cpu_model(), "sample": "double-double oracle, 5 steps of problems 0..%d (%.1f s)"
                         % (len(sample) - 1, tcpu)}
    return {"value": ksum / main["sec"], "ms_per_step": main["sec"] * 1e3, "unit": "eigvecs/s",
            "dtype": "f64", "config": cfg, "roofline": roof, "cpu_baseline": cpu}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="uniform_top",
                    choices=["logspace", "uniform_top", "laplacian", "batch", "kron",
                             "smallest_abs"])
    ap.add_argument("--n", type=int, default=0,
                    help="dense n (default 8192 / 16384) or the Laplacian grid side (128)")
    ap.add_argument("--k", type=int, default=0)
    ap.add_argument("--count", type=int, default=512, help="batch: number of problems")
    ap.add_argument("--sample", type=int, default=8, help="batch: problems checked on the CPU")
    ap.add_argument("--precision", default="crt", choices=["fp64", "split", "crt"],
                    help="dense: the main form (the other two run on the same input)")
    ap.add_argument("--slices", type=int, default=0,
                    help="split slices (default 9; 10 for the clustered batch)")
    ap.add_argument("--moduli", type=int, default=16, help="modular form: moduli (12..16)")
    ap.add_argument("--no-split", action="store_true", help="skip the other forms")
    ap.add_argument("--no-dd-check", action="store_true",
                    help="dense: skip the comparison of the first step with the double-double "
                         "oracle (about a minute of host time at n = 16384)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--product-reps", type=int, default=20)
    ap.add_argument("--product-only", action="store_true",
                    help="counter runs (dense, laplacian, kron): one copy of 2 GiB (a plain "
                         "copy kernel of known size, for calibrating byte counters) then "
                         "--product-reps launches of the product alone; prints their mean time")
    args = ap.parse_args()
    if args.slices == 0:
        args.slices = 10 if args.workload == "batch" else 9
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2602_23778_amd as rf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    rf.load_library()
    t0 = time.time()
    if args.workload in ("logspace", "uniform_top"):
        r = bench_dense(args, rf, torch, np)
        if r is None:
            return 0
    elif args.workload == "laplacian":
        r = bench_laplacian(args, rf, torch, np)
        if r is None:
            return 0
    elif args.workload == "kron":
        r = bench_kron(args, rf, torch, np)
        if r is None:
            return 0
    elif args.workload == "smallest_abs":
        r = bench_smallest_abs(args, rf, torch, np)
    else:
        r = bench_batch(args, rf, torch, np)
    print("bench done in %.1f s" % (time.time() - t0), file=sys.stderr, flush=True)
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": r["unit"],
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": r["dtype"],
        "data": "synthetic",
        "config": r["config"],
        "roofline": r["roofline"],
        "cpu_baseline": r["cpu_baseline"],
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
