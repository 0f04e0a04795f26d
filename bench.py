"""Benchmark of one refinement step (Algorithm 4 with Algorithm 1) on one MI355X.

Workload (default): dense FP64, n = 8192, k = 64, A = Q diag(lam) Q^T with Q a
product of 8192 seeded Householder reflectors, lam log-spaced in [1e-3, 1]
with the 64 targets separated by a factor 1.05 from the rest, X0 = true
eigenvectors + N(0, 1e-7^2) noise, orthonormalised.  A step is the whole hot
path: W = A X, Rayleigh quotients, residual, compact-WY factors, correction
matrix, WY update and normalisation, replayed as one HIP graph.

`value` is the FP64 form's refined eigenvectors per second (k eigenvectors
per step / seconds per step).  The split-precision form (INT8 slices on the
matrix cores, double-double W) runs on the same workload and is reported in
config.split with its speed ratio to the FP64 form and its error against the
oracle.  --workload uniform_top selects the n = 16384, k = 128 uniform
spectrum instead; --precision split makes the split form the timed one.

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
    try:
        return len(os.sched_getaffinity(0))
    except Exception:
        return os.cpu_count() or 1


def _problem(workload, n, k, dev):
    import synth
    if workload == "logspace":
        P = synth.dense_logspace(n, k, device=dev, torch_out=True)
        desc = ("dense, n=%d, k=%d, log-spaced spectrum in [1e-3, 1], separation ratio 1.05, "
                "Householder Q" % (n, k))
    elif workload == "uniform_top":
        P = synth.dense_uniform_top(n, k, device=dev, torch_out=True)
        desc = ("dense, n=%d, k=%d, rest U[0, 0.871), targets 0.872 + 1e-3 j, Householder Q"
                % (n, k))
    else:
        raise SystemExit("unknown workload %s" % workload)
    return P, desc


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
    return sec, st1, st_last, X_first


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="logspace", choices=["logspace", "uniform_top"])
    ap.add_argument("--n", type=int, default=0, help="default 8192 (logspace), 16384 (uniform_top)")
    ap.add_argument("--k", type=int, default=0, help="default 64 (logspace), 128 (uniform_top)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "split"])
    ap.add_argument("--slices", type=int, default=9)
    ap.add_argument("--no-split", action="store_true", help="skip the split-form comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--product-reps", type=int, default=20)
    ap.add_argument("--product-only", action="store_true",
                    help="counter runs: one copy of A (a plain copy kernel of known size, "
                         "for calibrating byte counters) then --product-reps launches of the "
                         "product alone; prints their mean time")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2602_23778_amd as rf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    rf.load_library()
    dev = "cuda:0"
    n = args.n or (8192 if args.workload == "logspace" else 16384)
    k = args.k or (64 if args.workload == "logspace" else 128)
    t0 = time.time()
    P, desc = _problem(args.workload, n, k, dev)
    A = P.A
    X0 = P.X0.to(dev).contiguous()
    torch.cuda.synchronize()
    print("input ready in %.1f s" % (time.time() - t0), file=sys.stderr, flush=True)

    main_prec = "split_int8" if args.precision == "split" else "fp64"
    slices = args.slices if main_prec == "split_int8" else 0
    ctx = rf.RefineContext(A, k, norm_a=P.norm_a, precision=main_prec, slices=slices)
    X = X0.clone()
    if args.product_only:
        Acopy = A.clone()          # reads and writes 8 n^2 bytes
        torch.cuda.synchronize()
        del Acopy
        ms = ctx.time_product(X, args.product_reps)
        print(json.dumps({"product_ms": ms, "n": n, "k": k, "precision": main_prec,
                          "slices": slices, "copy_bytes": 8 * n * n}), flush=True)
        ctx.close()
        return 0

    sec_per_step, st1, st_last, X_first = _time_steps(ctx, X, args.steps, args.warmup, torch)
    value = k / sec_per_step

    # dominant kernel: the product W = A X, timed with HIP events on the
    # context's stream, same launch configuration as inside the step
    ms_prod = ctx.time_product(X0.clone(), args.product_reps)
    ctx.close()
    flops = 2.0 * n * n * k
    eff_tflops = flops / (ms_prod * 1e-3) / 1e12
    if main_prec == "fp64":
        roof = {"bound": "mfma", "achieved": eff_tflops, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": eff_tflops / FP64_PEAK_TFLOPS}
    else:
        # INT8 operations actually issued: s(s+1)/2 digit products of 2 n^2 k each
        tops = slices * (slices + 1) / 2 * flops / (ms_prod * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": tops, "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
                "frac": tops / INT8_PEAK_TOPS}
    print("product %.1f us: %.1f eff TFLOP/s" % (ms_prod * 1e3, eff_tflops),
          file=sys.stderr, flush=True)

    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic_gemm_f64_dense_n8192_k64.json")
    if main_prec == "fp64" and os.path.exists(tpath) and (n, k) == (8192, 64):
        try:
            import hashlib
            with open(tpath) as f:
                tj = json.load(f)
            with open(os.path.join(ROOT, "paper_2602_23778_amd", "csrc", "k_gemm.hip"), "rb") as f:
                h = hashlib.sha256(f.read()).hexdigest()
            if tj.get("kernel_source_sha256") == h:
                traffic = tj.get("bytes_per_launch")
        except Exception:
            traffic = None
    roof["traffic"] = traffic

    # the other form on the same workload, for the split-vs-FP64 ratio
    other = None
    if not args.no_split:
        oprec = "fp64" if main_prec == "split_int8" else "split_int8"
        oslices = 0 if oprec == "fp64" else args.slices
        octx = rf.RefineContext(A, k, norm_a=P.norm_a, precision=oprec, slices=oslices)
        Xo = X0.clone()
        osec, ost1, ost_last, Xo_first = _time_steps(octx, Xo, args.steps, args.warmup, torch)
        oms = octx.time_product(X0.clone(), args.product_reps)
        octx.close()
        other = {"precision": oprec, "slices": oslices, "eigvecs_per_s": k / osec,
                 "ms_per_step": osec * 1e3, "product_us": oms * 1e3,
                 "product_eff_gflops": flops / (oms * 1e-3) / 1e9,
                 "corr_fro_last": ost_last.corr_fro}
        s1 = torch.sign((X_first * Xo_first).sum(0))
        other["max_dx_first_step_vs_main"] = float((X_first - Xo_first * s1).abs().max())

    cpu = None
    err = None
    if not args.no_cpu_baseline:
        import oracle
        A_h = A.cpu().numpy()
        X0_h = X0.cpu().numpy()
        ts = time.perf_counter()
        r = oracle.refine_step(A_h, X0_h, norm_a=P.norm_a)
        t_cpu = time.perf_counter() - ts
        g = X_first.cpu().numpy()
        s = np.sign(np.sum(g * r.X, 0))
        err = float(np.max(np.abs(g * s - r.X)))
        cpu = {"value": k / t_cpu, "unit": "eigvecs/s", "cores": _cores(), "kind": "oracle",
               "sample": "one full FP64 oracle step of the same workload (n=%d, k=%d), %.1f s"
                         % (n, k, t_cpu)}

    split_block = None
    if other is not None:
        if main_prec == "fp64":
            split_block = dict(other)
            split_block["speed_ratio_split_over_fp64"] = other["eigvecs_per_s"] / value
        else:
            split_block = {"fp64": other,
                           "speed_ratio_split_over_fp64": value / other["eigvecs_per_s"]}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "eigvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_per_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_prec == "fp64" else "i8",
        "data": "synthetic",
        "config": {"workload": ("%s form, " % ("FP64 plain" if main_prec == "fp64" else
                                               "split INT8 s=%d" % slices)) + desc,
                   "n": n, "k": k, "precision": main_prec,
                   "product_us": ms_prod * 1e3,
                   "product_eff_gflops": eff_tflops * 1e3,
                   "err_vs_oracle_first_step": err,
                   "corr_fro_first": st1.corr_fro, "corr_fro_last": st_last.corr_fro,
                   "resid_rel_last": st_last.resid_rel,
                   "split": split_block},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
