"""The tuners' persistent store (REFINE_TUNE_CACHE): a second process with the
same file skips the timing sweeps of the FP64, slice and modular products
(each logs a cache hit) and computes the same step."""
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys, numpy as np, torch
sys.path.insert(0, %r)
import paper_2602_23778_amd as rf, synth
rf.load_library()
P = synth.dense_spectrum(1024, 40, 7300)
A = torch.as_tensor(P.A).cuda()
out = []
for prec in ("fp64", "split_int8", "split_crt"):
    ctx = rf.RefineContext(A, 40, norm_a=1.0, precision=prec)
    X = torch.as_tensor(P.X0).cuda().clone()
    st = ctx.step(X)
    assert st.status == 0
    ctx.close()
    out.append(X.cpu().numpy())
np.save(sys.argv[1], np.stack(out))
""" % ROOT


def _run(tmp_path, tag):
    env = dict(os.environ, REFINE_TUNE_CACHE=str(tmp_path / "tune.txt"), REFINE_LOG="1")
    out = tmp_path / ("x_%s.npy" % tag)
    r = subprocess.run([sys.executable, "-c", SCRIPT, str(out)], env=env, capture_output=True,
                       text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    return r.stderr, np.load(out)


def test_second_process_reads_the_tuning_cache(tmp_path):
    err1, x1 = _run(tmp_path, "first")
    assert "tuning cache hit" not in err1
    lines = (tmp_path / "tune.txt").read_text().splitlines()
    kinds = {ln.split()[1] for ln in lines}
    assert {"gemm_f64", "split", "crt"} <= kinds, lines
    err2, x2 = _run(tmp_path, "second")
    hits = [ln for ln in err2.splitlines() if "tuning cache hit" in ln]
    assert len(hits) >= 3, err2[-2000:]
    # the same launch configurations, so the same results bit for bit
    assert np.array_equal(x1, x2)
