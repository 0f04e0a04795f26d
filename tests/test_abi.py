"""The C ABI library loads and exports every entry point that include/refine.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="refine.h"):
    with open(os.path.join(ROOT, "include", header)) as f:
        src = f.read()
    names = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(refine_\w+)\s*\(", src, re.M))
    return names


def test_every_header_declares_only_exported_symbols():
    import glob
    import paper_2602_23778_amd as rf
    lib = rf.load_library()
    headers = sorted(os.path.basename(h) for h in glob.glob(os.path.join(ROOT, "include", "*.h")))
    assert "refine.h" in headers and "refine_debug.h" in headers
    for h in headers:
        for n in _declared(h):
            assert hasattr(lib, n), (h, n)
    assert _declared("refine_debug.h") == {"refine_debug_workspace"}


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("refine_init", "refine_step", "refine_run", "refine_destroy", "refine_batch_init",
              "refine_batch_run", "refine_batch_destroy", "refine_status_string",
              "refine_options_default", "refine_get_info"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2602_23778_amd as rf
    lib = rf.load_library()
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(rf.EXPORTS) == _declared()


def test_host_only_entry_points():
    import paper_2602_23778_amd as rf
    o = rf.refine_options()
    rf.refine_options_default(o)
    assert o.delta_c == 10.0 and o.normalize == 1 and o.precision == rf.FP64
    assert "singular" in rf.refine_status_string(rf.EWY_SINGULAR)
    assert rf.refine_status_string(rf.OK) == "ok"
    # FP8 slices are declared and rejected on the host (refine.h)
    o.precision = rf.SPLIT_FP8
    m0 = rf.refine_matrix()
    m0.kind, m0.n, m0.a, m0.lda = rf.DENSE, 10, 1, 10
    assert rf.refine_init(ctypes.c_void_p(), m0, 3, o, None) == rf.EINVAL
    o.precision = rf.FP64
    # invalid arguments are rejected on the host before any device work
    ctx = ctypes.c_void_p()
    m = rf.refine_matrix()
    m.kind, m.n, m.a, m.lda = rf.DENSE, 10, None, 10
    assert rf.refine_init(ctx, m, 3, None, None) == rf.EINVAL
    assert rf.refine_step(None, 0, 0, None) == rf.EINVAL
