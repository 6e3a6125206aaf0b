"""The C-ABI library loads, exports every call declared in include/fmm.h and
rejects invalid arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1206_0115_amd import fmm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"\b(fmm_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_call():
    lib = fmm.lib()
    names = declared_functions()
    assert "fmm_plan" in names and "fmm_evaluate" in names and "fmm_release" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_plan_rejects_bad_arguments_without_device():
    lib = fmm.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: checks come first
    assert not lib.fmm_plan(None, 10, 3, 5)
    assert "NULL" in fmm.last_error()
    assert not lib.fmm_plan(fake, 0, 3, 5)
    assert "n must be" in fmm.last_error()
    assert not lib.fmm_plan(fake, 10, 0, 5)
    assert not lib.fmm_plan(fake, 10, 22, 5)
    assert "height" in fmm.last_error()
    assert not lib.fmm_plan(fake, 10, 3, 0)
    assert not lib.fmm_plan(fake, 10, 3, 13)
    assert "order" in fmm.last_error()


def test_calls_reject_null_plan():
    lib = fmm.lib()
    fake = ctypes.c_void_p(0x1000)
    assert lib.fmm_evaluate(None, fake, fake, fake, None) == fmm.FMM_ERR_ARG
    assert lib.fmm_evaluate_parts(None, fake, fake, fake, fake, fake, None) == fmm.FMM_ERR_ARG
    assert lib.fmm_plan_set_precision(None, 0) == fmm.FMM_ERR_ARG
    assert lib.fmm_plan_set_schedule(None, fmm.FMM_SCHEDULE_SERIAL) == fmm.FMM_ERR_ARG
    assert lib.fmm_plan_set_kernel(None, fmm.FMM_KERNEL_INV_R2) == fmm.FMM_ERR_ARG
    assert lib.fmm_plan_set_near(None, fmm.FMM_NEAR_MUTUAL) == fmm.FMM_ERR_ARG
    assert lib.fmm_plan_set_near(fake, 2) == fmm.FMM_ERR_ARG  # mode checked before the plan is touched
    assert "near-field mode" in fmm.last_error()
    assert lib.fmm_plan_set_m2l_fold_interval(None, 4) == fmm.FMM_ERR_ARG
    assert lib.fmm_plan_set_m2l_split(None, 2) == fmm.FMM_ERR_ARG
    assert lib.fmm_plan_m2l_split(None, None) == fmm.FMM_ERR_ARG
    assert lib.fmm_set_step_timing_events(9, None, None) == fmm.FMM_ERR_ARG
    assert lib.fmm_set_step_timing_events(fmm.FMM_TIME_LOC_SUM + 1, None, None) == fmm.FMM_ERR_ARG
    assert lib.fmm_set_step_timing_events(-1, None, None) == fmm.FMM_ERR_ARG
    for step in fmm.TIMED_STEPS.values():
        assert lib.fmm_set_step_timing_events(step, None, None) == fmm.FMM_OK
    assert lib.fmm_set_step_timing_events(fmm.FMM_TIME_P2P, fake, None) == fmm.FMM_ERR_ARG
    assert lib.fmm_set_step_timing_events(fmm.FMM_TIME_P2P, None, None) == fmm.FMM_OK
    assert lib.fmm_plan_info(None, None) == fmm.FMM_ERR_ARG
    assert lib.fmm_plan_export(None, 0, 0, fake, 8) == fmm.FMM_ERR_ARG
    assert lib.fmm_set_m2l_timing_events(fake, None) == fmm.FMM_ERR_ARG
    lib.fmm_release(None)  # NULL-safe


def test_info_struct_layout_matches_header():
    src = open(os.path.join(ROOT, "include", "fmm.h")).read()
    body = src[src.index("struct fmm_info {"):]
    body = body[:body.index("};")]
    fields = re.findall(r"(int64_t|int32_t|double)\s+([^;]+);", body)
    names = []
    for _, decl in fields:
        for part in decl.split(","):
            names.append(re.sub(r"\[.*\]", "", part).strip())
    assert names == [f[0] for f in fmm.FmmInfo._fields_]


def test_direct_sampled_rejects_bad_arguments_without_device():
    lib = fmm.lib()
    fake = ctypes.c_void_p(0x1000)
    args = lambda **kw: [kw.get(k, d) for k, d in (
        ("pos", fake), ("q", fake), ("n", 10), ("t", fake), ("nt", 4),
        ("kernel", fmm.FMM_KERNEL_INV_R), ("phi", fake), ("f", fake), ("s", None))]
    assert lib.fmm_direct_sampled(*args(pos=None)) == fmm.FMM_ERR_ARG
    assert "NULL" in fmm.last_error()
    assert lib.fmm_direct_sampled(*args(t=None)) == fmm.FMM_ERR_ARG
    assert lib.fmm_direct_sampled(*args(n=0)) == fmm.FMM_ERR_ARG
    assert lib.fmm_direct_sampled(*args(nt=0)) == fmm.FMM_ERR_ARG
    assert lib.fmm_direct_sampled(*args(kernel=3)) == fmm.FMM_ERR_ARG
    assert "kernel" in fmm.last_error()


def test_precision_enum_matches_header():
    src = open(os.path.join(ROOT, "include", "fmm.h")).read()
    body = src[src.index("enum fmm_precision {"):]
    body = re.sub(r"/\*.*?\*/", "", body[:body.index("};")], flags=re.S)
    vals = dict((k, int(v)) for k, v in re.findall(r"(FMM_\w+)\s*=\s*(\d+)", body))
    assert vals == {"FMM_FP64": fmm.FMM_FP64, "FMM_MIXED_FP32": fmm.FMM_MIXED_FP32,
                    "FMM_MIXED_BF16": fmm.FMM_MIXED_BF16, "FMM_FP64_SVD": fmm.FMM_FP64_SVD,
                    "FMM_MIXED_SVD": fmm.FMM_MIXED_SVD}
    assert vals["FMM_MIXED_BF16"] == 2  # the boundary's third mode keeps its value
