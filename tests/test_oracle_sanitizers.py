"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): ``oracle/asan_check.c`` drives every entry point of
``fmm_oracle.h`` on small seeded inputs, built with gcc together with
``fmm_oracle.c``; any invalid access, leak or undefined operation ends the
run with a report and a non-zero status."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "asan_check")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-std=c11", "-fopenmp", "-ffp-contract=off", "-I" + ORACLE,
           os.path.join(ORACLE, "asan_check.c"), os.path.join(ORACLE, "fmm_oracle.c"),
           "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    # a library preloaded by the environment may come before the ASan
    # runtime in the link order; that is not a finding of the oracle
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "asan_check: ok" in r.stdout
    assert "Sanitizer" not in r.stderr, r.stderr[-4000:]
