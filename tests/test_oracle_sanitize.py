"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

oracle/sanitize_main.c runs every oracle entry point once on small 2D and 3D problems
(each boundary kind, translation and rotation, terminal cotangents, the coupling
constants, the filter and the cyclic design pairs). Any out-of-bounds access, use after
free, leak or undefined operation aborts the run with a report.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORC = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "orc_sanitize")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-o", exe, os.path.join(ORC, "sanitize_main.c"), os.path.join(ORC, "lks_oracle.c"), "-lm"]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
    assert "all entry points returned 0" in r.stdout
