"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only, gcc) and run over every exported function on small
buffered 2D and 3D cases (tests/oracle_sanitize_main.c): no out-of-bounds
access, leak, use after free, signed overflow or other undefined behaviour
in the reference itself.  Built without OpenMP, so the run is sequential."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-Wno-unknown-pragmas", "-o", exe, os.path.join(HERE, "oracle_sanitize_main.c"),
           os.path.join(ROOT, "oracle", "sph_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr
    assert "oracle sanitizer run ok" in r.stdout
