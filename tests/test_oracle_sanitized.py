"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): oracle/sanitize_driver.c compiles it into one program and runs
every dimension, flux kind, limiter/blending combination, both diffusion
forms and open ends on small problems; any sanitizer report aborts it."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT


def test_oracle_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "orc_sanitized")
    src = os.path.join(ROOT, "oracle", "sanitize_driver.c")
    cmd = [gcc, "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "oracle"),
           src, "-o", exe, "-lm"]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-4000:]
    assert "runtime error" not in r.stdout and "AddressSanitizer" not in r.stdout, r.stdout[-4000:]
    assert "0 failed" in r.stdout
