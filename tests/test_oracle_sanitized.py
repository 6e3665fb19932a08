"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host code, gcc).

The driver ``oracle_sanitize_main.c`` includes the oracle's source and calls every public
entry point on small problems of each dimension 1..4, each flux family (advection, Burgers,
phase-space Vlasov), both prolongation modes and both time-step rules.  Memory errors, leaks
and undefined behaviour abort the run.  OpenMP is left out of this build so that the
sanitizers see the serial loops.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
           os.path.join(HERE, "oracle_sanitize_main.c"), "-o", exe, "-lm"]
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0 and "asan" in (b.stderr or "").lower():
        pytest.skip("the sanitizer runtime is not installed: " + b.stderr[-300:])
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "SANITIZED RUN OK" in r.stdout
