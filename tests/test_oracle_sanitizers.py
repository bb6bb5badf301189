"""The oracles under the address and undefined-behaviour sanitizers (CPU):
tests/oracle_sanitize_main.c drives every public D2Q9 and D3Q19 oracle call
(all bases and inits, sampling, structure factors, the error paths) over
small lattices; built with gcc and both sanitizers (no recovery), it must
run clean.  gcc only: no GPU code is involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_runs_clean_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitize"
    sanitize = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                "-fno-omit-frame-pointer"]
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-Wall", "-fopenmp", *sanitize,
           "-I", ORACLE, os.path.join(ROOT, "tests", "oracle_sanitize_main.c"),
           os.path.join(ORACLE, "flbref.c"), os.path.join(ORACLE, "flbref3.c"),
           "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    # the sanitizer runtime must be the first library loaded
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
