"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host only, gcc) and run over every exported function on small inputs
(`tests/pins/oracle_sanitize.c`): no out-of-bounds access, use after free,
leak, signed overflow, misaligned or null access on any path, edge cases
included (one agent, coincident agents, agents on the walls)."""
import os
import shutil
import subprocess
from pathlib import Path

import pytest

HERE = Path(__file__).resolve().parent


def test_oracle_under_asan_and_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = tmp_path / "oracle_sanitize"
    cmd = ["gcc", "-std=c11", "-g", "-O1", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           str(HERE / "pins" / "oracle_sanitize.c"), "-o", str(exe), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
