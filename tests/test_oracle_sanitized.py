"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): oracle/sanitize_check.c drives every oracle entry point on seeded
inputs and checks input-independent invariants; built with the sanitizers,
any out-of-bounds access, use after free, leak or undefined operation in the
oracle aborts it."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORC = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "sanitize_check")
        cmd = ["gcc", "-O1", "-g", "-std=c11", "-Wall", "-Wextra", "-Werror",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-fno-omit-frame-pointer", "-static-libasan", "-o", exe,
               os.path.join(ORC, "sanitize_check.c"), os.path.join(ORC, "gvom_oracle.c"),
               os.path.join(ORC, "sgt_oracle.c"), "-lm"]
        subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
        env = dict(os.environ)
        env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=1:verify_asan_link_order=0"
        env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        assert r.returncode == 0, r.stdout + r.stderr
        assert r.stdout.strip() == "ok"
