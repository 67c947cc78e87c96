"""The oracle's C sources built with gcc's AddressSanitizer and
UndefinedBehaviorSanitizer (host code only) and run through every entry
point by tests/sanitize_oracle.c: out-of-bounds accesses, leaks, use after
free, signed overflow, misaligned or null accesses abort the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "sanitize_oracle"
    srcs = [os.path.join(ROOT, "tests", "sanitize_oracle.c"), os.path.join(ROOT, "oracle", "lfr_oracle.c"),
            os.path.join(ROOT, "oracle", "lfr_oracle_grad.c")]
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", str(exe), *srcs, "-lm", "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ)
    # a library preloaded into every process comes before the ASan runtime
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, f"sanitized oracle run failed (rc {r.returncode}):\n{r.stdout}\n{r.stderr[-4000:]}"
    assert "sanitized oracle run ok" in r.stdout
    assert "runtime error" not in r.stderr
