"""The oracle's worker threads under ThreadSanitizer (CPU): the threaded trace of a small
scene runs race-free and gives the single-thread result (the paper's Section 3 relies on
thread-safe access to shared output; here every worker owns its output copy)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "oracle_threads_driver.c")


def test_threaded_oracle_is_race_free(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = tmp_path / "oracle_threads"
    flags = ["-O1", "-g", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math", "-pthread",
             "-fsanitize=" + "thread"]
    subprocess.check_call(["gcc", *flags, "-o", str(exe), DRIVER, "-lm"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ThreadSanitizer" not in r.stderr, r.stderr
    assert "ok: 1 and 6 threads agree" in r.stdout
