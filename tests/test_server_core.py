"""The served form's host-side scheduling (server_core.hpp: arena,
admission, completions, stop, several waiters on one request), built from
the same header the library uses and run against a simulated device, under
AddressSanitizer + UndefinedBehaviorSanitizer and under ThreadSanitizer
(host code only; no GPU)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "server_core_test.cpp")


def _build_and_run(tmp_path, flags, which):
    exe = tmp_path / ("sct_" + "_".join(f.strip("-").replace("=", "_").replace(",", "_") for f in flags))
    cmd = ["g++", "-std=c++17", "-g", "-O1", "-pthread", "-fno-omit-frame-pointer", *flags,
           "-I", os.path.join(ROOT, "include"), SRC, "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1",
               TSAN_OPTIONS="halt_on_error=1")
    res = subprocess.run([str(exe), which], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "passed" in res.stdout


def test_server_core_asan_ubsan(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"], "all")


def test_server_core_tsan(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=thread"], "threads")
