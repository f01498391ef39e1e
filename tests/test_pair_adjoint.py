"""The adjoint's reverse sweep over a pair's geometry (pair_gradient in
csrc/pair_adjoint.hpp, the code the pair_grad kernel runs) against
forward-mode dual numbers through the same pencil / line-map templates, on
the host: object-sphere and detector-bounded ranges (arc ends at corners),
near-opposed views, a sphere wider than the baseline's distance and a
baseline through the isocentre.  No GPU."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "pair_adjoint_test.cpp")


def test_pair_gradient_reverse_equals_forward_mode(tmp_path):
    exe = tmp_path / "pair_adjoint_test"
    cmd = ["/opt/rocm/bin/hipcc", "-std=c++17", "-O1", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           SRC, "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "passed" in res.stdout
