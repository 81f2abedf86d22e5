"""CPU check of the contraction planner with an emulated GETT (no GPU)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2103_08473_amd", "csrc")


def test_planner_specs_match_direct_loops(tmp_path):
    exe = str(tmp_path / "planner_harness")
    cmd = ["/opt/rocm/bin/hipcc", "-O1", "-std=c++17", "-I" + CSRC, "-I" + os.path.join(ROOT, "include"),
           os.path.join(HERE, "planner_harness.cpp"), os.path.join(CSRC, "einsum.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-2000:]
    assert "0 failures" in r.stdout
