"""Host-only check of the capacity planner (no GPU): a seed or member total
of 2^32 + k, which the device's uint32 scans would wrap to k, must fail the
call with an overflow instead of fitting a capacity."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1311_5334_amd", "csrc")


def test_capacity_planner_rejects_wrapped_totals(tmp_path):
    exe = str(tmp_path / "capacity_check")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-Wall", "-I" + CSRC,
                           os.path.join(HERE, "native", "capacity_check.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "capacity ok" in r.stdout
