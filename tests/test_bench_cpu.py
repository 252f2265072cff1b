"""Host-side logic of bench.py (no GPU): the one-GPU guard, the committed
traffic lookup, the per-launch step accounting."""
import os
import re
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_committed_traffic_follows_sources_and_form():
    path = os.path.join(ROOT, "profiles", "step_kernel_hbm_traffic.md")
    text = open(path).read()
    sha = re.search(r"^kernel_src_sha (\S+)$", text, re.M).group(1)
    rows = re.findall(r"^(\S+) traffic_bytes_per_launch (\d+) (\w+):\d+$", text, re.M)
    assert rows
    current = sha == bench.kernel_source_hash()
    for tag, nbytes, kind in rows:
        got = bench.committed_traffic(tag, kind)
        assert got == (int(nbytes) if current else None)
        other = "tile" if kind != "tile" else "march"
        assert bench.committed_traffic(tag, other) is None      # taken on another form
    assert bench.committed_traffic("no_such_workload", "tile") is None


def test_two_step_launches_count_two_steps():
    assert bench.STEPS_PER_LAUNCH == {"march2": 2}
    assert all(bench.STEPS_PER_LAUNCH.get(k, 1) == 1 for k in ("tile", "staged", "march", "march_pairs"))
