"""Host checks of bench.py's contract (no GPU): the single-GPU guard, and that the
committed HBM-traffic summary belongs to the kernel sources in the tree."""

import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_summary_matches_the_kernel_sources():
    """bench.py reports `traffic` only while the summary's hash equals the hash of the
    kernel sources; a kernel change without new counters must show up here."""
    r = _run("--kernel-sources-sha256")
    assert r.returncode == 0
    sha = r.stdout.strip()
    assert re.fullmatch(r"[0-9a-f]{64}", sha)
    text = open(os.path.join(ROOT, "profiles", "k_modes12_adr128_hbm_traffic.md")).read()
    fields = dict(l.strip().split(" = ", 1) for l in text.splitlines() if " = " in l)
    assert fields["kernel_sources_sha256"] == sha
    traffic = float(fields["traffic_bytes_per_launch"])
    alg = float(fields["algorithmic_bytes_per_launch"])
    assert alg <= traffic <= 1.25 * alg  # no wasted re-reads beyond a quarter of the algorithmic bytes


def test_measured_traffic_only_for_the_counted_workload():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.measured_traffic("adr128") is not None
    assert bench.measured_traffic("dr384") is None
