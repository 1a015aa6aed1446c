"""Host checks of bench.py's contract (no GPU): the single-GPU guard, and that an
HBM-traffic summary is used only while it belongs to the kernel sources in the tree."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_summaries_are_used_only_while_their_sources_match():
    """bench.py reports `traffic` only while a summary's recorded hash equals the hash
    of the sources it lists; a matching summary must also be plausible: at least the
    algorithmic bytes and at most a quarter above them (no wasted re-reads)."""
    for (workload, prec), name in bench.TRAFFIC_FILES.items():
        path = os.path.join(ROOT, "profiles", name)
        got = bench.measured_traffic(workload, prec)
        if not os.path.exists(path):
            assert got is None
            continue
        fields = bench._summary_fields(path)
        rels = [r.strip() for r in fields.get("kernel_sources", "").split(",") if r.strip()]
        current = bench.sources_sha256(rels) if rels else None
        if current is None or fields.get("kernel_sources_sha256") != current:
            assert got is None, name
        else:
            traffic = float(fields["traffic_bytes_per_launch"])
            alg = float(fields["algorithmic_bytes_per_launch"])
            assert got == traffic
            assert 0.95 * alg <= traffic <= 1.25 * alg, name


def test_measured_traffic_only_for_counted_workloads():
    assert bench.measured_traffic("nls192", "fp64") is None
    assert bench.measured_traffic("dr384", "nonsense") is None


def test_sources_hash_detects_a_change(tmp_path, monkeypatch):
    f = tmp_path / "k.hip"
    f.write_text("a")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h1 = bench.sources_sha256(["k.hip"])
    f.write_text("b")
    assert bench.sources_sha256(["k.hip"]) != h1
    assert bench.sources_sha256(["missing.hip"]) is None
