"""Host logic of bench.py that needs no device: the traffic figure read from
a committed counter summary only while the sources it was measured on are
unchanged, and the refusal of more than one GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _profile(tmp_path, text):
    d = tmp_path / "profiles"
    d.mkdir(exist_ok=True)
    (d / "p.md").write_text(text)


def test_traffic_only_for_the_sources_it_was_measured_on(tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_text("kernel source, first version\n")
    h = bench.sources_sha256([str(src)])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _profile(tmp_path, f"# summary\n\nsources_sha256: {h}\nbytes_per_launch: 431203035\n")
    assert bench.traffic_from_profile("p.md", [str(src)]) == 431203035.0
    # the older key name is read the same way
    _profile(tmp_path, f"kernels_sha256: {h}\nbytes_per_launch: 42010335\n")
    assert bench.traffic_from_profile("p.md", [str(src)]) == 42010335.0
    # a changed source, a missing summary or a malformed figure give none
    src.write_text("kernel source, second version\n")
    assert bench.traffic_from_profile("p.md", [str(src)]) is None
    assert bench.traffic_from_profile("absent.md", [str(src)]) is None
    h2 = bench.sources_sha256([str(src)])
    _profile(tmp_path, f"sources_sha256: {h2}\nbytes_per_launch: n/a\n")
    assert bench.traffic_from_profile("p.md", [str(src)]) is None


def test_hash_covers_every_source_in_order(tmp_path):
    a, b = tmp_path / "a", tmp_path / "b"
    a.write_text("x")
    b.write_text("y")
    assert bench.sources_sha256([str(a), str(b)]) != bench.sources_sha256([str(a)])
    assert bench.sources_sha256([str(a), str(b)]) != bench.sources_sha256([str(b), str(a)])


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
