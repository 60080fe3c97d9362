"""Host logic of bench.py, on the CPU: the source digest that keys the committed
HBM-traffic counters to the kernel code, the lookup of those counters, and the
single-GPU guard."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_source_digest_ignores_comments_and_blank_lines(tmp_path):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text("// header\nint f(int x) {\n  return x + 1;   // add one\n}\n")
    b.write_text("/* another\n   header */\n\nint f(int x) {\n\n  return x + 1;\n}\n")
    c.write_text("int f(int x) {\n  return x + 2;\n}\n")
    assert bench.source_digest(str(a)) == bench.source_digest(str(b))
    assert bench.source_digest(str(a)) != bench.source_digest(str(c))


def test_traffic_line_matches_the_lattice_kernel_source():
    """The committed counters were taken on the lattice kernel as it is now:
    read + written bytes between the algorithmic 268 MB and twice that."""
    t = bench.measured_traffic("fdm_lattice")
    assert t is not None
    assert 268435456 <= t <= 2 * 268435456


def test_traffic_lookup_rejects_other_code(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    src = tmp_path / "k.hip"
    src.write_text("int g() { return 3; }\n")
    good = bench.source_digest(str(src))
    (prof / "k.md").write_text(
        "    traffic family=fam source=k.hip code_sha256=%s fetch_bytes=10 write_bytes=20\n" % good)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("fam") == 30
    assert bench.measured_traffic("other") is None
    src.write_text("int g() { return 4; }\n")   # the kernel changed since the counters
    assert bench.measured_traffic("fam") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
