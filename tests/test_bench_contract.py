"""Host logic of bench.py (no GPU): the measured raster traffic and counters
stay valid across comment edits of the kernel source and are reported as null
once its code changes; more than one GPU is refused with a message."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_code_digest_ignores_comments_and_blank_lines(tmp_path):
    B = _bench()
    a = tmp_path / "a.hip"
    a.write_text("int f(int x) {  // doubles\n  return 2 * x;\n}\n")
    b = tmp_path / "b.hip"
    b.write_text("// a header comment\n\nint f(int x) {\n  return 2 * x;   // twice\n}\n\n")
    c = tmp_path / "c.hip"
    c.write_text("int f(int x) {\n  return 3 * x;\n}\n")
    assert B.code_digest(str(a)) == B.code_digest(str(b))
    assert B.code_digest(str(a)) != B.code_digest(str(c))


def test_traffic_is_reported_only_for_the_measured_source(tmp_path, monkeypatch):
    """A changed kernel source makes the bench report traffic as null."""
    B = _bench()
    src = tmp_path / "paper_2412_03489_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "hr_edges.hip").write_text("int g() { return 1; }\n")
    monkeypatch.setattr(B, "ROOT", str(tmp_path))
    assert B.raster_traffic() is None
    assert B.raster_counters() is None
    monkeypatch.setattr(B, "TRAFFIC_SOURCE_DIGEST", B.code_digest(str(src / "hr_edges.hip")))
    assert B.raster_traffic() == B.TRAFFIC_BYTES_PER_LAUNCH
    assert B.raster_counters() == B.COUNTERS_PER_LAUNCH


def test_gradient_counters_only_for_the_measured_source(tmp_path, monkeypatch):
    B = _bench()
    src = tmp_path / "paper_2412_03489_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "hr_raster.hip").write_text("int h() { return 2; }\n")
    monkeypatch.setattr(B, "ROOT", str(tmp_path))
    assert B.gradient_counters() is None
    monkeypatch.setattr(B, "GRADIENT_SOURCE_DIGEST", B.code_digest(str(src / "hr_raster.hip")))
    assert B.gradient_counters() == B.GRADIENT_COUNTERS_PER_LAUNCH


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
