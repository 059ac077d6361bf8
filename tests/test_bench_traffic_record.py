"""bench.py's rule for roofline.traffic on the CPU: the recorded HBM bytes
of the spread are reported only while the kernel source's SHA-256 and the
workload settings match the record, and are null otherwise. Runs against a
temporary profile record and source file, not the committed ones."""
import argparse
import hashlib
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _args(**kw):
    a = dict(config=2, precision="fp32", kernel="kaiser_bessel", sigma_xy=1.5, width_xy=8, sigma_t=1.25, width_t=10)
    a.update(kw)
    return argparse.Namespace(**a)


def _setup(tmp_path):
    src = tmp_path / "kernel.hip"
    src.write_text("// kernel source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "k_spread_traffic_test.md").write_text(
        "summary text\n\nrecord: kernel=k_spread source=kernel.hip sha256=" + sha + " config=2 precision=fp32 "
        "kernel_kind=kaiser_bessel sigma_xy=1.5 width_xy=8 sigma_t=1.25 width_t=10 band_bins=575 "
        "traffic_bytes_per_launch=123456789\n")
    return src


def test_record_used_while_source_and_settings_match(tmp_path, monkeypatch):
    b = _bench()
    _setup(tmp_path)
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.recorded_traffic(_args(), 575) == 123456789


def test_record_ignored_after_a_source_change(tmp_path, monkeypatch):
    b = _bench()
    src = _setup(tmp_path)
    src.write_text("// kernel source, edited\n")
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.recorded_traffic(_args(), 575) is None


def test_record_ignored_for_other_settings(tmp_path, monkeypatch):
    b = _bench()
    _setup(tmp_path)
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.recorded_traffic(_args(width_xy=12), 575) is None
    assert b.recorded_traffic(_args(precision="fp64"), 575) is None
    assert b.recorded_traffic(_args(), 574) is None
