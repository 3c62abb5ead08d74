"""Host logic of bench.py that decides what its JSON line reports (CPU only)."""
import hashlib
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture()
def bench(tmp_path, monkeypatch):
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    monkeypatch.setattr(mod, "ROOT", str(tmp_path))
    (tmp_path / "paper_2502_08034_amd" / "csrc").mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    return mod


def write(tmp_path, source, summary):
    (tmp_path / "paper_2502_08034_amd" / "csrc" / "kernels.hip").write_bytes(source)
    if summary is not None:
        (tmp_path / "profiles" / "k_sweep2_slab1024_pmc.md").write_text(summary)


SUMMARY = """# k_sweep2 counters

kernels.hip sha256 at measurement: {sha}

| quantity | value |
|---|---|
| traffic per launch | 4.0566 GB = 15.11 B/cell update |
"""


def test_traffic_read_when_the_source_matches(bench, tmp_path):
    src = b"__global__ void k() {}\n"
    write(tmp_path, src, SUMMARY.format(sha=hashlib.sha256(src).hexdigest()))
    assert bench.counter_traffic() == pytest.approx(4.0566e9)


def test_traffic_dropped_when_the_source_changed(bench, tmp_path):
    src = b"__global__ void k() {}\n"
    write(tmp_path, src + b"// edited\n", SUMMARY.format(sha=hashlib.sha256(src).hexdigest()))
    assert bench.counter_traffic() is None


def test_traffic_absent_without_a_summary(bench, tmp_path):
    write(tmp_path, b"x", None)
    assert bench.counter_traffic() is None
