"""Host logic of bench.py (no GPU): the one-GPU guard and the lookup of the
committed HBM counter summaries, which must give a figure only for the class
they were taken for and only while the kernel's source is unchanged."""
import hashlib
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert p.returncode == 2
    assert "one GPU only" in p.stderr
    assert p.stdout == ""


def _tree(tmp_path, cls, fname, src, src_text, recorded_sha, traffic="1.5e+06"):
    (tmp_path / "profiles").mkdir(exist_ok=True)
    csrc = tmp_path / "paper_2409_09471_amd" / "csrc"
    csrc.mkdir(parents=True, exist_ok=True)
    (csrc / src).write_text(src_text)
    (tmp_path / "profiles" / fname).write_text(
        "# counters\n\n| quantity | value |\n|---|---|\n\n"
        f"- class: {cls}\n- kernel_source_sha256: {recorded_sha}\n- traffic_bytes_per_launch: {traffic}\n")


@pytest.mark.parametrize("wl,cls", [("c2", "contract_f64"), ("c2", "contract_f32"), ("c2", "svd_jacobi"),
                                    ("c5", "contract_f64")])
def test_counter_traffic_follows_class_and_source(bench, tmp_path, monkeypatch, wl, cls):
    fname, src = bench.COUNTER_SUMMARIES[wl][cls]
    text = "__global__ void k() {}\n"
    sha = hashlib.sha256(text.encode()).hexdigest()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # no summary yet
    assert bench.counter_traffic(cls, wl) is None
    # matching class and source
    _tree(tmp_path, cls, fname, src, text, sha)
    assert bench.counter_traffic(cls, wl) == 1.5e6
    # the kernel source changed since the counters were taken
    (tmp_path / "paper_2409_09471_amd" / "csrc" / src).write_text(text + "// edited\n")
    assert bench.counter_traffic(cls, wl) is None
    # a summary recorded for another class is not used
    _tree(tmp_path, "qr", fname, src, text, sha)
    assert bench.counter_traffic(cls, wl) is None
    # a malformed figure is not used
    _tree(tmp_path, cls, fname, src, text, sha, traffic="n/a")
    assert bench.counter_traffic(cls, wl) is None


def test_counter_traffic_unknown_class(bench):
    assert bench.counter_traffic("qr") is None
    assert bench.counter_traffic("contract_f64", "c9") is None
