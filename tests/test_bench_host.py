"""bench.py host logic (no GPU): the measured HBM traffic of a kernel is
reported only while the sources it was measured on are unchanged, and more
than one GPU is refused before anything touches a device."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _copy_sources(tmp_path, monkeypatch):
    d = tmp_path / "csrc"
    shutil.copytree(bench.CSRC, d)
    monkeypatch.setattr(bench, "CSRC", str(d))
    return d


@pytest.mark.parametrize("kernel", ["bulk", "assembly"])
def test_traffic_follows_the_measured_sources(kernel, tmp_path, monkeypatch):
    d = _copy_sources(tmp_path, monkeypatch)
    key = next(k for k in bench.HBM_COUNTERS if k[1] == kernel)
    entry = bench.HBM_COUNTERS[key]
    # pretend the counters were taken on the sources as they are now
    monkeypatch.setitem(bench.HBM_COUNTERS, key,
                        dict(entry, src=bench.src_hash(bench.SRC_SECTIONS[kernel])))
    assert bench.counter_traffic(*key) == entry["bytes"]
    name, begin, end = bench.SRC_SECTIONS[kernel][0]
    path = d / name
    text = path.read_text()
    # a change outside the measured section keeps the figure
    path.write_text(text + "\n// a comment after everything\n" if begin is not None
                    else text)
    if begin is not None:
        assert bench.counter_traffic(*key) == entry["bytes"]
    # a change inside it withdraws the figure
    i = text.index(begin) + len(begin) if begin is not None else 0
    path.write_text(text[:i] + "\n// changed\n" + text[i:])
    assert bench.counter_traffic(*key) is None


def test_unmeasured_configuration_has_no_traffic():
    assert bench.counter_traffic(2, "bulk", 256, "fp64") is None
    assert bench.counter_traffic(1, "bulk", 512, "mixed") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
