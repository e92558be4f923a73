"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, and
under ThreadSanitizer (CPU).

The host analysis (``csrc/analysis.cpp``: validation, ordering, fronts,
maps, incidences, task order; multithreaded) and its files
(``csrc/analysis_io.cpp``) are compiled with g++ and both sanitizers, linked with the driver ``tests/host_sanitize/analysis_driver.cpp``
and run with leak checking on.  The driver analyses coded-mask shaped and
random patterns, a dense root, empty rows and a single unknown with 1, 3 and
7 threads, checks each result's invariants and that it survives a write and
read of its analysis file unchanged, feeds invalid patterns that must be
refused, and reads 520 damaged copies of one analysis file (each header and
descriptor byte changed in turn, random byte changes, truncations), each of
which must be refused.  An out-of-bounds access, use after free, leak, data
overflow or other undefined operation stops it with the sanitizer's report.
A second build under ThreadSanitizer runs the same multithreaded analyses
(without the damaged files) and fails on any data race.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FLAGS = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
         "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
         "-I" + os.path.join(ROOT, "include")]


def _build(tmp_path, sanitizers):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("g++ or the ROCm headers are missing")
    flags = FLAGS + sanitizers
    exe = str(tmp_path / "analysis_driver")
    csrc = os.path.join(ROOT, "paper_1305_5683_amd", "csrc")
    objs = []
    for name in ("analysis.cpp", "analysis_io.cpp"):
        o = str(tmp_path / (name + ".o"))
        subprocess.run([gxx] + flags + ["-c", os.path.join(csrc, name), "-o", o],
                       check=True, capture_output=True, text=True)
        objs.append(o)
    drv = os.path.join(ROOT, "tests", "host_sanitize", "analysis_driver.cpp")
    subprocess.run([gxx] + flags + [drv] + objs + ["-o", exe, "-lpthread"], check=True,
                   capture_output=True, text=True)
    return exe


@pytest.mark.timeout(900)
def test_host_analysis_under_sanitizers(tmp_path):
    exe = _build(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600,
                       cwd=str(tmp_path))
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "ALL OK" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr


@pytest.mark.timeout(900)
def test_host_analysis_has_no_data_races(tmp_path):
    """The same analyses (1, 3 and 7 threads) under ThreadSanitizer: the
    parallel phases (transpose, counting sorts, chunked groupings, fills by
    range) must share no unsynchronised memory."""
    exe = _build(tmp_path, ["-fsanitize=thread"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe, "threads"], capture_output=True, text=True, env=env,
                       timeout=600, cwd=str(tmp_path))
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "ALL OK" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr
