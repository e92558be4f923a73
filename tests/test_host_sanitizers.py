"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

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
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FLAGS = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
         "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
         "-I" + os.path.join(ROOT, "include")]


@pytest.mark.timeout(900)
def test_host_analysis_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("g++ or the ROCm headers are missing")
    exe = str(tmp_path / "analysis_driver")
    csrc = os.path.join(ROOT, "paper_1305_5683_amd", "csrc")
    objs = []
    for name in ("analysis.cpp", "analysis_io.cpp"):
        o = str(tmp_path / (name + ".o"))
        subprocess.run([gxx] + FLAGS + ["-c", os.path.join(csrc, name), "-o", o],
                       check=True, capture_output=True, text=True)
        objs.append(o)
    drv = os.path.join(ROOT, "tests", "host_sanitize", "analysis_driver.cpp")
    subprocess.run([gxx] + FLAGS + [drv] + objs + ["-o", exe, "-lpthread"], check=True,
                   capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600,
                       cwd=str(tmp_path))
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "ALL OK" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr
