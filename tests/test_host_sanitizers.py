"""The library's host C++ (hierarchy builder kuhn.cpp, sparse kernels sparse_host.cpp,
sliced-ELL layout sell_layout.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, host code only) and run through a driver
(host_sanitize_driver.cpp) that builds H(curl) and H(div) hierarchies with every
builder option and checks the Galerkin products, the layouts, triplet assembly and the
parallel sort against plain references.  Any out-of-bounds access, use after free, leak
or undefined behaviour fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2107_05613_amd", "csrc")
SOURCES = ["kuhn.cpp", "sparse_host.cpp", "sell_layout.cpp"]


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_code_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-pthread", "-o", exe,
           os.path.join(ROOT, "tests", "host_sanitize_driver.cpp")] + [os.path.join(CSRC, s) for s in SOURCES]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout + r.stderr)[-6000:]
    assert "0 failures" in r.stdout
