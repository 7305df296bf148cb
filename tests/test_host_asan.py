"""The library's host code built with AddressSanitizer (host side only; the GPU code is
compiled as usual) and driven on the CPU by tests/asan/host_driver.cpp: validation,
sizing and refusal paths over a grid of valid and invalid problems must run without an
AddressSanitizer report."""
import concurrent.futures as cf
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2406_00952_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
         "-I", os.path.join(ROOT, "include")]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_host_code_under_asan():
    d = tempfile.mkdtemp(prefix="wc_asan_")
    try:
        srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))

        def comp(src):
            out = os.path.join(d, src + ".o")
            r = subprocess.run([HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", out],
                               capture_output=True, text=True)
            assert r.returncode == 0, r.stderr[-2000:]
            return out

        with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
            objs = list(ex.map(comp, srcs))
        drv = os.path.join(d, "driver.o")
        r = subprocess.run([HIPCC, *FLAGS, "-c", os.path.join(ROOT, "tests", "asan",
                                                              "host_driver.cpp"), "-o", drv],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        exe = os.path.join(d, "driver")
        r = subprocess.run([HIPCC, "-Xarch_host", "-fsanitize=address", "--offload-arch=gfx950",
                            drv, *objs, "-o", exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
        assert "bad 0" in r.stdout
        assert "AddressSanitizer" not in r.stderr
    finally:
        shutil.rmtree(d, ignore_errors=True)
