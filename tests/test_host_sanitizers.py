"""The library's host code built with AddressSanitizer and UndefinedBehaviorSanitizer (device code
unchanged), driven through every argument check of the C ABI that runs without a GPU
(tests/host_sanitize/abi_checks.cpp): each check returns CGL_E_INVAL with a detail string, and no
sanitizer reports anything. Builds into a temporary directory; the product library is untouched."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2502_09502_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["api.cpp", "batch.cpp", "server.cpp", "eigen.cpp", "noalloc.hip", "kernels_plain.hip",
           "kernels_mfma.hip", "prox_paged.hip", "chol.hip"]
# sanitizers on the host pass only (each -fsanitize= right after -Xarch_host)
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang",
         "-target-feature", "-Xclang", "-packed-fp32-ops"]


@pytest.mark.slow
@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_abi_checks_under_host_sanitizers(tmp_path):
    from concurrent.futures import ThreadPoolExecutor

    def compile_one(src):
        obj = str(tmp_path / (src + ".o"))
        r = subprocess.run([HIPCC, *FLAGS, *SAN, "-x", "hip", "-c", os.path.join(CSRC, src),
                            "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    drv_obj = str(tmp_path / "abi_checks.o")
    r = subprocess.run([HIPCC, *FLAGS, *SAN, "-c",
                        os.path.join(ROOT, "tests", "host_sanitize", "abi_checks.cpp"),
                        "-o", drv_obj], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    drv = str(tmp_path / "abi_checks")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", *SAN, drv_obj, *objs, "-o", drv],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    run = subprocess.run([drv], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, (run.stdout[-3000:], run.stderr[-3000:])
    assert "0 failed" in run.stdout
    assert "ERROR: AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr
