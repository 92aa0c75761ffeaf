"""The C-ABI host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

srtm_api.hip is compiled with host-side ASan + UBSan (-Xarch_host, so no GPU code is
instrumented) and linked with test-only dispatch stand-ins (abi_stub_dispatch.hip) instead of
the kernel objects; the whole host-validation suite (test_abi.py) then runs against that library
with the sanitizer runtime preloaded and halt_on_error set, so any out-of-bounds access, use of
freed memory or undefined behaviour in argument validation, table checks or workspace sizing
fails the run.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2410_00627_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer"]
FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Wno-unused-command-line-argument"]


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_abi_validation_under_host_sanitizers(tmp_path):
    rt = _asan_runtime()
    if not os.path.exists(HIPCC) or rt is None:
        pytest.skip("hipcc or the clang ASan runtime not found")
    api, stub, lib = tmp_path / "api.o", tmp_path / "stub.o", tmp_path / "libsrtm_hostsan.so"
    for src, obj, extra in ((os.path.join(CSRC, "srtm_api.hip"), api, []),
                            (os.path.join(ROOT, "tests", "abi_stub_dispatch.hip"), stub, ["-I" + CSRC])):
        r = subprocess.run([HIPCC, *FLAGS, *SAN, *extra, "-c", src, "-o", str(obj)], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *SAN[:4], str(api), str(stub), "-o", str(lib)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    syms = subprocess.run(["nm", "-D", str(lib)], capture_output=True, text=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms, "the library is not instrumented"
    driver = ("import sys; from paper_2410_00627_amd import srtm; srtm.LIB_PATH = sys.argv[1]; import pytest; "
              "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', sys.argv[2]]))")
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", driver, str(lib), os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
