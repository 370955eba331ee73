"""Host-side AddressSanitizer / UndefinedBehaviorSanitizer runs (CPU only).

The library's host code (the C-ABI layer of hub_api.hip with its argument
checks, and the sphere / work-list builder sphere.cpp) is rebuilt with
ASan and UBSan for the host only (the device code is not instrumented) and
linked with the kernels' objects of the regular build.  test_abi.py then
runs against that build in a child process with the sanitizer runtime
preloaded: every entry point it drives (context set-up, host tables,
queries, sphere points, radius selection and the argument errors) must
finish without a sanitizer report.  The state-gradient table checker of
test_host_stencil.py is run under the same sanitizers there."""

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1711_08935_amd")
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
OUT = os.path.join(BUILD, "asan")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = "/opt/rocm/llvm/bin/clang++"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _runtime():
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return libs[-1] if libs else None


@pytest.fixture(scope="module")
def asan_lib():
    if not (os.path.exists(HIPCC) and os.path.exists(CLANGXX) and _runtime()):
        pytest.skip("hipcc / clang++ / the clang ASan runtime are not available")
    kernels = sorted(glob.glob(os.path.join(BUILD, "k_*.hip.o")))
    if not kernels:
        sys.path.insert(0, ROOT)
        from paper_1711_08935_amd.build import build
        build()
        kernels = sorted(glob.glob(os.path.join(BUILD, "k_*.hip.o")))
    os.makedirs(OUT, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    api = os.path.join(OUT, "hub_api.o")
    sph = os.path.join(OUT, "sphere.o")
    lib = os.path.join(OUT, "libhub_asan.so")
    subprocess.run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
                    "-Xclang", "-packed-fp32-ops", *SAN, *inc, "-c", os.path.join(CSRC, "hub_api.hip"), "-o", api],
                   check=True, capture_output=True)
    subprocess.run([CLANGXX, "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off", *SAN, *inc, "-c",
                    os.path.join(CSRC, "sphere.cpp"), "-o", sph], check=True, capture_output=True)
    subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined", api, sph, *kernels, "-o", lib], check=True,
                   capture_output=True)
    return lib


def test_abi_under_host_sanitizers(asan_lib):
    env = dict(os.environ, HUB_LIBRARY=asan_lib, LD_PRELOAD=_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "passed" in out
    for marker in ("ERROR: AddressSanitizer", "runtime error:", "SUMMARY: UndefinedBehaviorSanitizer"):
        assert marker not in out, out[-4000:]
