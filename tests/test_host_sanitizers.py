"""Host-side AddressSanitizer and UndefinedBehaviorSanitizer runs (CPU only):

  * the C-ABI layer (csrc/tc_api.cpp, host code only) linked with the
    library's other objects, driven by tests/sanitize/abi_driver.cpp through
    every argument-validation and workspace-sizing path that returns before
    device work;
  * the FP64 oracle (oracle/tc_oracle.c) driven by
    tests/sanitize/oracle_driver.c through every function on tiny ragged
    sizes.

Device code is never built with a sanitizer here.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "sanitize")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="2",
           UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    return r


@pytest.mark.slow
@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang not installed")
def test_abi_layer_under_host_sanitizers():
    from paper_1504_06289_amd import build
    csrc = os.path.join(ROOT, "paper_1504_06289_amd", "csrc")
    objs = [os.path.join(ROOT, "_build", os.path.basename(s) + ".o") for s in build.sources()
            if not s.endswith("tc_api.cpp")]
    if not all(os.path.exists(o) for o in objs):
        build.build()
    os.makedirs(OUT, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", csrc]
    api_o = os.path.join(OUT, "tc_api_san.o")
    # host side of the HIP translation unit only: no device code is compiled
    _run([CLANG, "-x", "hip", "--cuda-host-only", "--offload-arch=gfx950", "-std=c++17",
          *SAN, *inc, "-c", os.path.join(csrc, "tc_api.cpp"), "-o", api_o])
    drv_o = os.path.join(OUT, "abi_driver.o")
    _run([CLANG, "-std=c++17", *SAN, *inc, "-c",
          os.path.join(ROOT, "tests", "sanitize", "abi_driver.cpp"), "-o", drv_o])
    exe = os.path.join(OUT, "abi_driver")
    _run([CLANG, "-fsanitize=address,undefined", drv_o, api_o, *objs, "-L/opt/rocm/lib",
          "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    r = _run([exe], env=ENV, timeout=300)
    assert "all checks passed" in r.stdout


@pytest.mark.slow
@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_host_sanitizers():
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_driver")
    _run(["gcc", "-std=c11", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", *SAN, "-I", os.path.join(ROOT, "oracle"),
          os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "tc_oracle.c"), "-o", exe, "-lm"])
    r = _run([exe], env=ENV, timeout=300)
    assert "all checks passed" in r.stdout
