"""CPU sanitizer runs (AddressSanitizer + UndefinedBehaviorSanitizer) of the
host code: the C oracle, and the host side of the library's C ABI (basis
construction, eigensolvers, workspace queries and every argument check).
The device code is never built with a sanitizer: only api.cpp's host pass
is instrumented, and the drivers make no device call."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{cmd[0]} failed ({r.returncode}):\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc missing")
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", *SAN, "-fopenmp", "-std=c99", os.path.join(HERE, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe])
    r = _run([exe], env=ENV)
    assert "oracle driver ok" in r.stdout


def test_abi_host_code_under_asan_ubsan(tmp_path):
    from paper_1411_2860_amd import build as b
    hipcc = b.hipcc()
    clang = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(clang):
        pytest.skip("ROCm clang++ missing")
    others = [s for s in b.SOURCES if s != "api.cpp"]
    objs = [os.path.join(b.BUILD_DIR, os.path.splitext(s)[0] + ".o") for s in others]
    if not all(os.path.exists(o) for o in objs):
        b.build()
    api_o = str(tmp_path / "api_san.o")
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f]
    _run([hipcc, f"--offload-arch={b.ARCH}", "-O1", "-g", "-std=c++17", "-fPIC", "-x", "hip",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_san,
          "-c", os.path.join(b.CSRC, "api.cpp"), "-o", api_o])
    drv_o = str(tmp_path / "abi_driver.o")
    _run([clang, "-x", "c", "-O1", "-g", *SAN, "-I", os.path.join(ROOT, "include"), "-c",
          os.path.join(HERE, "abi_driver.c"), "-o", drv_o])
    exe = str(tmp_path / "abi_driver")
    _run([clang, *SAN, drv_o, api_o, *objs, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib",
          "-o", exe])
    # the HIP runtime keeps process-lifetime allocations: leaks inside it are
    # not this library's (suppressed by object name)
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libamd_comgr\n")
    env = dict(ENV, LSAN_OPTIONS=f"suppressions={supp}")
    r = _run([exe], env=env)
    assert "abi driver ok" in r.stdout
