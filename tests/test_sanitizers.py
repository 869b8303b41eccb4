"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle (plain C) is built with gcc and both sanitizers and driven through
every entry point on small problems of every kind; the library is built with
the sanitizers on its host code only (the device code is compiled as usual)
and driven through the entry points that need no device: problem validation
and the planning arithmetic behind bsde_problem_info, the quadrature and
gamma tables, the status strings.  Both drivers exit 0 only when every call
returns as expected; the sanitizers abort on the first invalid access or
undefined operation.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1909_13560_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, **kw)


def test_oracle_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_asan")
    r = _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer", "-o", exe, os.path.join(HERE, "oracle_driver.c"),
              os.path.join(ROOT, "oracle", "bsde_oracle.c"), "-lm"])
    assert r.returncode == 0, r.stderr
    r = _run([exe], timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all calls ok" in r.stdout


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    clang = os.path.join(ROCM, "llvm", "bin", "clang")
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm compilers not available")
    lib = str(tmp_path / "libbsde_asan.so")
    srcs = [os.path.join(CSRC, f)
            for f in ("capi.hip", "sweep.hip", "sweep2d.hip", "toeplitz.hip", "plan_math.cpp")]
    # sanitizers on the host code only: each -fsanitize= after -Xarch_host
    r = _run([hipcc, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-o", lib, *srcs])
    assert r.returncode == 0, r.stderr[-4000:]
    exe = str(tmp_path / "host_asan")
    r = _run([clang, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              "-o", exe, os.path.join(HERE, "host_driver.c"), lib, f"-Wl,-rpath,{tmp_path}",
              "-lm"])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")  # the HIP runtime keeps its globals
    r = _run([exe], timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all calls ok" in r.stdout
