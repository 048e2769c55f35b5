"""AddressSanitizer and UndefinedBehaviorSanitizer builds on the CPU.

- The oracle (oracle/kzk_oracle.c) built with gcc -fsanitize=address,undefined
  and driven through every entry point by oracle/sanitize_driver.c.
- The host runtime of libkzk (api.cpp: parameter checks, plan construction
  and its unwinding, status strings) built with the sanitizers on its host
  side only, driven by tests/abi_sanitize_driver.c on a machine without a
  GPU (the kernel launchers come from the built libkzk.so; no kernel runs).
  LeakSanitizer is on: a failed plan creation must release what it built.

Any finding aborts the driver with a non-zero exit status.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-4000:], r.stderr[-4000:])
    return r


def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp"] + SAN +
        ["-o", exe, os.path.join(ROOT, "oracle", "kzk_oracle.c"), os.path.join(ROOT, "oracle", "sanitize_driver.c"),
         "-lm"])
    r = run([exe], env=ENV)
    assert "all results finite" in r.stdout


HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
LIBDIR = os.path.join(ROOT, "paper_2103_06080_amd")


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm toolchain not installed")
def test_host_runtime_under_asan_and_ubsan(tmp_path):
    if not os.path.exists(os.path.join(LIBDIR, "libkzk.so")):
        pytest.skip("libkzk.so not built")
    obj, drv, exe = str(tmp_path / "api_san.o"), str(tmp_path / "drv.o"), str(tmp_path / "abi_san")
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f]
    run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + host_san +
        ["-c", os.path.join(LIBDIR, "csrc", "api.cpp"), "-o", obj])
    run([CLANG, "-O1", "-g"] + SAN + ["-c", os.path.join(ROOT, "tests", "abi_sanitize_driver.c"), "-o", drv])
    run([CLANG + "++"] + SAN[:1] + ["-o", exe, drv, obj, "-L" + LIBDIR, "-l:libkzk.so", "-Wl,-rpath," + LIBDIR,
                                    "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    r = run([exe], env=ENV)
    assert "every call returned as documented" in r.stdout
