"""The host code of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer.

engine.hip (every host-side entry point: validation, phases, sizing, layout,
batch assembly) is rebuilt with both sanitizers on its host code and linked
into a shared library that takes the kernels from the built liblbib.so; a
sanitized driver (tests/native/abi_sanitize.cpp) then runs argument
validation, the phase rules, workspace sizing, batch creation and a seeded
stream of malformed inputs through it.  Nothing here needs a GPU: the calls
exercised never reach the HIP runtime.  Any invalid access, leak or undefined
operation aborts the driver.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1907_00080_amd")
LIB = os.path.join(PKG, "liblbib.so")
ROCM = "/opt/rocm"


def _tool(*cands):
    for c in cands:
        if c and os.path.exists(c):
            return c
    return None


def test_host_abi_under_asan_and_ubsan(tmp_path):
    hipcc = _tool(os.path.join(ROCM, "bin", "hipcc"))
    clangxx = _tool(os.path.join(ROCM, "llvm", "bin", "clang++"), os.path.join(ROCM, "lib", "llvm", "bin", "clang++"))
    if hipcc is None or clangxx is None:
        pytest.skip("ROCm compilers not available")
    if not os.path.exists(LIB):
        pytest.skip("liblbib.so not built")
    inc = os.path.join(ROOT, "include")
    obj = str(tmp_path / "engine_san.o")
    san = str(tmp_path / "liblbib_san.so")
    drv = str(tmp_path / "abi_sanitize")
    # host code instrumented; device code as in the product build
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-omit-frame-pointer", "-I", inc, "-c", "-o", obj,
                    os.path.join(PKG, "csrc", "engine.hip")], check=True, capture_output=True)
    subprocess.run([clangxx, "-shared", "-fPIC", "-shared-libasan", "-fsanitize=address,undefined",
                    "-o", san, obj, "-L", PKG, "-llbib", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
                    f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"],
                   check=True, capture_output=True)
    subprocess.run([clangxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-shared-libasan",
                    "-fno-omit-frame-pointer", "-I", inc, "-o", drv,
                    os.path.join(ROOT, "tests", "native", "abi_sanitize.cpp"),
                    "-L", str(tmp_path), "-llbib_san", f"-Wl,-rpath,{tmp_path}"],
                   check=True, capture_output=True)
    rt = subprocess.run([clangxx, "-print-file-name=libclang_rt.asan-x86_64.so"], check=True,
                        capture_output=True, text=True).stdout.strip()
    env = dict(os.environ)
    env["LD_LIBRARY_PATH"] = os.path.dirname(rt) + os.pathsep + env.get("LD_LIBRARY_PATH", "")
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([drv], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
