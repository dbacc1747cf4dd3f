"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer on
the host, run over ordinary, edge and malformed inputs by a C driver (no GPU):
any out-of-bounds access, leak or undefined operation fails the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no host C compiler")
    exe = str(tmp_path / "oracle_sanitized")
    flags = ["-O1", "-g", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off",
             "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]
    subprocess.check_call([gcc] + flags + [os.path.join(ROOT, "oracle", "wcsim_oracle.c"),
                                           os.path.join(HERE, "oracle_sanitize_driver.c"),
                                           "-o", exe, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitized oracle run ok" in r.stdout
    assert "runtime error" not in r.stderr


def test_library_host_code_under_sanitizers(tmp_path):
    """libwcsim rebuilt with AddressSanitizer and UndefinedBehaviorSanitizer on
    its host code only (the device code is unchanged), driven through the C
    ABI on malformed arguments by a C++ driver built with the same compiler:
    every call is rejected on the host, with no sanitizer report."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    clangxx = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(hipcc) or not os.path.exists(clangxx):
        pytest.skip("ROCm compilers not available")
    from paper_2304_01841_amd import build as B

    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src in B.SRC:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.check_call([hipcc] + [f for f in B.HIPCC_FLAGS if f != "-shared"] + san +
                              ["-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj])
        objs.append(obj)
    lib = str(tmp_path / "libwcsim_san.so")
    subprocess.check_call([hipcc] + B.HIPCC_FLAGS + san + objs + ["-o", lib])
    exe = str(tmp_path / "lib_sanitized")
    subprocess.check_call([clangxx, "-std=c++17", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
                           os.path.join(HERE, "lib_sanitize_driver.cpp"), lib,
                           "-Wl,-rpath," + str(tmp_path), "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitized library run ok" in r.stdout
    assert "runtime error" not in r.stderr
