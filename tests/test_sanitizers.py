"""The oracle and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU).

A small C driver calls every whole-image entry point of the oracle on
ragged, strided, tiny and zero-iteration inputs; the oracle source and the
driver are built together with gcc's sanitizers (host code only) and must
run without a report.
"""
import os
import shutil
import subprocess

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not available")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    src = os.path.join(os.path.dirname(oracle.__file__), "fsr_oracle.c")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           src, os.path.join(HERE, "sanitize", "oracle_driver.c"), "-o", str(exe), "-lm"]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr
    assert res.stdout.count("empty") == 4


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="hipcc is not available")
def test_abi_validation_clean_under_asan_and_ubsan(tmp_path):
    """The library's host code built with the sanitizers (host pass only; the
    device code is built as usual) and driven through its validation layer,
    which refuses every call of the driver before any device is touched."""
    from paper_2202_13926_amd import build
    lib = tmp_path / "libfsr_sanitized.so"
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f for f in build.FLAGS if f != "-O3"]
    srcs = [os.path.join(build.CSRC, s) for s in build.SOURCES]
    subprocess.run([build.HIPCC, *flags, "-O1", "-g", *san, *srcs, "-o", str(lib)], check=True,
                   capture_output=True)
    clang = "/opt/rocm/llvm/bin/clang"
    obj = tmp_path / "abi_driver.o"
    exe = tmp_path / "abi_sanitized"
    subprocess.check_call([clang, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", os.path.join(build.ROOT, "include"), "-c",
                           os.path.join(HERE, "sanitize", "abi_driver.c"), "-o", str(obj)])
    subprocess.check_call([clang + "++", "-fsanitize=address,undefined", str(obj), str(lib),
                           "-L/opt/rocm/lib", "-lamdhip64", f"-Wl,-rpath,{tmp_path}",
                           "-Wl,-rpath,/opt/rocm/lib", "-o", str(exe)])
    # leaks: the HIP runtime's own allocations at exit are not this library's
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr
    assert "abi validation clean" in res.stdout
