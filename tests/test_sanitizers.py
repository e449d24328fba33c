"""CPU sanitizer job: the FP64 oracle and the library's host code (argument
validation, size queries, launch planning up to the first HIP call) run under
AddressSanitizer and UndefinedBehaviorSanitizer.

1. wmc_oracle.c is rebuilt with gcc -fsanitize=address,undefined
   -fno-sanitize-recover=all and every oracle pin runs against that build.
2. wmc_api.cpp is rebuilt with the sanitizers on its host code only (hipcc,
   -Xarch_host before each -fsanitize), linked with the regular kernel
   objects, and the host-side ABI tests run against that library.

Both runs load the sanitizer runtime into the Python process (LD_PRELOAD)
and fail on the first report.  Leak checking is off: the interpreter itself
keeps allocations until exit.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1903_07189_amd")
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:verify_asan_link_order=0:halt_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run_pytest(args, extra_env, tmp_path):
    env = dict(os.environ)
    env.update(SAN_ENV)
    env.update(extra_env)
    env["PYTHONDONTWRITEBYTECODE"] = "1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu"] + args, cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=900)
    out = r.stdout + r.stderr
    (tmp_path / "run.log").write_text(out)
    assert "ERROR: AddressSanitizer" not in out, out[-4000:]
    assert "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


def test_oracle_pins_under_asan_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "libwmc_oracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fno-fast-math",
                    "-ffp-contract=off", "-std=c99", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    os.path.join(ROOT, "oracle", "wmc_oracle.c"), "-o", lib, "-lm"], check=True)
    out = _run_pytest([os.path.join("tests", "test_oracle_pins.py")],
                      {"WMC_ORACLE_LIB": lib, "LD_PRELOAD": asan}, tmp_path)
    assert " passed" in out


def test_host_code_under_asan_ubsan(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not os.path.exists(hipcc) or not rt:
        pytest.skip("hipcc or clang's AddressSanitizer runtime is not installed")
    from paper_1903_07189_amd import _build
    objs = [os.path.join(_build.BUILD, os.path.splitext(s)[0] + ".o")
            for s in _build.SOURCES if s != "wmc_api.cpp"]
    if not all(os.path.exists(o) for o in objs):
        _build.build()
    api_o = str(tmp_path / "wmc_api_san.o")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    subprocess.run([hipcc, "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-fPIC",
                    "-ffp-contract=off", "-I" + os.path.join(ROOT, "include"),
                    "-I" + os.path.join(PKG, "csrc")] + san +
                   ["-c", os.path.join(PKG, "csrc", "wmc_api.cpp"), "-o", api_o],
                   check=True, capture_output=True)
    lib = str(tmp_path / "libwmc_san.so")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + san[:4] + objs +
                   [api_o, "-o", lib], check=True, capture_output=True)
    out = _run_pytest([os.path.join("tests", "test_abi.py")],
                      {"WMC_LIB": lib, "LD_PRELOAD": rt[-1]}, tmp_path)
    assert " passed" in out
