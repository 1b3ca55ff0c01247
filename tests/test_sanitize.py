"""Host sanitizer runs: the CPU oracle and the host logic of the C ABI built
with AddressSanitizer and UndefinedBehaviorSanitizer (leak checks on), each
driven through its entry points by a small program under tests/sanitize/.
GPU code is never built with a sanitizer: hipcc receives each -fsanitize
option behind -Xarch_host, and the program is linked by the host compiler."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN_ENV = {**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-ffp-contract=off", "-pthread",
          os.path.join(HERE, "sanitize", "oracle_driver.c"), "-o", exe, "-lm"])
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert "oracle sanitizer run ok" in r.stdout


def test_abi_host_logic_under_asan_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/llvm/bin/clang++"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm compilers not installed")
    san = []
    for opt in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
                "-fno-omit-frame-pointer"):
        san += ["-Xarch_host", opt]
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-ffp-contract=off",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *san, "-c", "-x", "hip"]
    objs = []
    for src in (os.path.join(ROOT, "paper_1911_08868_amd", "csrc", "host.cpp"),
                os.path.join(HERE, "sanitize", "abi_host_driver.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([hipcc, *common, src, "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "abi_host_driver")
    _run([clang, "-fsanitize=address,undefined", *objs, "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert "abi host sanitizer run ok" in r.stdout
