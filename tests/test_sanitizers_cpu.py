"""Host sanitizer builds, CPU only: the oracle (gcc) and the library's host
side (amdclang; the device code is built as usual, unsanitized) with
AddressSanitizer, LeakSanitizer and UndefinedBehaviorSanitizer, each driven
by a small program over its entry points (tests/sanitize/*_driver.*).  Any
finding aborts the program (-fno-sanitize-recover=all)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/bin/amdclang++"


def _run(exe, env_extra):
    env = dict(os.environ, **env_extra)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert res.returncode == 0, res.stdout + res.stderr[-4000:]
    return res.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "hv_oracle.c"),
                    "-o", exe, "-lm", "-pthread"], check=True)
    assert "oracle driver ok" in _run(exe, {"ASAN_OPTIONS": "detect_leaks=1"})


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="needs the ROCm compilers")
def test_library_host_side_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "libhv_san.so")
    exe = str(tmp_path / "abi_san")
    srcs = sorted(os.path.join(ROOT, "paper_2005_12489_amd", "csrc", f)
                  for f in os.listdir(os.path.join(ROOT, "paper_2005_12489_amd", "csrc")) if f.endswith(".hip"))
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                    "-mcode-object-version=5", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
                    *srcs, "-o", lib], check=True, capture_output=True)
    subprocess.run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", os.path.join(SAN, "abi_driver.cpp"), lib,
                    f"-Wl,-rpath,{tmp_path}", "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib",
                    "-o", exe], check=True)
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=1",
                     "LSAN_OPTIONS": f"suppressions={os.path.join(SAN, 'lsan.supp')}"})
    assert "abi driver ok" in out
