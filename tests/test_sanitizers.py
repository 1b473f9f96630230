"""Host code under the address and undefined-behaviour sanitizers (CPU only).

Two drivers are compiled with clang and -fsanitize=address,undefined (no
recovery, so any finding aborts):
  - tests/sanitize/abi_driver.c against the C-ABI layer (sobel4x5_api.cpp,
    host code only; the kernel translation units are replaced by the stubs in
    tests/sanitize/kernel_stubs.cpp, which the argument checks never reach):
    every validation entry point on valid, invalid and overflow-sized
    arguments;
  - tests/sanitize/oracle_driver.c against the oracle (oracle/sobel_oracle.c,
    built without OpenMP): every entry point on tiny and odd shapes under all
    four border rules, and its rejected arguments.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CLANG = "/opt/rocm/llvm/bin/clang"
CLANGXX = "/opt/rocm/llvm/bin/clang++"
SANFLAGS = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=all"]

pytestmark = pytest.mark.skipif(not (os.path.exists(CLANG) and os.path.exists(CLANGXX)),
                                reason="clang from ROCm not found")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s%s" % (" ".join(cmd), r.stdout[-4000:], r.stderr[-4000:])
    return r


def _env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return env


@pytest.fixture(scope="module")
def outdir(tmp_path_factory):
    return tmp_path_factory.mktemp("sanitize")


def test_abi_checks_under_sanitizers(outdir):
    hip_inc = "/opt/rocm/include"
    common = ["-D__HIP_PLATFORM_AMD__", "-I" + hip_inc, "-I" + os.path.join(ROOT, "include")]
    objs = []
    for src, lang in ((os.path.join(ROOT, "paper_2305_00515_amd", "csrc", "sobel4x5_api.cpp"), "c++"),
                      (os.path.join(SAN, "kernel_stubs.cpp"), "c++")):
        obj = str(outdir / (os.path.basename(src) + ".o"))
        _run([CLANGXX, "-std=c++17", "-Wno-unused-result", "-Wno-unused-value"] + SANFLAGS + common +
             ["-c", src, "-o", obj])
        objs.append(obj)
    drv = str(outdir / "abi_driver.o")
    _run([CLANG, "-std=c11"] + SANFLAGS + common + ["-c", os.path.join(SAN, "abi_driver.c"), "-o", drv])
    exe = str(outdir / "abi_driver")
    _run([CLANGXX] + SANFLAGS + [drv] + objs + ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64",
                                                 "-o", exe])
    r = _run([exe], env=_env())
    assert "abi checks ok" in r.stdout


def test_oracle_under_sanitizers(outdir):
    exe = str(outdir / "oracle_driver")
    _run([CLANG, "-std=c11"] + SANFLAGS + [os.path.join(ROOT, "oracle", "sobel_oracle.c"),
                                           os.path.join(SAN, "oracle_driver.c"), "-lm", "-o", exe])
    r = _run([exe], env=_env())
    assert "oracle checks ok" in r.stdout
