"""Host AddressSanitizer + UndefinedBehaviorSanitizer run of the C ABI.

Every HIP source of the library is compiled with the sanitizers on its host
pass only (each ``-fsanitize=`` behind ``-Xarch_host``; the gfx950 device code
is built as usual), linked with ``host_abi_check.c`` and run.  The program
calls only host code: argument validation, workspace sizing for every
method/precision/mode, the batched and warm-start layouts, status strings
(including codes outside the enum) and the no-device path of ``cpd_init``.
No GPU is needed; the run fails on any sanitizer report or unmet expectation.
"""
import hashlib
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2006_06281_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
CHECK_SRC = os.path.join(ROOT, "tests", "host_abi_check.c")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"

SAN_HOST = ["-Xarch_host", "-fsanitize=address",
            "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]
HIP_FLAGS = ["-O1", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-mllvm", "-amdgpu-mfma-vgpr-form", *SAN_HOST]


def _inputs():
    files = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                   if f.endswith((".hip", ".hpp")))
    return files + [os.path.join(INCLUDE, "fastcpd.h"), CHECK_SRC]


def _digest():
    h = hashlib.sha256()
    for f in _inputs():
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(HIP_FLAGS).encode())
    return h.hexdigest()[:16]


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(" ".join(cmd) + "\n" + r.stderr[-4000:])


def _build(out):
    os.makedirs(out, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))

    def comp(src):
        obj = os.path.join(out, os.path.basename(src) + ".o")
        _run([HIPCC, *HIP_FLAGS, "-c", src, "-o", obj], out)
        return obj

    with ThreadPoolExecutor(8) as ex:
        objs = list(ex.map(comp, srcs))
    chk = os.path.join(out, "check.o")
    _run([CLANG, "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-fno-omit-frame-pointer", "-I", INCLUDE, "-c", CHECK_SRC, "-o", chk], out)
    exe = os.path.join(out, "host_abi_check")
    _run([HIPCC, "--offload-arch=gfx950", *SAN_HOST, chk, *objs, "-o", exe], out)
    return exe


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                    reason="ROCm hipcc/clang not installed")
@pytest.mark.skipif(os.path.exists("/dev/kfd"),
                    reason="the program's no-device case needs a machine without a GPU")
def test_host_paths_clean_under_asan_ubsan():
    out = os.path.join("/tmp", "fastcpd_host_sanitizers", _digest())
    exe = os.path.join(out, "host_abi_check")
    if not os.path.exists(exe):
        shutil.rmtree(out, ignore_errors=True)
        exe = _build(out)
    env = dict(os.environ)
    # leak checking is off: the HIP runtime keeps process-lifetime allocations
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    log = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in log, log[-4000:]
    assert "runtime error:" not in log, log[-4000:]
    assert r.returncode == 0, log[-4000:]
    assert "all checks passed" in log, log[-4000:]
