"""The host code of libttm (argument validation, size planning, option
resolution, the batch and static-workspace checks) built with
AddressSanitizer and UndefinedBehaviorSanitizer and run without a GPU.

tests/sanitize/host_checks.cpp calls every entry point on seeded random
shapes and on malformed and oversized descriptors; each call returns before
it needs a device.  The sanitizers act on host code only (each -fsanitize=
is passed with -Xarch_host); the device code is compiled as usual.
"""
import concurrent.futures as cf
import hashlib
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2410_19747_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp")
BDIR = os.path.join(ROOT, "_build", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
         "-Xarch_host", "-fno-sanitize-recover=all",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


def _build():
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip")) + [DRIVER]
    h = hashlib.sha256(" ".join(FLAGS).encode())
    for s in srcs + [os.path.join(CSRC, "ttm_internal.h"), os.path.join(ROOT, "include", "ttm.h")]:
        h.update(open(s, "rb").read())
    exe = os.path.join(BDIR, "host_checks_" + h.hexdigest()[:16])
    if os.path.exists(exe):
        return exe
    os.makedirs(BDIR, exist_ok=True)

    def comp(src):
        obj = os.path.join(BDIR, os.path.basename(src) + ".o")
        r = subprocess.run([HIPCC] + FLAGS + ["-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(comp, srcs))
    r = subprocess.run([HIPCC] + FLAGS + objs + ["-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


@pytest.mark.skipif(shutil.which(HIPCC) is None and not os.path.exists(HIPCC), reason="hipcc not available")
def test_host_code_under_asan_and_ubsan():
    exe = _build()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "host_checks: ok" in r.stdout
