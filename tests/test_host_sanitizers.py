"""The library's host code under sanitizers, on the CPU: the C++ of the C ABI
(validation, tree planner, plan and batch caches, workspace layouts, tuning
table, fault hook) built with address + undefined-behaviour (and leak)
checking, and separately with the thread sanitizer, into a driver program
(tests/host_sanitize_driver.cpp) that calls only what runs on the host.  The
kernels' objects are linked in unchanged and never launched."""
import os
import shutil
import subprocess

import pytest

from paper_1307_7852_amd import build_lib as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "host_sanitize_driver.cpp")

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not on PATH")


def _kernel_objects():
    objs = []
    for src in B.SOURCES:
        if src.endswith(".hip"):
            os.makedirs(B.OBJ, exist_ok=True)
            _, rc, err, obj = B._compile(src, force=False)
            assert rc == 0, err
            objs.append(obj)
    return objs


def _build(tmp_path, name, san_flags):
    exe = str(tmp_path / name)
    cmd = (["hipcc", "-x", "hip", "--offload-arch=gfx950", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-g",
            "-O1"] + san_flags + [os.path.join(B.SRC, "knng_api.cpp"), "-x", "c++", DRIVER, "-x", "none"]
           + _kernel_objects() + ["-o", exe])
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def test_host_code_address_and_ub_sanitizers(tmp_path):
    exe = _build(tmp_path, "drv_asan", ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                                        "-Xarch_host", "-fno-sanitize-recover=undefined",
                                        "-Xarch_host", "-fno-omit-frame-pointer"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("KNNG_FAULT", None)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "host checks passed" in r.stdout


def test_host_code_thread_sanitizer(tmp_path):
    exe = _build(tmp_path, "drv_tsan", ["-Xarch_host", "-fsanitize=thread"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
    env.pop("KNNG_FAULT", None)
    r = subprocess.run([exe, "threads"], capture_output=True, text=True, timeout=900, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "host checks passed" in r.stdout
