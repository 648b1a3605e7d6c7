"""libqtn's host code under AddressSanitizer and ThreadSanitizer, on the
CPU: the planner, the workspace layout, the launch logic, the autotuner,
ranges with checkpoints, the no-allocation and batched entry points, general
circuits and the density-matrix form, driven through the C ABI with the HIP
runtime replaced by CPU stand-ins (tests/host_asan); and the thread pool of
the exact cost evaluation.  No device code runs."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ASAN_DIR = os.path.join(HERE, "host_asan")


def _libasan():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    except OSError:
        return None
    return p if p and os.path.isabs(p) and os.path.exists(p) else None


def test_host_code_under_address_sanitizer():
    if not os.path.isdir(ASAN_DIR):
        pytest.skip("host sanitizer harness not present")
    asan = _libasan()
    if asan is None or shutil.which("g++") is None or not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("g++, libasan or hipcc not available")
    import importlib.util
    spec = importlib.util.spec_from_file_location("qtn_host_asan_build", os.path.join(ASAN_DIR, "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    lib = mod.build()
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    r = subprocess.run([sys.executable, os.path.join(ASAN_DIR, "drive.py"), lib], capture_output=True,
                       text=True, env=env, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert out.rstrip().endswith("done") or "\ndone" in out, out[-2000:]


def _load_build():
    import importlib.util
    spec = importlib.util.spec_from_file_location("qtn_host_asan_build", os.path.join(ASAN_DIR, "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_thread_pool_under_thread_sanitizer():
    if not os.path.isdir(ASAN_DIR):
        pytest.skip("host sanitizer harness not present")
    if not os.path.exists("/opt/rocm/llvm/bin/clang++") or not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("clang++ or hipcc not available")
    exe = _load_build().build_threads()
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "ThreadSanitizer" not in out, out[-4000:]
    assert r.returncode == 0 and "done" in out, out[-4000:]
