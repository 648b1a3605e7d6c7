"""Builds libqtn's host code with AddressSanitizer (or ThreadSanitizer)
against CPU stand-ins for the HIP runtime (stubs.cpp): C++ sources with g++,
HIP sources host-only with hipcc (no device code).  Test infrastructure; the
product library is built by paper_2010_14962_amd/build.py."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2010_14962_amd", "csrc")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
BASE = ["-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include")]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("%s failed:\n%s" % (" ".join(cmd), r.stdout + r.stderr))


def build() -> str:
    """The AddressSanitizer library (for Python drivers); returns its path."""
    OUT = os.path.join(HERE, "_build")
    LIB = os.path.join(OUT, "libqtn_host_asan.so")
    # host compilers take the sanitizer directly; on hipcc lines it is marked
    # as host-only (these compile no device code at all)
    GXX_SAN = ["-fsanitize=address"]
    HIPCC_SAN = ["-Xarch_host", "-fsanitize=address"]
    os.makedirs(OUT, exist_ok=True)
    jobs = []
    for src in ("planner.cpp", "api.cpp", "costmodel.cpp", "ranges.cpp"):
        jobs.append(["g++"] + BASE + GXX_SAN + ["-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-c",
                                               os.path.join(CSRC, src), "-o", os.path.join(OUT, src + ".o")])
    for src in ("runtime.hip", "mlp.hip"):
        jobs.append([HIPCC, "--offload-arch=gfx950", "--cuda-host-only"] + BASE + HIPCC_SAN +
                    ["-c", os.path.join(CSRC, src), "-o", os.path.join(OUT, src + ".o")])
    jobs.append(["g++"] + BASE + GXX_SAN + ["-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-c",
                                           os.path.join(HERE, "stubs.cpp"), "-o", os.path.join(OUT, "stubs.o")])
    with ThreadPoolExecutor(min(len(jobs), 8)) as ex:
        list(ex.map(_run, jobs))
    objs = [os.path.join(OUT, f) for f in sorted(os.listdir(OUT)) if f.endswith(".o") and f != "fatbin.o"]
    # the host-only objects name the device code image they would register;
    # give each such symbol an empty definition
    nm = subprocess.run(["nm", "-u"] + objs, capture_output=True, text=True).stdout
    names = sorted({l.split()[-1] for l in nm.splitlines() if "__hip_fatbin_" in l})
    fat_c = os.path.join(OUT, "fatbin.c")
    with open(fat_c, "w") as f:
        for n in names:
            f.write("char %s[64];\n" % n)
    _run(["gcc", "-fPIC", "-c", fat_c, "-o", os.path.join(OUT, "fatbin.o")])
    _run(["g++", "-shared", "-fsanitize=address", "-o", LIB] + objs + [os.path.join(OUT, "fatbin.o")])
    return LIB


def build_threads() -> str:
    """The host objects, the stand-ins and threads_main.cpp compiled with
    clang and ThreadSanitizer into one executable (the sanitizer runtime
    must be the program's own); returns its path."""
    OUT = os.path.join(HERE, "_build_thread")
    os.makedirs(OUT, exist_ok=True)
    clang = "/opt/rocm/llvm/bin/clang++"
    SAN = ["-fsanitize=thread"]
    jobs = []
    for src in ("planner.cpp", "api.cpp", "costmodel.cpp", "ranges.cpp"):
        jobs.append([clang] + BASE + SAN + ["-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-c",
                                           os.path.join(CSRC, src), "-o", os.path.join(OUT, src + ".o")])
    for src in ("runtime.hip", "mlp.hip"):
        jobs.append([HIPCC, "--offload-arch=gfx950", "--cuda-host-only"] + BASE + ["-Xarch_host", "-fsanitize=thread"] +
                    ["-c", os.path.join(CSRC, src), "-o", os.path.join(OUT, src + ".o")])
    for src in ("stubs.cpp", "threads_main.cpp"):
        jobs.append([clang] + BASE + SAN + ["-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-c",
                                           os.path.join(HERE, src), "-o", os.path.join(OUT, src + ".o")])
    with ThreadPoolExecutor(min(len(jobs), 8)) as ex:
        list(ex.map(_run, jobs))
    objs = [os.path.join(OUT, f) for f in sorted(os.listdir(OUT)) if f.endswith(".o") and f != "fatbin.o"]
    nm = subprocess.run(["nm", "-u"] + objs, capture_output=True, text=True).stdout
    names = sorted({l.split()[-1] for l in nm.splitlines() if "__hip_fatbin_" in l})
    fat_c = os.path.join(OUT, "fatbin.c")
    with open(fat_c, "w") as f:
        for n in names:
            f.write("char %s[64];\n" % n)
    _run(["gcc", "-fPIC", "-c", fat_c, "-o", os.path.join(OUT, "fatbin.o")])
    exe = os.path.join(OUT, "threads_main")
    _run([clang, "-fsanitize=thread", "-o", exe] + objs + [os.path.join(OUT, "fatbin.o"), "-lpthread"])
    return exe


if __name__ == "__main__":
    print(build_threads() if sys.argv[1:] == ["thread"] else build())
    sys.exit(0)
