"""Sanitizer build of the library's host code (CPU checks only).

    python -m paper_2404_07249_amd.build_asan        # -> _build_asan/libpb3_asan.so

The host C++ sources (plan construction, workspace layout, batching) are
compiled by g++ with AddressSanitizer and UndefinedBehaviorSanitizer; the
HIP sources are compiled as in the normal build, without sanitizers (GPU
code is not instrumented).  Load the result with the sanitizer runtimes
preloaded (see tests/test_host_sanitizers.py), e.g.

    LD_PRELOAD="$(g++ -print-file-name=libasan.so) $(g++ -print-file-name=libubsan.so)" \\
    PB3_LIBRARY=paper_2404_07249_amd/_build_asan/libpb3_asan.so python -m pytest tests/test_abi.py
"""

from __future__ import annotations

import concurrent.futures as cf
import os

from . import build as B

OUT_DIR = os.path.join(B.HERE, "_build_asan")
OUT = os.path.join(OUT_DIR, "libpb3_asan.so")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
GXX_FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
             f"-I{B.INCLUDE}", f"-I{B.CSRC}"] + SAN


def build() -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    jobs = []
    for name in sorted(os.listdir(B.CSRC)):
        src = os.path.join(B.CSRC, name)
        obj = os.path.join(OUT_DIR, name + ".o")
        if name.endswith(".cpp"):
            jobs.append(["g++", "-c", src, "-o", obj] + GXX_FLAGS)
        elif name.endswith(".hip"):
            jobs.append([B._hipcc(), "-x", "hip", "-c", src, "-o", obj] + B.HIP_FLAGS)
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with cf.ThreadPoolExecutor(workers) as ex:
        list(ex.map(B._run, jobs))
    objs = [j[j.index("-o") + 1] for j in jobs]
    tmp = OUT + ".tmp"
    B._run([B._hipcc(), "-shared", "-fPIC", f"--offload-arch={B.ARCH}", "-o", tmp] + objs +
           ["-lasan", "-lubsan"])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
