"""Build libpin.so (HIP, gfx950) in-tree: ``python -m paper_1305_1505_amd.build``.

Every kernel is instantiated per supported grid size and precision (csrc/sizes.hpp), one
translation unit each, compiled in parallel with hipcc and linked into
``paper_1305_1505_amd/libpin.so``.  Packed-FP32 instructions are disabled for all device code.
"""

import concurrent.futures
import os
import re
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libpin.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]
HOST_SOURCES = ["capi.cpp", "plan.cpp", "serve.cpp", "host_math.cpp", "registry.cpp"]


def sizes():
    text = open(os.path.join(CSRC, "sizes.hpp")).read()
    return [int(m) for m in re.findall(r"X\((\d+)\)", text)]


def _run(cmd):
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError("command failed: %s\n%s%s" % (" ".join(cmd), proc.stdout, proc.stderr))
    return proc


def build(jobs=None, verbose=False):
    """Compile every translation unit and link libpin.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    tasks = []
    for n in sizes():
        for fp64 in (0, 1):
            obj = os.path.join(BUILD, f"inst_{fp64}_{n}.o")
            tasks.append([HIPCC, *COMMON, f"-DPIN_INST_N={n}", f"-DPIN_INST_FP64={fp64}",
                          "-c", os.path.join(CSRC, "inst.hip"), "-o", obj])
    # fragmentation: float64 decisions in the order the method states them, no contraction
    tasks.append([HIPCC, *COMMON, "-ffp-contract=off", "-c", os.path.join(CSRC, "fragment.hip"),
                  "-o", os.path.join(BUILD, "fragment.o")])
    # allocation-free collapse times: static device scratch and its table kernels
    tasks.append([HIPCC, *COMMON, "-c", os.path.join(CSRC, "noalloc.hip"), "-o", os.path.join(BUILD, "noalloc.o")])
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src.replace(".cpp", ".o"))
        tasks.append([HIPCC, *COMMON, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
    objs = [t[-1] for t in tasks]
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        for cmd, fut in zip(tasks, [ex.submit(_run, t) for t in tasks]):
            fut.result()
            if verbose:
                print("built", os.path.basename(cmd[-1]), flush=True)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs,
          "-L", os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
