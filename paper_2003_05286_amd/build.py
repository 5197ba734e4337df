"""Build libsdq.so (the HIP library) in-tree for gfx950.

Compiles the per-tile-count kernel instantiations (n <= 128) and the gang
kernels (n > 128) in parallel with hipcc and links them with the dispatch
and runtime objects into
paper_2003_05286_amd/libsdq.so; then links tests/_bin/sdq_abi_check, the
C-ABI driver over the same objects with the host runtime built under
AddressSanitizer and UndefinedBehaviorSanitizer.  Always recompiles.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsdq.so")
ARCH = "gfx950"
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
NTS = range(1, 9)
# the sanitized C-ABI driver (a test program, built beside the library)
ABI_CHECK = os.path.join(ROOT, "tests", "_bin", "sdq_abi_check")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            # packed FP32 instructions stay off (not used by this FP64 code
            # either way; the host pass warns that it does not know the feature)
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _compile(args):
    src, obj, extra = args
    cmd = [hipcc()] + _flags() + extra + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{err}")
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    tasks = []
    for nt in NTS:
        tasks.append((os.path.join(CSRC, "sdq_nt.hip"), os.path.join(BUILD, f"sdq_nt{nt}.o"),
                      [f"-DSDQ_NT={nt}"]))
        tasks.append((os.path.join(CSRC, "sdq_nt_dense.hip"), os.path.join(BUILD, f"sdq_nt_dense{nt}.o"),
                      [f"-DSDQ_NT={nt}"]))
    tasks.append((os.path.join(CSRC, "sdq_nt9.hip"), os.path.join(BUILD, "sdq_nt9.o"), []))
    tasks.append((os.path.join(CSRC, "sdq_dispatch.hip"), os.path.join(BUILD, "sdq_dispatch.o"), []))
    tasks.append((os.path.join(CSRC, "sdq_gang.hip"), os.path.join(BUILD, "sdq_gang.o"), []))
    tasks.append((os.path.join(CSRC, "sdq_complex.hip"), os.path.join(BUILD, "sdq_complex.o"), []))
    tasks.append((os.path.join(CSRC, "sdq_noalloc.hip"), os.path.join(BUILD, "sdq_noalloc.o"), []))
    tasks.append((os.path.join(CSRC, "sdq_runtime.cpp"), os.path.join(BUILD, "sdq_runtime.o"), []))
    jobs = jobs or min(len(tasks), os.cpu_count() or 4, 16)
    # the largest instantiations first
    tasks.sort(key=lambda t: -int(t[2][0].split("=")[1]) if t[2] else 0)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, tasks))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + \
        ["-L", os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, LIB)
    build_abi_check(objs)
    if verbose:
        print("built", LIB, "and", ABI_CHECK)
    return LIB


def build_abi_check(objs) -> str:
    """The C-ABI driver of tests/abi_check.cpp linked with the host runtime
    compiled by g++ under AddressSanitizer and UndefinedBehaviorSanitizer
    (host code only; the HIP objects are the library's own, the sanitizer
    runtimes are linked statically into the executable)."""
    os.makedirs(os.path.dirname(ABI_CHECK), exist_ok=True)
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    cflags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
              "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"), "-I", CSRC] + san
    rt = os.path.join(BUILD, "sdq_runtime_san.o")
    drv = os.path.join(BUILD, "abi_check_san.o")
    jobs = [["g++"] + cflags + ["-c", os.path.join(CSRC, "sdq_runtime.cpp"), "-o", rt],
            ["g++"] + cflags + ["-c", os.path.join(ROOT, "tests", "abi_check.cpp"), "-o", drv]]
    with cf.ThreadPoolExecutor(2) as ex:
        for cmd, r in zip(jobs, ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), jobs)):
            if r.returncode != 0:
                raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
    hip_objs = [o for o in objs if os.path.basename(o) != "sdq_runtime.o"]
    cmd = ["g++"] + san + ["-static-libasan", "-static-libubsan", "-o", ABI_CHECK, drv, rt] + hip_objs + \
        ["-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lrocprofiler-sdk-roctx",
         "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    return ABI_CHECK


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
