"""Build the HIP library (gfx950) in-tree: paper_2503_08586_amd/liblens_mi355x.so."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblens_mi355x.so")
SOURCES = ["lens_kernels.hip", "lens_sampler.hip", "lens_peaks.hip", "lens_runtime.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions stay off in every HIP build of this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
    "-I" + CSRC,
]


def build(verbose: bool = False) -> str:
    """Compile every source to an object, link the shared library (atomic replace)."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, "-x", "hip"] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed on %s" % src)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


ASAN_DRIVER = os.path.join(HERE, "_build", "runtime_asan_driver")
# host code only: the device code is the library's own (sanitizers on the GPU
# side are neither wanted nor available)
ASAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def build_asan_driver(verbose: bool = False) -> str:
    """The C-ABI driver tests/runtime_sanitize_driver.cpp, linked with the
    runtime compiled with host-side AddressSanitizer and UBSan and with the
    library's own kernel objects (build() first)."""
    objdir = os.path.join(HERE, "_build")
    kobjs = [os.path.join(objdir, os.path.splitext(s)[0] + ".o") for s in SOURCES if s.endswith(".hip")]
    rt = os.path.join(objdir, "lens_runtime_asan.o")
    drv = os.path.join(objdir, "runtime_sanitize_driver.o")
    steps = [
        [HIPCC, "-x", "hip"] + FLAGS + ASAN_HOST + ["-c", os.path.join(CSRC, "lens_runtime.cpp"), "-o", rt],
        [HIPCC, "-x", "hip"] + FLAGS + ASAN_HOST + ["-c", os.path.join(ROOT, "tests", "runtime_sanitize_driver.cpp"),
                                                     "-o", drv],
        [HIPCC, "--offload-arch=gfx950"] + ASAN_HOST + [drv, rt] + kobjs + ["-lpthread", "-o", ASAN_DRIVER],
    ]
    for cmd in steps:
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("sanitizer driver build failed")
    return ASAN_DRIVER


if __name__ == "__main__":
    print(build(verbose=True))
