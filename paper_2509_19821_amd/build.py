"""Build the HIP library (gfx950) in-tree: paper_2509_19821_amd/_build/libgmpea.so."""
from __future__ import annotations

import json
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(OUT_DIR, "libgmpea.so")
SOURCES = ["gmpea_kernels.hip", "gmpea_kernels_wide.hip", "gmpea_abi.cpp", "lattice.cpp"]
ARCH = "gfx950"
LIBS = ["-lpthread", "-lrocprofiler-sdk-roctx"]  # roctx: ranges over the ABI's calls


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the GMPEA library needs ROCm to build")
    return path


def flags() -> list:
    return ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-Wall",
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
            # keep packed-FP32 instructions out of the generated code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # no implicit multiply-add fusion: the kernels write fmaf where they
            # want one, so results do not depend on the inlining context
            "-ffp-contract=off"]


def build(verbose: bool = False, jobs: int = 3) -> str:
    """Compile every source to an object file, then link the shared library.
    Always compiles (no staleness shortcut)."""
    os.makedirs(OUT_DIR, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc()] + flags() + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for pr in procs:
        _wait(pr)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + LIBS
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    with open(os.path.join(OUT_DIR, "build_info.json"), "w") as fh:
        json.dump({"hip_version": hip_version(), "arch": ARCH}, fh)
    return LIB


def hip_version() -> str:
    """major.minor.patch of the HIP toolchain (from hip_version.h)."""
    inc = os.path.join(os.path.dirname(os.path.dirname(hipcc())), "include", "hip", "hip_version.h")
    vals = {}
    with open(inc) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) == 3 and parts[0] == "#define" and parts[1] in (
                    "HIP_VERSION_MAJOR", "HIP_VERSION_MINOR", "HIP_VERSION_PATCH"):
                vals[parts[1]] = parts[2]
    return "%s.%s.%s" % (vals["HIP_VERSION_MAJOR"], vals["HIP_VERSION_MINOR"],
                         vals["HIP_VERSION_PATCH"])


def _wait(pr):
    src, p = pr
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    if p.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (src, text))
    # surface real warnings, not the host pass's note about the GPU-only feature
    lines = [ln for ln in text.splitlines() if ln.strip() and "packed-fp32-ops" not in ln]
    if lines:
        sys.stderr.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    print(build(verbose=True))
