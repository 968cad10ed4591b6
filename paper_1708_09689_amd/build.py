"""Build the HIP library libpvdtm.so for gfx950 in-tree.

    python -m paper_1708_09689_amd.build

Compiles paper_1708_09689_amd/csrc/*.hip (device code + launchers) and
csrc/*.cpp (C ABI, host drivers) with hipcc into
paper_1708_09689_amd/lib/libpvdtm.so.
"""

from __future__ import annotations

import concurrent.futures
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libpvdtm.so")
ARCH = os.environ.get("PV_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    f"--offload-arch={ARCH}",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-Wall", "-Wno-unused-function",
]


def source_hash() -> str:
    """SHA-256 (first 16 hex digits) of the library's sources and C header,
    stamped into the build and compared by the binding when it loads the
    library: a library built from other sources is refused."""
    import hashlib
    files = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")) +
                   glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(INCLUDE, "*.h")))
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode() + b"\0")
        with open(f, "rb") as fh:
            h.update(fh.read())
        h.update(b"\0")
    return h.hexdigest()[:16]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def embed_kernel_sources(objdir: str) -> str:
    """C++ file holding the text of the sweep kernel headers, which the
    library compiles at run time (hipRTC) for stencils outside the built-in
    families."""
    parts = ["// Written by build.py: kernel headers compiled at run time for generated stencils.",
             "namespace pv {", "extern const char* const kRtcKernelsHpp;", "extern const char* const kRtcSweepHpp;"]
    for sym, name in (("kRtcKernelsHpp", "pv_kernels.hpp"), ("kRtcSweepHpp", "pv_sweep.hpp")):
        with open(os.path.join(CSRC, name)) as fh:
            text = fh.read()
        if ")PVRTC" in text:
            raise RuntimeError(f"{name} holds the raw-string delimiter")
        parts.append(f'const char* const {sym} = R"PVRTC({text})PVRTC";')
    parts.append("}  // namespace pv")
    out = os.path.join(objdir, "pv_rtc_source.cpp")
    body = "\n".join(parts) + "\n"
    if not os.path.exists(out) or open(out).read() != body:
        with open(out, "w") as fh:
            fh.write(body)
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    srcs.append(embed_kernel_sources(objdir))
    objs = [os.path.join(objdir, os.path.basename(src) + ".o") for src in srcs]
    stamp = f'-DPV_SOURCE_HASH="{source_hash()}"'
    cmds = [[hipcc(), *HIP_FLAGS, stamp, "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj] for src, obj in zip(srcs, objs)]
    if verbose:
        for cmd in cmds:
            print(" ".join(cmd), flush=True)
    # one compiler per translation unit, in parallel (the stencil families
    # are separate units); MAX_JOBS caps the number of jobs
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", "0")) or (os.cpu_count() or 1), 16))
    with concurrent.futures.ThreadPoolExecutor(jobs) as pool:
        for cmd, done in zip(cmds, pool.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds)):
            if done.returncode != 0:
                sys.stderr.write(done.stdout + done.stderr)
                raise subprocess.CalledProcessError(done.returncode, cmd)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-lhiprtc", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
