"""Build libhjx.so (HIP, gfx950) in-tree.

hipcc compiles the kernels and the host engine for gfx950 only.  Packed
FP32 instructions are disabled for device code (-packed-fp32-ops), and the
host code keeps IEEE evaluation order (-ffp-contract=off on the host side).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhjx.so")
SOURCES = ["hjx_kernels.hip", "hjx_steps.hip", "hjx_adjoint.hip", "hjx_batch.hip", "hjx_claw.hip", "hjx_shapes.hip", "hjx_api.cpp"]
ARCH = os.environ.get("HJX_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Xarch_host", "-ffp-contract=off",
    "-I", os.path.join(ROOT, "include"),
]


OBJDIR = os.path.join(CSRC, "_build")


def _deps(path, seen=None):
    """The file and every file it includes with #include "...", recursively."""
    import re
    seen = set() if seen is None else seen
    if path in seen or not os.path.exists(path):
        return seen
    seen.add(path)
    with open(path, encoding="utf-8") as f:
        for m in re.finditer(r'^\s*#\s*include\s+"([^"]+)"', f.read(), re.M):
            _deps(os.path.normpath(os.path.join(os.path.dirname(path), m.group(1))), seen)
    return seen


def _stale(obj, src):
    """An object is stale when it is missing or older than its source or a
    header the source includes."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in _deps(src))


def build(verbose=False, force=True):
    """Compile every source for gfx950 and link libhjx.so.  force=False
    recompiles only the objects older than their sources or headers (the
    objects are kept in csrc/_build)."""
    os.makedirs(OBJDIR, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        path = os.path.join(CSRC, src)
        if not force and not _stale(obj, path):
            continue
        cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", path, "-o", obj + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd, obj))
    failed = [cmd for p, cmd, _ in procs if p.wait() != 0]
    if failed:
        raise RuntimeError("compile failed: " + " ".join(failed[0]))
    for _, _, obj in procs:
        os.replace(obj + ".tmp", obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-L/opt/rocm/lib",
           "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    import sys
    print(build(verbose=True, force="--changed" not in sys.argv))
