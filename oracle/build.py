"""Compile the FP64 CPU oracle (test infrastructure only) into oracle/libhjxo.so.

The oracle is plain C99, built with gcc at -O2 with floating-point
contraction off, so every expression rounds exactly as written.  The same
source is compiled twice: once in double (hjxo_*), once in double complex for
complex-step directional derivatives (hjxo_cs_*).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hjxo.c")
LIB = os.path.join(HERE, "libhjxo.so")

CFLAGS = ["-std=c99", "-O2", "-fPIC", "-fopenmp", "-ffp-contract=off", "-Wall", "-Wextra",
          "-Wno-unused-function"]


def build(verbose=False):
    objs = []
    for tag, defs in (("re", []), ("cs", ["-DHJXO_CSTEP"])):
        obj = os.path.join(HERE, f"hjxo_{tag}.o")
        cmd = ["gcc", *CFLAGS, *defs, "-c", SRC, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-shared", "-fopenmp", "-o", tmp, *objs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
