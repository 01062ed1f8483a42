"""Compile libddst.so (all HIP sources) for gfx950 in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = ["dense.hip", "vec.hip", "hodlr.hip", "hbs.hip", "prof.hip", "noalloc.hip", "api.hip"]
LIB = os.path.join(HERE, "libddst.so")


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False) -> str:
    csrc = os.path.join(HERE, "csrc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    flags = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]
    objs = []
    procs = []
    for s in SRC:
        o = os.path.join(objdir, s.replace(".hip", ".o"))
        cmd = [hipcc(), *flags, "-c", os.path.join(csrc, s), "-o", o]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                            stderr=subprocess.STDOUT, text=True)))
        objs.append(o)
    failed = False
    for cmd, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed = True
            sys.stderr.write(" ".join(cmd) + "\n" + out)
        elif verbose and out.strip():
            filtered = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l)
            if filtered.strip():
                sys.stderr.write(filtered + "\n")
    if failed:
        raise RuntimeError("HIP compilation failed")
    tmp = LIB + ".tmp"
    subprocess.run([hipcc(), "-shared", "--offload-arch=gfx950", "-fPIC", *objs, "-o", tmp],
                   check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
