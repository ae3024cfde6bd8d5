"""Builds the HIP library liblbm.so in-tree for gfx950 with hipcc.

Packed FP32 instructions are disabled (-packed-fp32-ops): the kernels are
written in scalar float arithmetic and must not be contracted into them.
"""
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = ["abi.cpp", "kernels.hip", "adjoint.hip", "util.hip"]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose=False, extra=()):
    """Compiles every source to an object in parallel, then links."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    flags = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics", "-Wno-unused-result",
             "-I", os.path.join(HERE, "..", "include"), *extra]
    objdir = tempfile.mkdtemp(prefix="lbm_build_")
    try:
        jobs = []
        for src in srcs:
            obj = os.path.join(objdir, os.path.basename(src) + ".o")
            cmd = [hipcc(), *flags, "-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            jobs.append((obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                               text=True)))
        failed = False
        for obj, proc in jobs:
            out, err = proc.communicate()
            if proc.returncode != 0:
                failed = True
                sys.stderr.write(out + err)
            elif verbose and err:
                sys.stderr.write(err)
        if failed:
            raise RuntimeError("hipcc failed")
        tmp = LIB + ".tmp"
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *[o for o, _ in jobs]]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("link failed")
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(objdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
