"""Build the gfx950 HIP library libkfmi.so in-tree with hipcc.

Every .hip file under csrc/ is compiled for gfx950 with packed-FP32
instruction selection disabled and multiply-add contraction limited to single
expressions, then linked into one shared library next to this file.
"""
import glob
import hashlib
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkfmi.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=on: multiply-adds are fused only within one source expression, so every inlined copy of a
# function (and every kernel variant) rounds alike and the results do not depend on the launch shape.
COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on", "-Xclang", "-target-feature",
          "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def source_digest():
    """First 16 hex digits of the SHA-256 of every kernel source and the public header: compiled into the
    library, it keys the autotune cache, so timings taken with other kernels are never reused."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.hpp")))
    files.append(os.path.join(HERE, "..", "include", "kfmi.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def build(verbose=False, jobs=8):
    srcs = sources()
    objdir = tempfile.mkdtemp(prefix="kfmi_build_")
    objs = []
    procs = []
    digest = f'-DKF_SOURCE_DIGEST="{source_digest()}"'
    for s in srcs:
        o = os.path.join(objdir, os.path.basename(s) + ".o")
        cmd = [HIPCC] + COMMON + [digest, "-c", s, "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stderr=subprocess.PIPE, stdout=subprocess.PIPE), s))
        objs.append(o)
        if len(procs) >= jobs:
            _wait(procs)
            procs = []
    _wait(procs)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    os.rmdir(objdir)
    return LIB


def _wait(procs):
    for p, s in procs:
        out, err = p.communicate()
        msg = "\n".join(l for l in err.decode().splitlines() if "packed-fp32-ops" not in l and l.strip())
        if p.returncode != 0:
            sys.stderr.write(msg + "\n")
            raise RuntimeError(f"hipcc failed on {s}")
        if msg and ("warning" in msg or "error" in msg):
            sys.stderr.write(msg + "\n")


if __name__ == "__main__":
    print(build(verbose=True))
