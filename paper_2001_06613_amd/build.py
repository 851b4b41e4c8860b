"""Build libstml.so for gfx950 with hipcc (in-tree, next to this file)."""

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "libstml.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# packed FP32 instructions stay off: hipcc would otherwise form them from
# scalar or float2 code
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

SOURCES = ["kernels.hip", "cg_tiles.hip", "cnn.hip", "affine.hip",
           "noalloc.hip", "stml.cpp"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {cmd[-1]}")
    return r


def build(verbose=False):
    """Compile every source and link libstml.so; always rebuilds."""
    tmp = tempfile.mkdtemp(prefix="stml_build_")
    try:
        objs = []
        for src in SOURCES:
            obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
            cmd = [HIPCC, "-x", "hip", f"--offload-arch={ARCH}", "-O3",
                   "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
                   "-I", os.path.join(ROOT, "include")] + DEVICE_FLAGS + \
                  ["-c", os.path.join(CSRC, src), "-o", obj]
            r = _run(cmd)
            if verbose and r.stderr:
                sys.stderr.write(r.stderr)
            objs.append(obj)
        out_tmp = os.path.join(tmp, "libstml.so")
        _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o",
              out_tmp] + objs)
        shutil.move(out_tmp, OUT)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
