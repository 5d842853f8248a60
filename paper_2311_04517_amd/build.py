"""Build ``libhpclust.so`` (the gfx950 HIP kernels and their C ABI) in-tree.

Every HIP translation unit is compiled for gfx950 only, with packed-FP32
instruction selection disabled (the compiler would otherwise form
v_pk_* FP32 operations on its own).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhpclust.so")
SOURCES = [os.path.join(CSRC, "hpclust.hip"), os.path.join(CSRC, "setenc.hip")]
HEADERS = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
HEADERS.append(os.path.join(ROOT, "include", "hpclust.h"))

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def source_digest() -> str:
    """SHA-256 over the code of the HIP sources and headers under csrc/,
    comments and whitespace removed (identifies the kernels a profile was
    taken on; documentation edits leave it unchanged)."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in sorted(p for p in SOURCES + HEADERS if os.path.dirname(p) == CSRC):
        with open(f) as fh:
            code = fh.read()
        code = re.sub(r"/\*.*?\*/", " ", code, flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(os.path.basename(f).encode())
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()


def build(verbose: bool = False, extra=None) -> str:
    """Compile every translation unit (in parallel, each its own device code
    object) and link the shared library."""
    objs = [os.path.join(CSRC, os.path.basename(s) + ".o") for s in SOURCES]
    compile_flags = [f for f in FLAGS if f != "-shared"]
    procs = []
    for src, obj in zip(SOURCES, objs):
        cmd = [HIPCC, *compile_flags, *(extra or []), "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
    failed = [cmd for p, cmd in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", OUT + ".tmp"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(OUT + ".tmp", OUT)
    for obj in objs:
        os.remove(obj)
    return OUT


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
