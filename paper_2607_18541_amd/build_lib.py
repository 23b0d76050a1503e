"""Builds liblz.so (host C++ + gfx950 HIP kernels) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "liblz.so")

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".cpp", ".hip")))


def build(verbose=False, jobs=8):
    objs = []
    procs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in sources():
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        if src.endswith(".hip"):
            cmd = ["hipcc", "-x", "hip"] + HIP_FLAGS + ["-c", src, "-o", obj]
        else:
            cmd = ["hipcc", "-O3", "-std=c++17", "-fPIC", "-Wall", "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    bad = [c for p, c in procs if p.wait() != 0]
    if bad:
        raise RuntimeError("compile failed: " + " ".join(bad[0]))
    link = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", OUT + ".tmp"] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
