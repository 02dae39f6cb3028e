"""Build the gfx950 shared library libhamls.so in-tree with hipcc.

Every HIP source is compiled for gfx950 only, one object per source and in
parallel (into _build/), then linked.  Packed FP32 instructions are disabled
(-packed-fp32-ops); the membership predicate additionally disables contraction
locally in its source.
"""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhamls.so")
OBJ = os.path.join(ROOT, "_build")
SRC = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
HDR = sorted(glob.glob(os.path.join(HERE, "csrc", "*.h"))) + [os.path.join(ROOT, "include", "hamls.h")]


def flags():
    return ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-Wno-unknown-pragmas"]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in SRC + HDR)


def _filtered(text: str) -> str:
    # hipcc's host pass does not know the packed-fp32 target feature
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    jobs = []
    for src in SRC:
        obj = os.path.join(OBJ, os.path.basename(src) + ".o")
        jobs.append((src, obj, [hipcc] + flags() + ["-c", "-o", obj, src]))

    def run(job):
        src, obj, cmd = job
        if verbose:
            print(" ".join(cmd), flush=True)
        return src, subprocess.run(cmd, capture_output=True, text=True)

    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    failed = False
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for src, r in ex.map(run, jobs):
            out = _filtered(r.stdout + r.stderr)
            if r.returncode != 0:
                failed = True
                sys.stderr.write(f"--- {os.path.basename(src)}\n{out}\n")
            elif verbose and out.strip():
                sys.stderr.write(out + "\n")
    if failed:
        raise RuntimeError("hipcc failed")
    link = [hipcc, "--offload-arch=gfx950", "-fPIC", "-shared", "-o", LIB + ".tmp"] + [j[1] for j in jobs]
    if verbose:
        print(" ".join(link), flush=True)
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
