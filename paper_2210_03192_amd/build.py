"""Build libdf3c.so (HIP for gfx950) in-tree.

Steps: generate the index tables (csrc/gen_tables.py), compile every .hip
translation unit with hipcc for gfx950 in parallel, link a shared library next
to this file.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdf3c.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    "-O3", f"--offload-arch={ARCH}", "-std=c++20", "-fPIC",
    # no packed FP32 instructions in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))


def _newest_header():
    paths = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    gen = os.path.join(CSRC, "gen")
    if os.path.isdir(gen):
        paths += [os.path.join(gen, f) for f in os.listdir(gen) if f.endswith(".hpp")]
    return max(os.path.getmtime(p) for p in paths)


def _compile(src, verbose, force=True):
    obj = os.path.join(OBJ, src.replace(".hip", ".o"))
    if not force and os.path.exists(obj):
        t = os.path.getmtime(obj)
        deps = [_newest_header()]
        if src == "runtime.hip":
            deps.append(os.path.getmtime(os.path.join(HERE, "..", "include", "df3c.h")))
        if t > os.path.getmtime(os.path.join(CSRC, src)) and t > max(deps):
            return obj, ""
    cmd = ["hipcc", *HIPCC_FLAGS, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{msgs}")
    return obj, msgs


def build(verbose: bool = False, jobs: int = 0, force: bool = True) -> str:
    """Compile and link; force=False reuses objects newer than their sources."""
    subprocess.run([sys.executable, os.path.join(CSRC, "gen_tables.py"),
                    os.path.join(CSRC, "gen")], check=True)
    os.makedirs(OBJ, exist_ok=True)
    srcs = _sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    objs = []
    with cf.ThreadPoolExecutor(jobs) as ex:
        for obj, msgs in ex.map(lambda s: _compile(s, verbose, force), srcs):
            objs.append(obj)
            if msgs and verbose:
                print(msgs, flush=True)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, force="--incremental" not in sys.argv)
