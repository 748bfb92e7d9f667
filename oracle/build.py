"""Build the CPU oracle (test infrastructure) with gcc.

Produces liboracle.so (double) and liboracle_ld.so (x87 long double) next to
this file.  Plain IEEE arithmetic: no -ffast-math.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> None:
    src = os.path.join(HERE, "oracle.c")
    for out, extra in (("liboracle.so", []), ("liboracle_ld.so", ["-DORACLE_LONG"])):
        cmd = ["gcc", "-O2", "-fopenmp", "-Wall", "-shared", "-fPIC", *extra, src,
               "-o", os.path.join(HERE, out), "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)


if __name__ == "__main__":
    build(verbose=True)
