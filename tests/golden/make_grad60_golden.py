"""Write grad60_atoms.txt: oracle gradient rows of sampled atoms of the
60-atom water cluster (20 waters, the differentiable workload).

L = sum_ab G_ab J_ab with J_ab = sum_P (ab|P) d_P, d ~ N(0,1) (seed 5) and G
the symmetric random density (seed 6); dL/dR_X for the atoms listed, by the
oracle's explicit three-centre derivative integrals restricted to the triplets
that touch those atoms (their rows are then complete).  Calls only oracle/ and
the seeded input builders.

    python tests/golden/make_grad60_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2210_03192_amd import inputs  # noqa: E402

# two oxygens (index % 3 == 0) and four hydrogens, spread over the cluster
ATOMS = (0, 1, 29, 33, 47, 58)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grad60_atoms.txt")


def main():
    s = inputs.grad_60_system()
    d = inputs.fitting_coefficients(s.aux.nbf, 5)
    G = inputs.symmetric_density(s.orb.nbf, 6)
    rows = []
    for X in ATOMS:
        m = np.zeros(len(s.xyz), np.uint8)
        m[X] = 1
        g = oracle.coulomb_J_grad(s.xyz, s.aux, s.orb, d, G, atom_mask=m)
        rows.append((X, g[X]))
        print(f"atom {X}: {g[X]}", flush=True)
    with open(OUT, "w") as f:
        f.write("# dL/dR of sampled atoms of the 60-atom water cluster (inputs.grad_60_system),\n"
                "# L = sum_ab G_ab J_ab, d = fitting_coefficients(naux, 5),\n"
                "# G = symmetric_density(nao, 6).  Written by make_grad60_golden.py with the\n"
                "# CPU oracle (explicit derivatives of all three centres, double precision).\n"
                "# columns: atom  dL/dX  dL/dY  dL/dZ  (hartree/bohr)\n")
        for X, g in rows:
            f.write(f"{X} {float(g[0])!r} {float(g[1])!r} {float(g[2])!r}\n")


if __name__ == "__main__":
    main()
