"""The generated VRR1 operand tables (csrc/gen_tables.py, GenV<L>::ofs) read
with the kernels' item formula (Eq. vrr1, 1- and 2-quantal steps in place)
reproduce the oracle's primitive (s|e s) integrals.

With L_P = 0 the VRR1 targets [e0|0]^(0) are ordinary primitive integrals
(e s|s) (Section 2.5.3 with m = 0), so every level e <= 8 of every stage
layout (odd and even L) is pinned to the oracle.  The emulation mirrors the
per-item arithmetic of the device code, with each stage reading its inputs
before any output is written (the kernels' barrier between the two).
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
from tests.helpers import single_triplet

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "..", "paper_2210_03192_amd", "csrc"))
import gen_tables as gt  # noqa: E402


def _emulate(L, A, B, C, za, zb, zc):
    """[e0|0]^(0) for levels 0..L from the generated item tables."""
    g = za + zb
    P = (za * A + zb * B) / g
    rho = g * zc / (g + zc)
    PA, PC = P - A, P - C
    T = rho * PC @ PC
    pre = 2 * math.pi ** 2.5 / (math.sqrt(g + zc) * g * zc) * math.exp(-za * zb / g * (A - B) @ (A - B))
    F = oracle.boys(L, T)
    ofs, NT, NW = gt.vofs(L)
    rec = np.zeros(NT + NW)
    rec[0] = pre * F[0]
    for mm in range(1, L + 1):
        rec[NT + mm - 1] = pre * F[mm]
    rp = rho / g * PC
    i2g = 0.5 / g
    rg = rho / g
    k = 0
    for j, twoq in gt.vstages(L):
        n = gt.ncart(j) * (L - j + 1) + (gt.ncart(j - 1) * (L - j + 2) if twoq else 0)
        res = []
        for (u0, u1, u2, l0, l1, l2, y0, y1, dst, ax, f1, f2) in ofs[k:k + n]:
            ip = (ax >> 2) & 3
            c1 = f1 * i2g
            val = PA[ip] * rec[u0] - rp[ip] * rec[u1] + c1 * (rec[l0] - rg * rec[l1])
            if ax & 16:
                i = ax & 3
                x1 = PA[ip] * rec[u1] - rp[ip] * rec[u2] + c1 * (rec[l1] - rg * rec[l2])
                val = PA[i] * val - rp[i] * x1 + f2 * i2g * (rec[y0] - rg * rec[y1])
            res.append((dst, val))
        for dst, val in res:
            rec[dst] = val
        k += n
    assert k == len(ofs)
    return rec[:NT]


@pytest.mark.parametrize("L", range(0, 9))
def test_vrr1_tables_reproduce_oracle(L):
    rng = np.random.default_rng(1000 + L)
    A, B, C = rng.uniform(-1.5, 1.5, (3, 3))
    za, zb, zc = rng.uniform(0.3, 2.0, 3)
    got = _emulate(L, A, B, C, za, zb, zc)
    for e in range(L + 1):
        xyz, aux, orb, trip = single_triplet(A, B, C, e, 0, 0, za, zb, zc)
        ref = oracle.eval_batch(xyz, aux, orb, trip)[0]
        part = got[gt.offT(e):gt.offT(e) + gt.ncart(e)]
        np.testing.assert_allclose(part, ref, rtol=1e-11, atol=1e-14 * np.abs(ref).max())


def test_vrr1_missing_operands_carry_zero_coefficients():
    for L in range(0, 10):
        for (u0, u1, u2, l0, l1, l2, y0, y1, dst, ax, f1, f2) in gt.vofs(L)[0]:
            if (l0, l1) == (0, 0):
                assert f1 == 0
            if ax & 16 and (y0, y1) == (0, 0):
                assert f2 == 0
