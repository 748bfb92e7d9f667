"""The derivative engine's formulas, emulated on the CPU with the generated
tables (GenY, GenSolid::jh_*, VRR1 stages), reproduce the oracle's derivative
integrals for one primitive triplet.

The engine transposes the HRR of each shifted class onto G~ once per pair,
  omega^{A+,x}_e = sum_ab G~_ab sum_i [a + 1_x + i = e] C(b,i) AB^{b-i}   (and B+, A-, B-),
forms per primitive the digested ket Y_e = sum_u e!/(e-u)! H_u [e-u 0|0]^(L_P)
and takes
  dA_x = 2 zeta_a omega^{A+,x}.Y - omega^{A-,x}.Y,
  dB_x = 2 zeta_b omega^{B+,x}.Y - omega^{B-,x}.Y.
These must equal sum_ab G~_ab sum_m d_m d/dA_x (a b|P_m) (and d/dB_x), checked
against the oracle's shifted-class integrals (raising and lowering) and against
central differences of the oracle's integrals in the centre coordinates.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
from tests.helpers import single_triplet
from tests.test_jengine_tables import _vrr1

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "..", "paper_2210_03192_amd", "csrc"))
import gen_tables as gt  # noqa: E402


def _omegas(LA, LB, Gt, AB):
    """The twelve weight vectors, rows j = 3 s + x (s = A+, B+, A-, B-), as the
    kernel gathers them."""
    EA, EB = max(LA - 1, 0), LA + LB + 1
    es = [e for lev in range(EA, EB + 1) for e in gt.carts(lev)]
    om = np.zeros((12, len(es)))
    for s in range(4):
        las = LA + 1 if s == 0 else LA - 1 if s == 2 else LA
        for x in range(3):
            for ei, e in enumerate(es):
                k = sum(e) - las
                if k < 0:
                    continue
                v = 0.0
                for bi, b in enumerate(gt.carts(LB)):
                    bb = list(b)
                    cb = 1.0
                    if s == 1:
                        bb[x] += 1
                    if s == 3:
                        if b[x] == 0:
                            continue
                        cb = b[x]
                        bb[x] -= 1
                    for i in gt.carts(k):
                        if any(i[t] > bb[t] for t in range(3)):
                            continue
                        a = [e[t] - i[t] for t in range(3)]
                        if s == 0:
                            a[x] -= 1
                        if s == 2:
                            a[x] += 1
                        if min(a) < 0:
                            continue
                        ca = a[x] if s == 2 else 1.0
                        bn = math.prod(math.comb(bb[t], i[t]) for t in range(3))
                        v += ca * cb * bn * Gt[gt.cidx(tuple(a)), bi] * \
                            math.prod(AB[t] ** (bb[t] - i[t]) for t in range(3))
                om[3 * s + x, ei] = v
    return om


def _engine_grad(LP, LA, LB, A, B, C, za, zb, zc, dprime, Gt):
    EA, EB = max(LA - 1, 0), LA + LB + 1
    g = za + zb
    P = (za * A + zb * B) / g
    rho = g * zc / (g + zc)
    PA, PC = P - A, P - C
    pre = 2 * math.pi ** 2.5 / (math.sqrt(g + zc) * g * zc) * math.exp(-za * zb / g * (A - B) @ (A - B))
    F = oracle.boys(LP + EB, rho * PC @ PC)
    V = _vrr1(EB, LP, PA, rho / g * PC, 0.5 / g, rho / g, pre, F)
    s, w = rho / (2 * g * zc), rho / zc * PC
    sw = [s ** k * np.prod(w ** np.array(n)) for k in range(LP + 1) for n in gt.carts(LP - k)]
    hs, hc, hsw, hb = gt.jh_terms(LP)
    H = [sum(hb[q] * dprime[hc[q]] * sw[hsw[q]] for q in range(hs[u], hs[u + 1]))
         for u in range(len(hs) - 1)]
    ys, yc, yh, yv = gt.gy_terms(LP, EA, EB)
    Y = np.array([sum(yc[q] * H[yh[q]] * V[yv[q]] for q in range(ys[e], ys[e + 1]))
                  for e in range(len(ys) - 1)])
    om = _omegas(LA, LB, Gt, A - B)
    t = om @ Y
    dA = 2 * za * t[0:3] - t[6:9]
    dB = 2 * zb * t[3:6] - t[9:12]
    return dA, dB


def _block(A, B, C, la, lb, LP, za, zb, zc):
    xyz, aux, orb, trip = single_triplet(A, B, C, la, lb, LP, za, zb, zc, pure=1)
    return oracle.eval_batch(xyz, aux, orb, trip)[0].reshape(2 * LP + 1, gt.ncart(la), gt.ncart(lb))


CASES = [(0, 1, 1), (2, 2, 2), (1, 3, 1), (4, 3, 2), (6, 3, 3), (3, 2, 0), (0, 0, 0), (5, 2, 1)]


@pytest.mark.parametrize("LP,la,lb", CASES)
def test_grad_engine_matches_raised_and_lowered_integrals(LP, la, lb):
    rng = np.random.default_rng(900 + 11 * LP + 3 * la + lb)
    A, B, C = rng.uniform(-1.2, 1.2, (3, 3))
    za, zb, zc = rng.uniform(0.4, 1.8, 3)
    d = rng.normal(size=2 * LP + 1)
    Gt = rng.normal(size=(gt.ncart(la), gt.ncart(lb)))
    T = oracle.solid_transform(LP)
    dA, dB = _engine_grad(LP, la, lb, A, B, C, za, zb, zc, T.T @ d, Gt)

    # d/dA_x (ab|P) = 2 za (a+1_x b|P) - a_x (a-1_x b|P), and likewise for B
    def contract(blk):
        return np.einsum("m,mab->ab", d, blk)
    up_a = contract(_block(A, B, C, la + 1, lb, LP, za, zb, zc))
    up_b = contract(_block(A, B, C, la, lb + 1, LP, za, zb, zc))
    dn_a = contract(_block(A, B, C, la - 1, lb, LP, za, zb, zc)) if la > 0 else None
    dn_b = contract(_block(A, B, C, la, lb - 1, LP, za, zb, zc)) if lb > 0 else None
    refA, refB = np.zeros(3), np.zeros(3)
    for ai, a in enumerate(gt.carts(la)):
        for bi, b in enumerate(gt.carts(lb)):
            for x in range(3):
                ap = list(a); ap[x] += 1
                vA = 2 * za * up_a[gt.cidx(tuple(ap)), bi]
                if a[x] > 0:
                    am = list(a); am[x] -= 1
                    vA -= a[x] * dn_a[gt.cidx(tuple(am)), bi]
                bp = list(b); bp[x] += 1
                vB = 2 * zb * up_b[ai, gt.cidx(tuple(bp))]
                if b[x] > 0:
                    bm = list(b); bm[x] -= 1
                    vB -= b[x] * dn_b[ai, gt.cidx(tuple(bm))]
                refA[x] += Gt[ai, bi] * vA
                refB[x] += Gt[ai, bi] * vB
    scale = max(np.abs(refA).max(), np.abs(refB).max())
    np.testing.assert_allclose(dA, refA, rtol=1e-10, atol=1e-13 * scale)
    np.testing.assert_allclose(dB, refB, rtol=1e-10, atol=1e-13 * scale)


@pytest.mark.parametrize("LP,la,lb", [(2, 2, 2), (4, 3, 2), (1, 1, 0)])
def test_grad_engine_matches_central_differences(LP, la, lb):
    rng = np.random.default_rng(950 + 11 * LP + 3 * la + lb)
    A, B, C = rng.uniform(-1.2, 1.2, (3, 3))
    za, zb, zc = rng.uniform(0.4, 1.8, 3)
    d = rng.normal(size=2 * LP + 1)
    Gt = rng.normal(size=(gt.ncart(la), gt.ncart(lb)))
    T = oracle.solid_transform(LP)
    dA, dB = _engine_grad(LP, la, lb, A, B, C, za, zb, zc, T.T @ d, Gt)

    def L(A_, B_):
        return np.einsum("m,mab,ab->", d, _block(A_, B_, C, la, lb, LP, za, zb, zc), Gt)
    h = 1e-4
    fdA = np.array([(L(A + h * np.eye(3)[x], B) - L(A - h * np.eye(3)[x], B)) / (2 * h)
                    for x in range(3)])
    fdB = np.array([(L(A, B + h * np.eye(3)[x]) - L(A, B - h * np.eye(3)[x])) / (2 * h)
                    for x in range(3)])
    scale = max(np.abs(fdA).max(), np.abs(fdB).max())
    np.testing.assert_allclose(dA, fdA, rtol=1e-6, atol=1e-8 * scale)
    np.testing.assert_allclose(dB, fdB, rtol=1e-6, atol=1e-8 * scale)


def test_grad_engine_y_table_terms():
    """Every (u <= e, |u| <= L_P) pair of every target appears once, with the
    falling-factorial weight."""
    for LP in range(7):
        for (lp, EA, EB) in gt.grad_geometries():
            if lp != LP:
                continue
            ys, yc, yh, yv = gt.gy_terms(LP, EA, EB)
            es = [e for lev in range(EA, EB + 1) for e in gt.carts(lev)]
            assert len(ys) == len(es) + 1
            for ei, e in enumerate(es):
                want = sorted((gt.offT(sum(u)) + gt.cidx(u),
                               gt.offT(sum(e) - sum(u)) + gt.cidx(tuple(e[t] - u[t] for t in range(3))),
                               math.prod(math.perm(e[t], u[t]) for t in range(3)))
                              for u in [(x, y, z) for x in range(e[0] + 1) for y in range(e[1] + 1)
                                        for z in range(e[2] + 1)] if sum(u) <= LP)
                got = sorted(zip(yh[ys[ei]:ys[ei + 1]], yv[ys[ei]:ys[ei + 1]], yc[ys[ei]:ys[ei + 1]]))
                assert got == want


@pytest.mark.parametrize("la,lb", [(0, 0), (1, 0), (1, 1), (2, 1), (2, 2), (3, 1), (3, 2), (3, 3)])
def test_omega_term_table_matches_gather(la, lb):
    """The generated terms of the transposed shifted HRRs (GenOmega) give the
    twelve weight vectors of the gather above for a random G~ and AB."""
    rng = np.random.default_rng(960 + 5 * la + lb)
    Gt = rng.normal(size=(gt.ncart(la), gt.ncart(lb)))
    AB = rng.uniform(-1.5, 1.5, 3)
    ref = _omegas(la, lb, Gt, AB)
    st, co, pw, ab = gt.omega_terms(la, lb)
    flat = Gt.reshape(-1)
    got = np.array([sum(co[q] * flat[ab[q]] * np.prod(AB ** np.array(pw[q]))
                        for q in range(st[i], st[i + 1])) for i in range(len(st) - 1)])
    np.testing.assert_allclose(got, ref.reshape(-1), rtol=1e-12, atol=1e-14 * np.abs(ref).max())
