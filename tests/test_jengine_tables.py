"""The generated J-engine tables (GenSolid<l>::jh_*, GenTab<LP,EA,EB>::jx_*)
read with the kernels' formulas reproduce the oracle's d-contracted integrals.

For one primitive triplet (bra level e at A with exponent za, s at B, pure aux
shell of l = L_P at C) the engine forms
  H_u = sum_{c >= u} C(c,u) d'_c sW_{|u|}[c-u],   d' = T^T d,
  M_{u,e'} = H_u V_{e'},  V = [e'0|0]^(L_P)  (VRR1 at m = L_P),
  X_e = sum_u e!/(e-u)! M_{u,e-u},
which must equal sum_m d_m (P_m | e s) for every e in [l_a, l_a + l_b]
(Eq. cVRR2 in n-quantal form applied to the prerequisites of Eq. a0cv2, with
the fitting coefficients digested into the ket).  The VRR1 stage is the
emulation of test_vrr1_tables (itself pinned to the oracle at L_P = 0).
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


def _vrr1(L, LP, PA, rp, i2g, rg, pre, F):
    ofs, NT, NW = gt.vofs(L)
    rec = np.zeros(NT + NW)
    rec[0] = pre * F[LP]
    for mm in range(1, L + 1):
        rec[NT + mm - 1] = pre * F[LP + mm]
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
    return rec[:NT]


def _engine_X(LP, EA, EB, A, B, C, za, zb, zc, dprime):
    g = za + zb
    P = (za * A + zb * B) / g
    rho = g * zc / (g + zc)
    PA, PC = P - A, P - C
    pre = 2 * math.pi ** 2.5 / (math.sqrt(g + zc) * g * zc) * math.exp(-za * zb / g * (A - B) @ (A - B))
    F = oracle.boys(LP + EB, rho * PC @ PC)
    V = _vrr1(EB, LP, PA, rho / g * PC, 0.5 / g, rho / g, pre, F)
    # sW_k[n] = s^k (rho/zc PC)^n, k + |n| = LP, in sw_off(k) + cidx(n) order
    s, w = rho / (2 * g * zc), rho / zc * PC
    sw = [s ** k * np.prod(w ** np.array(n)) for k in range(LP + 1) for n in gt.carts(LP - k)]
    hs, hc, hsw, hb = gt.jh_terms(LP)
    H = [sum(hb[q] * dprime[hc[q]] * sw[hsw[q]] for q in range(hs[u], hs[u + 1]))
         for u in range(len(hs) - 1)]
    geo = gt.Geo(LP, EA, EB)
    M = np.zeros(gt.jm_off(geo, LP + 1))
    for k in range(LP + 1):
        for ui, u in enumerate(gt.carts(k)):
            for col in range(geo.nek(k)):
                M[gt.jm_off(geo, k) + ui * geo.nek(k) + col] = \
                    H[gt.offT(k) + ui] * V[gt.offT(geo.emin(k)) + col]
    xs, xm, xc = gt.jx_terms(geo)
    return np.array([sum(xc[q] * M[xm[q]] for q in range(xs[e], xs[e + 1]))
                     for e in range(len(xs) - 1)])


@pytest.mark.parametrize("LP,la,lb", [(0, 0, 0), (1, 1, 0), (2, 1, 1), (3, 2, 1), (4, 2, 2),
                                      (6, 3, 3), (6, 4, 4), (5, 4, 0), (2, 0, 0)])
def test_jengine_tables_reproduce_oracle(LP, la, lb):
    rng = np.random.default_rng(500 + 7 * LP + la + 3 * lb)
    A, B, C = rng.uniform(-1.2, 1.2, (3, 3))
    za, zb, zc = rng.uniform(0.4, 1.8, 3)
    d = rng.normal(size=2 * LP + 1)
    T = oracle.solid_transform(LP)
    X = _engine_X(LP, la, la + lb, A, B, C, za, zb, zc, T.T @ d)
    ref = []
    for e in range(la, la + lb + 1):
        xyz, aux, orb, trip = single_triplet(A, B, C, e, 0, LP, za, zb, zc, pure=1)
        blk = oracle.eval_batch(xyz, aux, orb, trip)[0].reshape(2 * LP + 1, gt.ncart(e))
        ref.append(d @ blk)
    ref = np.concatenate(ref)
    np.testing.assert_allclose(X, ref, rtol=1e-10, atol=1e-13 * np.abs(ref).max())


def test_jengine_table_sizes():
    for LP in range(7):
        hs, hc, hsw, hb = gt.jh_terms(LP)
        assert len(hs) - 1 == gt.offT(LP + 1)
        # every (c, u <= c) pair appears once
        assert len(hc) == sum(int(np.prod([c[i] + 1 for i in range(3)])) for c in gt.carts(LP))
        for la in range(5):
            for lb in range(la + 1):
                geo = gt.Geo(LP, la, la + lb)
                xs, xm, xc = gt.jx_terms(geo)
                # each M entry is used by exactly one target
                assert sorted(xm) == list(range(gt.jm_off(geo, LP + 1)))


def test_combine_blocks_hold_every_term_once():
    """The wavefront layout of the CVRR2 combination (blocks of 64 targets,
    terms interleaved, weight-0 padding) holds exactly the CSR terms."""
    for c in [(6, 4, 8), (6, 3, 6), (4, 2, 4), (2, 1, 2), (0, 0, 0), (3, 3, 3)]:
        g = gt.Geo(*c)
        st, pi, w = gt.combine(g)
        boff, bm, tg, il = gt.combine_blocks(st, pi, w)
        got = {}
        for b in range(len(bm)):
            for l in range(64):
                t = tg[64 * b + l]
                terms = [il[boff[b] + 64 * j + l] for j in range(bm[b])]
                if t == 0xffff:
                    assert all(x == 0 for x in terms)
                    continue
                got[t] = sorted(x for x in terms if x >> 16)
                assert len(got[t]) == st[t + 1] - st[t]
        want = {t: sorted((w[q] << 16) | pi[q] for q in range(st[t], st[t + 1]))
                for t in range(len(st) - 1) if st[t + 1] > st[t]}
        assert got == want
