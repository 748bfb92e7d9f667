"""The gamma engine's formulas, emulated on the CPU with the generated tables
(GenTab::g_*, GenSolid::jy_*, VRR1 stages), reproduce the oracle's
sum_ab D_ab (P_m|ab) for one primitive triplet.

Per pair the engine transposes the HRR onto D~,
  w_e = sum_ab D~_ab sum_i [a + i = e] C(b,i) AB^{b-i},
and per primitive forms G_u = sum_{e >= u} w_e e!/(e-u)! [e-u 0|0]^(L_P) and
y_c = sum_{u <= c} C(c,u) sW_{|u|}[c-u] G_u; gamma_m = sum_c T_mc y_c.
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


def _w(LA, LB, Dt, AB):
    es = [e for lev in range(LA, LA + LB + 1) for e in gt.carts(lev)]
    w = np.zeros(len(es))
    for ei, e in enumerate(es):
        k = sum(e) - LA
        for bi, b in enumerate(gt.carts(LB)):
            for i in gt.carts(k):
                if any(i[t] > b[t] for t in range(3)):
                    continue
                a = tuple(e[t] - i[t] for t in range(3))
                if min(a) < 0:
                    continue
                w[ei] += Dt[gt.cidx(a), bi] * math.prod(math.comb(b[t], i[t]) for t in range(3)) * \
                    math.prod(AB[t] ** (b[t] - i[t]) for t in range(3))
    return w


def _engine_gamma(LP, LA, LB, A, B, C, za, zb, zc, Dt):
    EA, EB = LA, LA + LB
    g = za + zb
    P = (za * A + zb * B) / g
    rho = g * zc / (g + zc)
    PA, PC = P - A, P - C
    pre = 2 * math.pi ** 2.5 / (math.sqrt(g + zc) * g * zc) * math.exp(-za * zb / g * (A - B) @ (A - B))
    F = oracle.boys(LP + EB, rho * PC @ PC)
    V = _vrr1(EB, LP, PA, rho / g * PC, 0.5 / g, rho / g, pre, F)
    s, wv = rho / (2 * g * zc), rho / zc * PC
    sw = [s ** k * np.prod(wv ** np.array(n)) for k in range(LP + 1) for n in gt.carts(LP - k)]
    w = _w(LA, LB, Dt, A - B)
    gs, gc, ge, gvi = gt.gg_terms(gt.Geo(LP, EA, EB))
    Gu = [sum(gc[q] * w[ge[q]] * V[gvi[q]] for q in range(gs[u], gs[u + 1]))
          for u in range(len(gs) - 1)]
    ys, yu, yw, yb = gt.jy_terms(LP)
    y = np.array([sum(yb[q] * sw[yw[q]] * Gu[yu[q]] for q in range(ys[c], ys[c + 1])
                      if yu[q] < len(Gu))
                  for c in range(gt.ncart(LP))])
    return oracle.solid_transform(LP) @ y


@pytest.mark.parametrize("LP,la,lb", [(0, 0, 0), (2, 1, 1), (3, 3, 2), (4, 3, 3), (6, 2, 2),
                                      (1, 4, 4), (6, 4, 4), (5, 3, 0)])
def test_gamma_engine_tables_reproduce_oracle(LP, la, lb):
    rng = np.random.default_rng(700 + 11 * LP + 3 * la + lb)
    A, B, C = rng.uniform(-1.2, 1.2, (3, 3))
    za, zb, zc = rng.uniform(0.4, 1.8, 3)
    Dt = rng.normal(size=(gt.ncart(la), gt.ncart(lb)))
    got = _engine_gamma(LP, la, lb, A, B, C, za, zb, zc, Dt)
    xyz, aux, orb, trip = single_triplet(A, B, C, la, lb, LP, za, zb, zc, pure=1)
    blk = oracle.eval_batch(xyz, aux, orb, trip)[0].reshape(2 * LP + 1, gt.ncart(la), gt.ncart(lb))
    ref = np.einsum("mab,ab->m", blk, Dt)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-13 * np.abs(ref).max())


def test_gamma_engine_table_shapes():
    for LP in range(7):
        ys, yu, yw, yb = gt.jy_terms(LP)
        hs, hc, hw, hb = gt.jh_terms(LP)
        assert len(yu) == len(hc) and len(ys) == gt.ncart(LP) + 1
        for la in range(5):
            for lb in range(la + 1):
                geo = gt.Geo(LP, la, la + lb)
                gs, gc, ge, gv = gt.gg_terms(geo)
                assert len(gs) - 1 == gt.offT(min(LP, la + lb) + 1)
                assert max(ge, default=0) < gt.offT(la + lb + 1) - gt.offT(la)


@pytest.mark.parametrize("la,lb", [(0, 0), (2, 1), (3, 2), (3, 3), (4, 4), (4, 0)])
def test_hrrt_term_table_matches_gather(la, lb):
    """The generated terms of the HRR transposed onto D~ (GenHrrT) give w_e of
    the gather above for a random D~ and AB."""
    rng = np.random.default_rng(760 + 5 * la + lb)
    Dt = rng.normal(size=(gt.ncart(la), gt.ncart(lb)))
    AB = rng.uniform(-1.5, 1.5, 3)
    ref = _w(la, lb, Dt, AB)
    st, co, pw, ab = gt.hrrt_terms(la, lb)
    flat = Dt.reshape(-1)
    got = np.array([sum(co[q] * flat[ab[q]] * np.prod(AB ** np.array(pw[q]))
                        for q in range(st[i], st[i + 1])) for i in range(len(st) - 1)])
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())
