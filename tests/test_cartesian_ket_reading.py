"""The Cartesian-ket reading the store kernels use for aux shells with
pure = 0, checked in exact-enough arithmetic on primitive integrals.

The paper's VRR2 (Section 2.2, Eq. vrr2) drops the ket's own lowering term;
the two-term recursion it keeps is exact only after the solid-harmonic
projection.  The kernels rebuild a Cartesian ket of l quanta as

  (e0|c) = sum_{cs} sum_{|d| = cs, 2d <= c} c! / ((c - 2d)! d!) T'_{c-2d},

where T' is the two-term ket of degree l - 2 cs whose Boys values are
F'_m = (4 eta)^{-cs} sum_j C(cs, j) (-rho/eta)^j F_{m+j}.  Here both sides
are evaluated by plain recursions in Python (full three-term Obara-Saika for
the left side), independent of the oracle and of the kernels."""
import itertools
import math
from functools import lru_cache

import numpy as np
import pytest
from scipy.special import hyp1f1


def _boys(m, T):
    return hyp1f1(m + 0.5, m + 1.5, -T) / (2 * m + 1)


def _sub(v, i):
    v = list(v)
    v[i] -= 1
    return tuple(v)


class _Prim:
    def __init__(self, seed):
        rng = np.random.default_rng(seed)
        self.A, self.B, self.C = rng.uniform(-1.5, 1.5, (3, 3))
        za, zb, self.eta = np.exp(rng.uniform(np.log(0.2), np.log(5.0), 3))
        self.zeta = za + zb
        self.P = (za * self.A + zb * self.B) / self.zeta
        self.rho = self.zeta * self.eta / (self.zeta + self.eta)
        self.W = (self.zeta * self.P + self.eta * self.C) / (self.zeta + self.eta)
        T = self.rho * float(np.sum((self.P - self.C) ** 2))
        self.F = [_boys(m, T) for m in range(40)]

    def bra(self, F):
        """[e0|0]^(m) from the base sequence F (bra VRR, linear in F)."""
        P, A, W, zeta, rho = self.P, self.A, self.W, self.zeta, self.rho

        @lru_cache(None)
        def b(e, m):
            if min(e) < 0:
                return 0.0
            if sum(e) == 0:
                return F[m]
            i = next(k for k in range(3) if e[k] > 0)
            e1 = _sub(e, i)
            r = (P - A)[i] * b(e1, m) + (W - P)[i] * b(e1, m + 1)
            if e1[i] > 0:
                r += e1[i] / (2 * zeta) * (b(_sub(e1, i), m) - rho / zeta * b(_sub(e1, i), m + 1))
            return r
        return b

    def full(self, e, c):
        """Three-term ket recursion (full Obara-Saika), m = 0."""
        b = self.bra(self.F)
        W, C, zeta, eta, rho = self.W, self.C, self.zeta, self.eta, self.rho

        @lru_cache(None)
        def f(e, c, m):
            if min(e) < 0 or min(c) < 0:
                return 0.0
            if sum(c) == 0:
                return b(e, m)
            i = next(k for k in range(3) if c[k] > 0)
            c1 = _sub(c, i)
            r = (W - C)[i] * f(e, c1, m + 1)
            if e[i] > 0:
                r += e[i] / (2 * (zeta + eta)) * f(_sub(e, i), c1, m + 1)
            if c1[i] > 0:
                r += c1[i] / (2 * eta) * (f(e, _sub(c1, i), m) - rho / eta * f(e, _sub(c1, i), m + 1))
            return r
        return f(e, c, 0)

    def two_term(self, e, c, cs):
        """Two-term ket (the paper's VRR2) with the modified Boys values."""
        q = -self.rho / self.eta
        F = [(4 * self.eta) ** (-cs) * sum(math.comb(cs, j) * q ** j * self.F[m + j]
                                           for j in range(cs + 1)) for m in range(30)]
        b = self.bra(F)
        W, C, zeta, eta = self.W, self.C, self.zeta, self.eta

        @lru_cache(None)
        def t(e, c, m):
            if min(e) < 0 or min(c) < 0:
                return 0.0
            if sum(c) == 0:
                return b(e, m)
            i = next(k for k in range(3) if c[k] > 0)
            c1 = _sub(c, i)
            r = (W - C)[i] * t(e, c1, m + 1)
            if e[i] > 0:
                r += e[i] / (2 * (zeta + eta)) * t(_sub(e, i), c1, m + 1)
            return r
        return t(e, c, 0)

    def composed(self, e, c):
        l = sum(c)
        v = 0.0
        for cs in range(l // 2 + 1):
            for d in itertools.product(range(cs + 1), repeat=3):
                if sum(d) != cs or any(2 * d[i] > c[i] for i in range(3)):
                    continue
                t = tuple(c[i] - 2 * d[i] for i in range(3))
                w = 1.0
                for i in range(3):
                    w *= math.factorial(c[i]) / (math.factorial(t[i]) * math.factorial(d[i]))
                v += w * self.two_term(e, t, cs)
        return v


def _carts(l):
    return [(l - i, i - j, j) for i in range(l + 1) for j in range(i + 1)]


@pytest.mark.parametrize("l", range(7))
def test_cartesian_ket_from_two_term_kets(l):
    p = _Prim(100 + l)
    for c in _carts(l):
        for e in [(0, 0, 0), (1, 0, 0), (0, 2, 1), (2, 1, 1), (0, 0, 4)]:
            ref = p.full(e, c)
            assert abs(p.composed(e, c) - ref) <= 1e-13 * max(1.0, abs(ref)), (c, e)


def test_two_term_alone_is_not_cartesian_for_l_2():
    """The dropped term matters: for l = 2 the two-term ket alone differs from
    the Cartesian one by O(1) (so the lower-degree launch is needed)."""
    p = _Prim(7)
    e, c = (1, 0, 0), (2, 0, 0)
    assert abs(p.two_term(e, c, 0) - p.full(e, c)) > 1e-3 * abs(p.full(e, c))
