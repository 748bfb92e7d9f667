"""The n-quantal CVRR2 of Section 2.5.4 and the GPU path's generated tables.

* A test-only symbolic application of Eq. cVRR2,
      (a, c + 1_i)_{k,n} = (a, c)_{k, n + 1_i} + a_i (a - 1_i, c)_{k+1, n},
  repeated until the ket is empty, reproduces the paper's worked example
  (tests/golden/cvrr2_worked_example.txt) except the one printed coefficient
  that the fixture flags (printed 1, recursion 2).
* The closed form used by the GPU table generator,
      (a0|c) = sum_{u <= min(a,c)} prod_i C(c_i,u_i) a_i!/(a_i-u_i)! (a-u 0)_{|u|, c-u},
  equals the recursion for every target of every (l_a, L_P) up to (5, 6), and
  the generated combine tables (u != 0 terms; u = 0 is the prerequisite block
  itself) index the prerequisites consistently with that form.
"""
import math
import os
import sys
from collections import defaultdict

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2210_03192_amd", "csrc"))
import gen_tables  # noqa: E402  (the GPU path's table generator, host code)

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "cvrr2_worked_example.txt")


def expand(a, c):
    """{(a', k, n): coefficient} of (a 0|c) by repeated Eq. cVRR2 (always
    peeling the first non-zero axis of c)."""
    out = defaultdict(int)
    stack = [(tuple(a), tuple(c), 0, (0, 0, 0), 1)]
    while stack:
        a, c, k, n, w = stack.pop()
        if sum(c) == 0:
            out[(a, k, n)] += w
            continue
        i = 0 if c[0] else (1 if c[1] else 2)
        c1 = list(c)
        c1[i] -= 1
        n1 = list(n)
        n1[i] += 1
        stack.append((a, tuple(c1), k, tuple(n1), w))
        if a[i] > 0:
            a1 = list(a)
            a1[i] -= 1
            stack.append((tuple(a1), tuple(c1), k + 1, n, w * a[i]))
    return {key: v for key, v in out.items() if v}


def closed_form(a, c):
    out = {}
    for ux in range(min(a[0], c[0]) + 1):
        for uy in range(min(a[1], c[1]) + 1):
            for uz in range(min(a[2], c[2]) + 1):
                u = (ux, uy, uz)
                w = 1
                for i in range(3):
                    w *= math.comb(c[i], u[i]) * math.perm(a[i], u[i])
                out[(tuple(a[i] - u[i] for i in range(3)), sum(u),
                     tuple(c[i] - u[i] for i in range(3)))] = w
    return out


def _golden():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        f = [x.strip() for x in line.split("|")]
        t = lambda s: tuple(int(v) for v in s.split(","))
        rows.append((t(f[0]), t(f[1]), t(f[2]), int(f[3]), t(f[4]), int(f[5])))
    return rows


def test_worked_example_against_recursion():
    rows = _golden()
    by_target = defaultdict(dict)
    for a, c, ap, k, n, w in rows:
        by_target[(a, c)][(ap, k, n)] = w
    mismatches = []
    for (a, c), printed in by_target.items():
        rec = expand(a, c)
        assert set(rec) == set(printed), (a, c)
        for key, w in printed.items():
            if rec[key] != w:
                mismatches.append(((a, c), key, w, rec[key]))
    # exactly the flagged coefficient of (d_xx s|d_xx) -> (s s)_{2,0}
    assert mismatches == [(((2, 0, 0), (2, 0, 0)), ((0, 0, 0), 2, (0, 0, 0)), 1, 2)]


@pytest.mark.parametrize("la", range(0, 6))
@pytest.mark.parametrize("lc", range(0, 7))
def test_closed_form_equals_recursion(la, lc):
    for a in gen_tables.carts(la):
        for c in gen_tables.carts(lc):
            assert closed_form(a, c) == expand(a, c), (a, c)


@pytest.mark.parametrize("geo", [(2, 2, 2), (4, 2, 4), (6, 3, 6), (6, 4, 8), (3, 0, 4), (1, 4, 4)])
def test_generated_combine_tables(geo):
    """Decode every generated term back to (e', k, n) and compare with the
    closed form; the u = 0 term must be the target's own pi_0 entry."""
    LP, EA, EB = geo
    g = gen_tables.Geo(LP, EA, EB)
    start, pi, w = gen_tables.combine(g)
    decode = {}
    for k in range(LP + 1):
        for ni, n in enumerate(gen_tables.carts(LP - k)):
            for lev in range(g.emin(k), g.emax(k) + 1):
                for e in gen_tables.carts(lev):
                    decode[g.pi_index(k, e, n)] = (e, k, n)
    t = 0
    for c in gen_tables.carts(LP):
        for lev in range(EA, EB + 1):
            for e in gen_tables.carts(lev):
                terms = {decode[pi[q]]: w[q] for q in range(start[t], start[t + 1])}
                ref = closed_form(e, c)
                assert ref.pop((e, 0, c)) == 1
                assert decode[g.pi_index(0, e, c)] == (e, 0, c) and g.pi_index(0, e, c) == t
                assert terms == ref, (e, c)
                t += 1
    assert t == len(start) - 1
