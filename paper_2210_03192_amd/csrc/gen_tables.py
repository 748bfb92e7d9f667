"""Generate the index tables of the gfx950 kernels as C++ headers.

Section 3 of the paper builds its kernels from compile-time metadata (orbital
lists, recurrence index maps).  Evaluating the larger maps in the C++ constant
evaluator is slow, so this script computes them once at build time and writes
them as literal arrays (gen/tables_lp<L>.hpp, gen/tables_common.hpp).

Conventions (must match tables.hpp):
  * Cartesian order inside a shell of l quanta: for i = 0..l, for j = 0..i:
    (l-i, i-j, j);  offT(j) = number of Cartesians of all levels below j.
  * A geometry (LP, EA, EB) computes (e0|P) for e in levels EA..EB.
    pi_k(e', n): k = 0..LP, n of level LP-k, e' of levels emin(k)..emax(k) with
    emin(k) = max(0, EA-k), emax(k) = EB-k; entry r = pi_off(k) + idx(n) nek(k)
    + (offT(|e'|) - offT(emin(k))) + idx(e').
  * n-q CVRR2 (Eq. cVRR2 applied |c| times):
        (e0|c) = sum_{u <= min(e,c)} prod_i C(c_i,u_i) e_i!/(e_i-u_i)! pi_{|u|}(e-u, c-u)
  * real solid harmonics: Re/Im (x+iy)^|m| times the associated-Legendre
    polynomial in (z, r^2) from (l-m) P_{l,m} = (2l-1) z P_{l-1,m}
    - (l+m-1) r^2 P_{l-2,m}, P_{m,m} = 1; rows m = -l..l scaled to unit norm
    under the Cartesian overlap of a shell whose x^l member has unit norm.
  * n-q HRR: (a b|P) = sum_{i <= b} prod_x C(b_x,i_x) AB_x^{b_x-i_x} (a+i 0|P).
"""
import math
import os
import sys
from fractions import Fraction

LMAX_AUX = 6
LMAX_ORB = 4
LMAX_GRAD_ORB = 4


def ncart(l):
    return (l + 1) * (l + 2) // 2 if l >= 0 else 0


def offT(j):
    return j * (j + 1) * (j + 2) // 6 if j > 0 else 0


def carts(l):
    return [(l - i, i - j, j) for i in range(l + 1) for j in range(i + 1)]


def cidx(q):
    i = q[1] + q[2]
    return i * (i + 1) // 2 + q[2]


def rdir(e):
    return 0 if e[0] > 0 else (1 if e[1] > 0 else 2)


# ----------------------------------------------------------------- geometry
class Geo:
    def __init__(self, LP, EA, EB):
        self.LP, self.EA, self.EB = LP, EA, EB

    def emin(self, k):
        return max(0, self.EA - k)

    def emax(self, k):
        return self.EB - k

    def nek(self, k):
        return offT(self.emax(k) + 1) - offT(self.emin(k)) if self.emax(k) >= self.emin(k) else 0

    def pi_off(self, k):
        return sum(ncart(self.LP - q) * self.nek(q) for q in range(k))

    def sw_off(self, k):
        return sum(ncart(self.LP - q) for q in range(k))

    @property
    def NPI(self):
        return self.pi_off(self.LP + 1)

    def pi_index(self, k, ep, n):
        return (self.pi_off(k) + cidx(n) * self.nek(k) + offT(sum(ep)) - offT(self.emin(k))
                + cidx(ep))


def pimap(g):
    sw, v = [], []
    for k in range(g.LP + 1):
        for n in range(ncart(g.LP - k)):
            for e in range(g.nek(k)):
                sw.append(g.sw_off(k) + n)
                v.append(offT(g.emin(k)) + e)
    assert len(sw) == g.NPI
    return sw, v


def combine(g):
    """Terms with u != 0, targets in [c][e''] order (the u = 0 term is the
    prerequisite block pi_0 itself, which the kernels use as the target array)."""
    start, pi, w = [], [], []
    for C in carts(g.LP):
        for e in range(g.EA, g.EB + 1):
            for E in carts(e):
                start.append(len(pi))
                for ux in range(min(E[0], C[0]) + 1):
                    for uy in range(min(E[1], C[1]) + 1):
                        for uz in range(min(E[2], C[2]) + 1):
                            u = (ux, uy, uz)
                            if u == (0, 0, 0):
                                continue
                            wt = 1
                            for i in range(3):
                                wt *= math.comb(C[i], u[i]) * math.perm(E[i], u[i])
                            ep = tuple(E[i] - u[i] for i in range(3))
                            nn = tuple(C[i] - u[i] for i in range(3))
                            pi.append(g.pi_index(sum(u), ep, nn))
                            w.append(wt)
    start.append(len(pi))
    assert max(w, default=0) < 2**31
    return start, pi, w


# ----------------------------------------------------------- solid harmonics
def pmul(p, q):
    r = {}
    for a, x in p.items():
        for b, y in q.items():
            k = (a[0] + b[0], a[1] + b[1], a[2] + b[2])
            r[k] = r.get(k, 0) + x * y
    return {k: v for k, v in r.items() if v != 0}


def padd(p, s, q, t):
    r = {}
    for k, v in p.items():
        r[k] = r.get(k, 0) + s * v
    for k, v in q.items():
        r[k] = r.get(k, 0) + t * v
    return {k: v for k, v in r.items() if v != 0}


def dfact(n):
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def solid(l):
    one, X, Y, Z = {(0, 0, 0): 1}, {(1, 0, 0): 1}, {(0, 1, 0): 1}, {(0, 0, 1): 1}
    R2 = {(2, 0, 0): 1, (0, 2, 0): 1, (0, 0, 2): 1}
    rows = {}
    for am in range(l + 1):
        A, B = one, {}
        for _ in range(am):
            A, B = padd(pmul(X, A), 1, pmul(Y, B), -1), padd(pmul(Y, A), 1, pmul(X, B), 1)
        pm2, pm1 = {}, one
        for ll in range(am + 1, l + 1):
            nx = padd(pmul(Z, pm1), Fraction(2 * ll - 1, ll - am), pmul(R2, pm2),
                      -Fraction(ll + am - 1, ll - am))
            pm2, pm1 = pm1, nx
        for sgn in (1, -1):
            if am == 0 and sgn < 0:
                continue
            S = pmul(pm1, A if sgn > 0 else B)
            row = [Fraction(S.get(q, 0)) for q in carts(l)]
            nrm = Fraction(0)
            qs = carts(l)
            for i, a in enumerate(qs):
                for j, b in enumerate(qs):
                    s = [a[t] + b[t] for t in range(3)]
                    if any(v % 2 for v in s):
                        continue
                    ov = Fraction(dfact(s[0] - 1) * dfact(s[1] - 1) * dfact(s[2] - 1), dfact(2 * l - 1))
                    nrm += row[i] * row[j] * ov
            f = 1.0 / math.sqrt(nrm)
            rows[sgn * am] = [float(v) * f if v != 0 else 0.0 for v in row]
    return [rows[m] for m in range(-l, l + 1)]


# ---------------------------------------------------------------- J engine
# With d'_c = sum_m d_m T_mc (the Cartesian image of the fitting coefficients
# of one aux shell) the d-contracted CVRR2 targets are
#   X_e = sum_c d'_c (e0|c) = sum_prim sum_u e!/(e-u)! H_u V_{e-u},
#   H_u = sum_{c >= u, |c| = LP} C(c, u) d'_c sW_{|u|}[c - u]
# (the powers of rho/(2 gamma zeta_c) cancel against those of the prerequisite
# monomials sW_k[n] = s^k (rho/zeta_c PC)^n, k + |n| = LP), and V = [e'0|0]^(LP).
# The kernels accumulate M_{u,e'} = sum_prim H_u V_{e'} per k = |u| and combine
# X_e = sum_u e!/(e-u)! M_{u,e-u} once per shell pair.
def jh_terms(LP):
    """Per u (flat index offT(|u|) + cidx(u), |u| <= LP): the terms
    (c index within level LP, sW index sw_off(|u|) + cidx(c - u), C(c, u))."""
    def sw_off(k):
        return sum(ncart(LP - q) for q in range(k))
    start, cc, sw, b = [], [], [], []
    for k in range(LP + 1):
        for u in carts(k):
            start.append(len(cc))
            for ci, c in enumerate(carts(LP)):
                if all(c[i] >= u[i] for i in range(3)):
                    n = tuple(c[i] - u[i] for i in range(3))
                    cc.append(ci)
                    sw.append(sw_off(k) + cidx(n))
                    b.append(math.comb(c[0], u[0]) * math.comb(c[1], u[1]) * math.comb(c[2], u[2]))
    start.append(len(cc))
    return start, cc, sw, b


def jm_off(g, k):
    """Offset of block k of M (ncart(k) rows x nek(k) columns, row-major)."""
    return sum(ncart(q) * g.nek(q) for q in range(k))


def jx_terms(g):
    """Per target e (levels EA..EB, flat order): the terms (index into M,
    e!/(e-u)!) of X_e = sum_u e!/(e-u)! M_{u, e-u}."""
    start, mi, co = [], [], []
    for lev in range(g.EA, g.EB + 1):
        for e in carts(lev):
            start.append(len(mi))
            for ux in range(e[0] + 1):
                for uy in range(e[1] + 1):
                    for uz in range(e[2] + 1):
                        k = ux + uy + uz
                        if k > g.LP:
                            continue
                        u = (ux, uy, uz)
                        r = (e[0] - ux, e[1] - uy, e[2] - uz)
                        col = offT(sum(r)) + cidx(r) - offT(g.emin(k))
                        assert 0 <= col < g.nek(k)
                        mi.append(jm_off(g, k) + cidx(u) * g.nek(k) + col)
                        co.append(math.perm(e[0], ux) * math.perm(e[1], uy) * math.perm(e[2], uz))
    start.append(len(mi))
    return start, mi, co


def combine_blocks(st, pi, w):
    """The CVRR2 combination terms re-laid for whole wavefronts: targets with
    terms, ordered by decreasing term count, in blocks of 64 (one per wave);
    block b holds m_b = its largest term count and its terms interleaved,
    term j of lane l at word boff[b] + 64 j + l (weight 0 past a target's own
    terms), so every lane of a wave runs the same loop with coalesced loads."""
    cnt = [st[t + 1] - st[t] for t in range(len(st) - 1)]
    order = sorted((t for t in range(len(cnt)) if cnt[t] > 0), key=lambda t: (-cnt[t], t))
    boff, bm, tg, il = [0], [], [], []
    for b0 in range(0, len(order), 64):
        ts = order[b0:b0 + 64]
        m = cnt[ts[0]]
        bm.append(m)
        for j in range(m):
            for l in range(64):
                if l < len(ts) and j < cnt[ts[l]]:
                    q = st[ts[l]] + j
                    il.append((w[q] << 16) | pi[q])
                else:
                    il.append(0)
        boff.append(len(il))
        tg.extend(ts + [0xffff] * (64 - len(ts)))
    return boff, bm, tg, il


def gg_terms(g):
    """Per u (flat index offT(|u|) + cidx(u), |u| <= min(LP, EB)): the terms
    (e!/(e-u)!, target index of e relative to level EA, VRR1 index of e - u) of
    G_u = sum_{e >= u} w_e e!/(e-u)! [e-u 0|0]^(LP) over the targets e of the
    class (the adjoint digestion engine)."""
    start, co, ei, vi = [], [], [], []
    targets = [e for lev in range(g.EA, g.EB + 1) for e in carts(lev)]
    for k in range(min(g.LP, g.EB) + 1):
        for u in carts(k):
            start.append(len(co))
            for t, e in enumerate(targets):
                if all(e[i] >= u[i] for i in range(3)):
                    r = tuple(e[i] - u[i] for i in range(3))
                    co.append(math.perm(e[0], u[0]) * math.perm(e[1], u[1]) * math.perm(e[2], u[2]))
                    ei.append(t)
                    vi.append(offT(sum(r)) + cidx(r))
    start.append(len(co))
    return start, co, ei, vi


def jy_terms(LP):
    """The terms of jh_terms regrouped per c: (u index, sW index, C(c, u)) of
    y_c = sum_{u <= c} C(c,u) sW_{|u|}[c-u] G_u."""
    hs, hc, hw, hb = jh_terms(LP)
    per_c = [[] for _ in range(ncart(LP))]
    for u in range(len(hs) - 1):
        for q in range(hs[u], hs[u + 1]):
            per_c[hc[q]].append((u, hw[q], hb[q]))
    start, uu, ww, bb = [], [], [], []
    for lst in per_c:
        start.append(len(uu))
        for u, w, b in lst:
            uu.append(u)
            ww.append(w)
            bb.append(b)
    start.append(len(uu))
    return start, uu, ww, bb


def gy_terms(LP, EA, EB):
    """Per target e (levels EA..EB, flat order): the terms (e!/(e-u)!, H_u
    index offT(|u|) + cidx(u), VRR1 index offT(|e-u|) + cidx(e-u)) of the
    per-primitive digested ket Y_e = sum_u e!/(e-u)! H_u [e-u 0|0]^(LP),
    |u| <= LP (the derivative engine)."""
    start, co, hu, vi = [], [], [], []
    for lev in range(EA, EB + 1):
        for e in carts(lev):
            start.append(len(co))
            for ux in range(e[0] + 1):
                for uy in range(e[1] + 1):
                    for uz in range(e[2] + 1):
                        k = ux + uy + uz
                        if k > LP:
                            continue
                        r = (e[0] - ux, e[1] - uy, e[2] - uz)
                        co.append(math.perm(e[0], ux) * math.perm(e[1], uy) * math.perm(e[2], uz))
                        hu.append(offT(k) + cidx((ux, uy, uz)))
                        vi.append(offT(sum(r)) + cidx(r))
    start.append(len(co))
    return start, co, hu, vi


def omega_terms(LA, LB):
    """Per weight vector j = 3 s + x (shift s = A+, B+, A-, B-; direction x)
    and target e (levels max(LA-1,0) .. LA+LB+1, flat order): the terms
    (integer coefficient, AB exponents (px, py, pz), G~ index a NB + b) of
      omega^{s,x}_e = sum_ab G~_ab sum_i [shifted a + i = e] C(b', i) AB^{b'-i}
    (the HRRs of the four shifted blocks transposed onto G~; the coefficient
    holds the binomials and the a_x or b_x factor of the lowered blocks)."""
    EA, EB = max(LA - 1, 0), LA + LB + 1
    es = [e for lev in range(EA, EB + 1) for e in carts(lev)]
    NB = ncart(LB)
    start, co, pw, ab = [], [], [], []
    for j in range(12):
        s, x = divmod(j, 3)
        las = LA + 1 if s == 0 else LA - 1 if s == 2 else LA
        for e in es:
            start.append(len(co))
            k = sum(e) - las
            if k < 0:
                continue
            for bi, b in enumerate(carts(LB)):
                bb = list(b)
                cb = 1
                if s == 1:
                    bb[x] += 1
                if s == 3:
                    if b[x] == 0:
                        continue
                    cb = b[x]
                    bb[x] -= 1
                for i in carts(k):
                    if any(i[t] > bb[t] for t in range(3)):
                        continue
                    a = [e[t] - i[t] for t in range(3)]
                    if s == 0:
                        a[x] -= 1
                    if s == 2:
                        a[x] += 1
                    if min(a) < 0:
                        continue
                    ca = a[x] if s == 2 else 1
                    co.append(ca * cb * math.prod(math.comb(bb[t], i[t]) for t in range(3)))
                    pw.append(tuple(bb[t] - i[t] for t in range(3)))
                    ab.append(cidx(tuple(a)) * NB + bi)
    start.append(len(co))
    return start, co, pw, ab


def hrrt_terms(LA, LB):
    """Per target e (levels LA .. LA+LB, flat order): the terms (C(b,i)
    product, AB exponents b - i, D~ index a NB + b) of the HRR transposed onto
    D~, w_e = sum_ab D~_ab sum_i [a + i = e] C(b,i) AB^{b-i} (gamma engine)."""
    NB = ncart(LB)
    start, co, pw, ab = [], [], [], []
    for lev in range(LA, LA + LB + 1):
        for e in carts(lev):
            start.append(len(co))
            k = lev - LA
            for bi, b in enumerate(carts(LB)):
                for i in carts(k):
                    if any(i[t] > b[t] for t in range(3)):
                        continue
                    a = tuple(e[t] - i[t] for t in range(3))
                    if min(a) < 0:
                        continue
                    co.append(math.prod(math.comb(b[t], i[t]) for t in range(3)))
                    pw.append(tuple(b[t] - i[t] for t in range(3)))
                    ab.append(cidx(a) * NB + bi)
    start.append(len(co))
    return start, co, pw, ab


def grad_geometries():
    """(LP, EA, EB) = (L_P, max(l_a - 1, 0), l_a + l_b + 1) of the gradient
    classes (l_a >= l_b, up to the gradient's orbital limit)."""
    return sorted({(LP, max(la - 1, 0), la + lb + 1)
                   for LP in range(LMAX_AUX + 1)
                   for la in range(LMAX_GRAD_ORB + 1) for lb in range(la + 1)})


# ----------------------------------------------------------------------- HRR
def hrr(LA, LB):
    hc_start, hc_pow, hc_binom = [], [], []
    n = 0
    for q in carts(LB):
        hc_start.append(n)
        for ix in range(q[0] + 1):
            for iy in range(q[1] + 1):
                for iz in range(q[2] + 1):
                    hc_pow += [q[0] - ix, q[1] - iy, q[2] - iz, 0]
                    hc_binom.append(math.comb(q[0], ix) * math.comb(q[1], iy) * math.comb(q[2], iz))
                    n += 1
    hc_start.append(n)
    e = []
    for A in carts(LA):
        for q in carts(LB):
            for ix in range(q[0] + 1):
                for iy in range(q[1] + 1):
                    for iz in range(q[2] + 1):
                        E = (A[0] + ix, A[1] + iy, A[2] + iz)
                        e.append(offT(sum(E)) - offT(LA) + cidx(E))
    return hc_start, hc_pow, hc_binom, e


# ---------------------------------------------------------------------- VRR1
def vstages(L):
    if L == 0:
        return []
    if L % 2:
        return [(1, False)] + [(1 + 2 * s, True) for s in range(1, (L - 1) // 2 + 1)]
    return [(2 + 2 * s, True) for s in range(L // 2)]


def vtab(L):
    items = []

    def one_q(o, c, m):
        e = carts(o)[c]
        i = rdir(e)
        e1 = list(e)
        e1[i] -= 1
        e2 = list(e)
        e2[i] -= 2
        return (0, c, m, i, 0, cidx(e1), cidx(e2) if e[i] >= 2 else -1, e[i] - 1, -1, 0)

    for j, twoq in vstages(L):
        if twoq:
            for c in range(ncart(j - 1)):
                for m in range(L - j + 2):
                    items.append(one_q(j - 1, c, m))
            for c in range(ncart(j)):
                for m in range(L - j + 1):
                    e = carts(j)[c]
                    i = rdir(e)
                    x = list(e)
                    x[i] -= 1
                    ip = rdir(x)
                    x1, x2, y = list(x), list(x), list(e)
                    x1[ip] -= 1
                    x2[ip] -= 2
                    y[i] -= 2
                    items.append((1, c, m, i, ip, cidx(x1), cidx(x2) if x[ip] >= 2 else -1,
                                  x[ip] - 1, cidx(y) if e[i] >= 2 else -1, e[i] - 1))
        else:
            for c in range(ncart(j)):
                for m in range(L - j + 1):
                    items.append(one_q(j, c, m))
    return items


def vofs(L):
    """Operand and destination offsets of every VRR1 item, relative to the T
    region of a primitive record (the layout of device.hpp's vrr1): T holds the
    m = 0 values of all levels at offT(level) + c; W (at NT) holds the higher m
    of the two most recent levels, the lower one first.  Per item:
    (u0, u1, u2, l0, l1, l2, y0, y1, dst, axes, f1, f2) with
    axes = i | ip << 2 | q << 4 (for a 1-quantal item ip = i).  A missing operand
    points at offset 0 and has a zero coefficient."""
    NT = offT(L + 1)
    items = vtab(L)
    out, k = [], 0
    for j, twoq in vstages(L):
        hu = j - 2 if twoq else j - 1
        hl = hu - 1
        win_u = ncart(hl) * (L - hl) if hl >= 0 else 0
        wout_hi = ncart(j - 1) * (L - j + 1) if twoq else L
        n = ncart(j) * (L - j + 1) + (ncart(j - 1) * (L - j + 2) if twoq else 0)

        def up(c, mm):
            return offT(hu) + c if mm == 0 else NT + win_u + (mm - 1) * ncart(hu) + c

        def lw(c, mm):
            if c < 0:
                return 0
            return offT(hl) + c if mm == 0 else NT + (mm - 1) * ncart(hl) + c

        for (q, c, m, i, ip, a1, a2, f1, y, f2) in items[k:k + n]:
            lvl = j if (q == 1 or not twoq) else j - 1
            wout = wout_hi if lvl == j else 0
            dst = offT(lvl) + c if m == 0 else NT + wout + (m - 1) * ncart(lvl) + c
            if q == 0:
                assert (a2 >= 0) or f1 == 0
                out.append((up(a1, m), up(a1, m + 1), 0, lw(a2, m), lw(a2, m + 1), 0, 0, 0, dst,
                            i | (i << 2), f1, 0))
            else:
                assert (a2 >= 0 or f1 == 0) and (y >= 0 or f2 == 0)
                yy = (up(y, m), up(y, m + 1)) if y >= 0 else (0, 0)
                out.append((up(a1, m), up(a1, m + 1), up(a1, m + 2), lw(a2, m), lw(a2, m + 1),
                            lw(a2, m + 2), yy[0], yy[1], dst, i | (ip << 2) | 16, f1, f2))
        k += n
    assert k == len(items)
    nw = L
    for j in range(1, L + 1):
        nw = max(nw, (ncart(j - 1) * (L - j + 1)) + ncart(j) * (L - j))
    assert all(0 <= x < NT + nw for t in out for x in t[:9])
    return out, NT, nw


# -------------------------------------------------------------------- output
def arr(ctype, name, vals):
    if not vals:
        vals = [0]
    body = ",".join(str(v) for v in vals)
    return f"  static constexpr {ctype} {name}[{len(vals)}] = {{{body}}};\n"


def _write_if_changed(path, text):
    """Keep the timestamp of unchanged headers so incremental builds stay valid."""
    if os.path.exists(path):
        with open(path) as f:
            if f.read() == text:
                return
    with open(path, "w") as f:
        f.write(text)


def geometries():
    """(LP, EA, EB) = (L_P, l_a, l_a + l_b) of every (l_a, l_b) pair up to the
    orbital limit, in both orders: the forward classes use l_a >= l_b, the
    derivative classes also need the raised / lowered pairs; and (L_P, l_Q, l_Q)
    of the two-centre metric up to the aux limit."""
    out = set()
    for LP in range(LMAX_AUX + 1):
        for la in range(LMAX_ORB + 1):
            for lb in range(LMAX_ORB + 1):
                out.add((LP, la, la + lb))
        # two-centre metric (P|Q): Q as a bra of l_Q with an s partner
        for lq in range(LMAX_AUX + 1):
            out.add((LP, lq, lq))
    return sorted(out)


def write(outdir):
    os.makedirs(outdir, exist_ok=True)
    geos = geometries()
    for LP in range(LMAX_AUX + 1):
        s = ["// generated by gen_tables.py -- do not edit\n#pragma once\n#include <cstdint>\n",
             "namespace df3c {\n"]
        for (lp, EA, EB) in geos:
            if lp != LP:
                continue
            g = Geo(LP, EA, EB)
            sw, v = pimap(g)
            st, pi, w = combine(g)
            s.append(f"template <> struct GenTab<{LP}, {EA}, {EB}> {{\n")
            s.append(f"  static constexpr int NPI = {g.NPI};\n")
            s.append(f"  static constexpr int NTGT = {len(st) - 1};\n")
            s.append(arr("int16_t", "pi_sw", sw))
            s.append(arr("int16_t", "pi_v", v))
            s.append(arr("int32_t", "cb_start", st))
            # one word per term: weight << 16 | prerequisite index
            assert max(pi, default=0) < 65536 and max(w, default=0) < 65536
            s.append(arr("uint32_t", "cb_pw", [(ww << 16) | pp for pp, ww in zip(pi, w)]))
            boff, bm, tg, il = combine_blocks(st, pi, w)
            s.append(f"  static constexpr int NCB = {len(bm)}, CBM = {max(bm, default=0)};\n")
            s.append(arr("int32_t", "cb_boff", boff))
            s.append(arr("int16_t", "cb_bm", bm))
            s.append(arr("uint16_t", "cb_tg", tg))
            s.append(arr("uint32_t", "cb_il", il))
            js, jm, jc = jx_terms(g)
            s.append(f"  static constexpr int NM = {jm_off(g, LP + 1)};\n")
            s.append(arr("int16_t", "jx_start", js))
            # one word per term: coefficient << 16 | index into M
            assert max(jm, default=0) < 65536 and max(jc, default=0) < 65536
            s.append(arr("uint32_t", "jx_mc", [(cc << 16) | mm for mm, cc in zip(jm, jc)]))
            gs, gc, ge, gv = gg_terms(g)
            s.append(arr("int16_t", "g_start", gs))
            # one word per term: coefficient << 16 | target index << 8 | VRR1 index
            assert max(ge, default=0) < 256 and max(gv, default=0) < 256 and max(gc, default=0) < 65536
            s.append(arr("uint32_t", "g_t", [(c << 16) | (e << 8) | v for c, e, v in zip(gc, ge, gv)]))
            s.append("};\n")
        for (lp, EA, EB) in grad_geometries():
            if lp != LP:
                continue
            ys, yc, yh, yv = gy_terms(LP, EA, EB)
            s.append(f"template <> struct GenY<{LP}, {EA}, {EB}> {{\n")
            s.append(arr("int16_t", "y_start", ys))
            # one word per term: coefficient << 16 | H_u index << 8 | VRR1 index
            assert max(yh) < 256 and max(yv) < 256 and max(yc) < 65536
            s.append(arr("uint32_t", "y_t", [(c << 16) | (h << 8) | v for c, h, v in zip(yc, yh, yv)]))
            s.append("};\n")
        s.append("}  // namespace df3c\n")
        _write_if_changed(os.path.join(outdir, f"tables_lp{LP}.hpp"), "".join(s))
    s = ["// generated by gen_tables.py -- do not edit\n#pragma once\n#include <cstdint>\n",
         "namespace df3c {\n"]
    for l in range(LMAX_AUX + 1):
        rows = solid(l)
        start, col, val = [], [], []
        for r in rows:
            start.append(len(col))
            for c, x in enumerate(r):
                if x != 0.0:
                    col.append(c)
                    val.append(repr(x))
        start.append(len(col))
        s.append(f"template <> struct GenSolid<{l}> {{\n")
        s.append(arr("int16_t", "start", start))
        s.append(arr("int16_t", "col", col))
        s.append(arr("double", "val", val))
        s.append(arr("double", "dense", [repr(x) for r in rows for x in r]))
        hs, hc, hw, hb = jh_terms(l)
        s.append(arr("int16_t", "jh_start", hs))
        # one word per term: binomial << 16 | sW index << 8 | c
        assert max(hc, default=0) < 256 and max(hw, default=0) < 256 and max(hb, default=0) < 65536
        s.append(arr("uint32_t", "jh_t", [(bb << 16) | (ww << 8) | cc
                                          for cc, ww, bb in zip(hc, hw, hb)]))
        ys, yu, yw, yb = jy_terms(l)
        s.append(arr("int16_t", "jy_start", ys))
        # one word per term: binomial << 16 | sW index << 8 | u
        assert max(yu, default=0) < 256 and max(yw, default=0) < 256
        s.append(arr("uint32_t", "jy_t", [(bb << 16) | (ww << 8) | uu
                                          for uu, ww, bb in zip(yu, yw, yb)]))
        s.append("};\n")
    for la in range(LMAX_ORB + 1):
        for lb in range(LMAX_ORB + 1):
            hs, hp, hb, e = hrr(la, lb)
            s.append(f"template <> struct GenHrr<{la}, {lb}> {{\n")
            s.append(f"  static constexpr int NHC = {hs[-1]};\n")
            s.append(arr("int16_t", "hc_start", hs))
            s.append(arr("int8_t", "hc_pow", hp))
            s.append(arr("int16_t", "hc_binom", hb))
            s.append(arr("int16_t", "e", e))
            s.append("};\n")
    for la in range(LMAX_GRAD_ORB + 1):
        for lb in range(la + 1):
            st, co, pw, ab = omega_terms(la, lb)
            s.append(f"template <> struct GenOmega<{la}, {lb}> {{\n")
            s.append(arr("int32_t", "o_start", st))
            # one word per term: coefficient << 24 | px << 20 | py << 16 | pz << 12 | G~ index
            assert max(co, default=0) < 256 and max(ab, default=0) < 4096
            assert max((max(p) for p in pw), default=0) < 16
            s.append(arr("uint32_t", "o_t", [(c << 24) | (p[0] << 20) | (p[1] << 16) | (p[2] << 12) | i
                                             for c, p, i in zip(co, pw, ab)]))
            s.append("};\n")
    for la in range(LMAX_ORB + 1):
        for lb in range(la + 1):
            st, co, pw, ab = hrrt_terms(la, lb)
            s.append(f"template <> struct GenHrrT<{la}, {lb}> {{\n")
            s.append(arr("int32_t", "w_start", st))
            # one word per term: coefficient << 24 | px << 20 | py << 16 | pz << 12 | D~ index
            assert max(co, default=0) < 256 and max(ab, default=0) < 4096
            s.append(arr("uint32_t", "w_t", [(c << 24) | (p[0] << 20) | (p[1] << 16) | (p[2] << 12) | i
                                             for c, p, i in zip(co, pw, ab)]))
            s.append("};\n")
    for L in range(2 * LMAX_ORB + 2):
        items = vtab(L)
        s.append(f"template <> struct GenV<{L}> {{\n")
        s.append(f"  static constexpr int N = {len(items)};\n")
        ofs, nt, nw = vofs(L)
        s.append(f"  static constexpr int NT = {nt}, NW = {nw};\n")
        s.append(arr("VO", "ofs", ["{" + ",".join(str(x) for x in t) + ",0,0,0,0}" for t in ofs]))
        s.append("};\n")
    s.append("}  // namespace df3c\n")
    _write_if_changed(os.path.join(outdir, "tables_common.hpp"), "".join(s))


# Boys table of device.hpp (kept in the library's code object): F_m(i DT) for
# i = 0..NGRID-1 and m = 0..MTAB-1, row-major, from the series
#   F_m(T) = exp(-T) sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1))
# (all terms positive) in 40-digit decimal arithmetic, rounded once to double.
BOYS_DT = Fraction(1, 8)
BOYS_TMAX = 36
BOYS_NGRID = int(BOYS_TMAX / BOYS_DT) + 1
BOYS_MTAB = 17 + 10  # highest order used + Taylor terms


def boys_table():
    import decimal
    ctx = decimal.Context(prec=40)
    out = []
    for i in range(BOYS_NGRID):
        T = ctx.divide(decimal.Decimal(i * BOYS_DT.numerator), decimal.Decimal(BOYS_DT.denominator))
        eT = ctx.exp(-T)
        two_t = ctx.multiply(2, T)
        for m in range(BOYS_MTAB):
            term = ctx.divide(decimal.Decimal(1), decimal.Decimal(2 * m + 1))
            tot = term
            k = 1
            while True:
                term = ctx.divide(ctx.multiply(term, two_t), decimal.Decimal(2 * m + 2 * k + 1))
                tot = ctx.add(tot, term)
                if term < tot * decimal.Decimal("1e-36"):
                    break
                k += 1
            out.append(float(ctx.multiply(eT, tot)))
    return out


def write_boys(outdir):
    vals = boys_table()
    lines = [f"// generated by gen_tables.py -- do not edit: F_m(i/8), i < {BOYS_NGRID}, "
             f"m < {BOYS_MTAB}, row-major\n"]
    for i in range(0, len(vals), 4):
        lines.append(", ".join(repr(v) for v in vals[i:i + 4]) + ",\n")
    _write_if_changed(os.path.join(outdir, "boys_table.inc"), "".join(lines))


if __name__ == "__main__":
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(__file__), "gen")
    write(out)
    write_boys(out)
