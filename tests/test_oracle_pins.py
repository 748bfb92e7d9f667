"""Pins of the CPU oracle against things other than itself.

Each test ties a part of the oracle to a closed form, a library routine, an
independent quadrature, a symmetry or a limit that the mathematics fixes:

  * Boys function (Appendix "Notation" definition): F_m(0) = 1/(2m+1), the
    incomplete-gamma identity via scipy, Gauss-Legendre quadrature of the
    defining integral, the large-T asymptote, dF_m/dT = -F_{m+1};
  * real solid harmonics: harmonic polynomials, orthonormal under the
    Cartesian overlap, proportional to scipy's spherical harmonics;
  * (s|ss): the closed form of Section 2.5.2 with F_0 from erf;
  * any primitive class with l <= 2 (and a few l = 3): brute-force quadrature
    of the defining 6-D integral (tests/quadrature.py);
  * (P|ab) = (P|ba)^T, translation invariance, rotation covariance of p shells;
  * J equals the contraction of the blocks; the gradient matches central
    differences of the oracle's own J and sums to zero over atoms although
    every centre is differentiated explicitly.
"""
import itertools
import math

import numpy as np
import pytest
from scipy.special import gamma, gammainc, sph_harm_y

import oracle
from helpers import block_shape, single_triplet
from paper_2210_03192_amd import inputs
from quadrature import carts, primitive_block

RNG = np.random.default_rng(1234)
T_GRID = [0.0, 1e-12, 1e-6, 0.01, 0.3, 1.0, 2.5, 7.0, 12.0, 20.0, 29.9, 34.99, 35.01, 40.0,
          60.0, 100.0, 117.0, 150.0, 400.0, 2000.0]


# --------------------------------------------------------------------------- Boys
def test_boys_at_zero():
    F = oracle.boys(30, 0.0)
    assert np.allclose(F, 1.0 / (2 * np.arange(31) + 1), rtol=1e-15, atol=0)


@pytest.mark.parametrize("T", [t for t in T_GRID if t >= 0.01])
def test_boys_incomplete_gamma(T):
    """F_m(T) = Gamma(m+1/2) P(m+1/2, T) / (2 T^{m+1/2}) (scipy.special)."""
    mmax = 24
    F = oracle.boys(mmax, T)
    m = np.arange(mmax + 1)
    ref = gamma(m + 0.5) * gammainc(m + 0.5, T) / (2 * T ** (m + 0.5))
    ok = ref > 1e-300
    assert np.allclose(F[ok], ref[ok], rtol=2e-14, atol=0)


@pytest.mark.parametrize("T", [1e-12, 1e-8, 1e-6])
def test_boys_small_T_series(T):
    """F_m(T) = 1/(2m+1) - T/(2m+3) + T^2/(2(2m+5)) - T^3/(6(2m+7)) + ... (Taylor
    expansion of the defining integral)."""
    F = oracle.boys(20, T)
    m = np.arange(21)
    ref = 1 / (2 * m + 1) - T / (2 * m + 3) + T ** 2 / (2 * (2 * m + 5)) - T ** 3 / (6 * (2 * m + 7))
    assert np.allclose(F, ref, rtol=1e-15, atol=0)


@pytest.mark.parametrize("T", [0.0, 1e-3, 0.5, 3.0, 15.0, 34.0, 36.0, 80.0])
def test_boys_gauss_legendre(T):
    """Defining integral int_0^1 y^{2m} exp(-T y^2) dy by 150-point Gauss-Legendre (numpy nodes, ~1e-14)."""
    x, w = np.polynomial.legendre.leggauss(150)
    y, w = (x + 1) / 2, w / 2
    F = oracle.boys(16, T)
    for m in range(17):
        ref = math.fsum(w * y ** (2 * m) * np.exp(-T * y * y))
        assert abs(F[m] - ref) <= 1e-13 * ref, (m, F[m], ref)


@pytest.mark.parametrize("T", [117.0, 200.0, 1000.0])
def test_boys_asymptotic(T):
    """For large T, F_m(T) -> (2m-1)!!/2^{m+1} sqrt(pi/T^{2m+1}) (error ~ e^{-T})."""
    F = oracle.boys(20, T)
    for m in range(21):
        df = math.prod(range(2 * m - 1, 0, -2)) if m > 0 else 1
        ref = df / 2 ** (m + 1) * math.sqrt(math.pi / T ** (2 * m + 1))
        assert abs(F[m] / ref - 1) < 1e-14


@pytest.mark.parametrize("T", [0.7, 9.0, 33.0, 37.0, 90.0])
def test_boys_derivative(T):
    """dF_m/dT = -F_{m+1}, by a 4th-order central difference."""
    h = 1e-3 * max(T, 1)
    Fs = [oracle.boys(12, T + k * h) for k in (-2, -1, 1, 2)]
    dF = (Fs[0] - 8 * Fs[1] + 8 * Fs[2] - Fs[3]) / (12 * h)
    F = oracle.boys(12, T)
    assert np.allclose(dF[:-1], -F[1:], rtol=1e-8, atol=0)


def test_boys_long_double_agrees():
    for T in T_GRID:
        a = oracle.boys(20, T)
        b = oracle.boys(20, T, precision="long")
        assert np.allclose(a, b, rtol=3e-15, atol=0), T


# ------------------------------------------------------------ solid harmonics
def _poly(l, coeffs):
    return {c: v for c, v in zip(carts(l), coeffs)}


def _laplacian(l, poly):
    out = {}
    for (x, y, z), v in poly.items():
        for k, e in enumerate((x, y, z)):
            if e >= 2:
                q = [x, y, z]
                q[k] -= 2
                out[tuple(q)] = out.get(tuple(q), 0.0) + v * e * (e - 1)
    return out


@pytest.mark.parametrize("l", range(0, 9))
def test_solid_harmonics_are_harmonic(l):
    T = oracle.solid_transform(l)
    for row in T:
        lap = _laplacian(l, _poly(l, row))
        assert all(abs(v) < 1e-12 for v in lap.values())


def _cart_overlap(l):
    q = carts(l)
    S = np.zeros((len(q), len(q)))
    df = lambda n: math.prod(range(n, 0, -2)) if n > 0 else 1
    for i, a in enumerate(q):
        for j, b in enumerate(q):
            s = [a[k] + b[k] for k in range(3)]
            if any(v % 2 for v in s):
                continue
            S[i, j] = np.prod([df(v - 1) for v in s]) / df(2 * l - 1)
    return S


@pytest.mark.parametrize("l", range(0, 9))
def test_solid_harmonics_orthonormal(l):
    T = oracle.solid_transform(l)
    assert np.allclose(T @ _cart_overlap(l) @ T.T, np.eye(2 * l + 1), atol=1e-13)


@pytest.mark.parametrize("l", range(0, 8))
def test_solid_harmonics_match_scipy(l):
    """Each row, as a function on the unit sphere, is a fixed positive multiple of
    the real combination of scipy's complex Y_lm: m > 0 -> Re, m < 0 -> Im, with
    scipy's Condon-Shortley phase (-1)^m removed."""
    rng = np.random.default_rng(501)  # own stream: independent of test order
    T = oracle.solid_transform(l)
    q = np.array(carts(l))
    pts = rng.normal(size=(40, 3))
    pts /= np.linalg.norm(pts, axis=1, keepdims=True)
    theta = np.arccos(pts[:, 2])
    phi = np.arctan2(pts[:, 1], pts[:, 0])
    mono = np.prod(pts[:, None, :] ** q[None, :, :], axis=2)
    for m in range(-l, l + 1):
        Y = sph_harm_y(l, abs(m), theta, phi) * (-1) ** abs(m)
        ref = Y.real if m >= 0 else Y.imag
        val = mono @ T[m + l]
        big = np.abs(ref) > 1e-3
        ratio = val[big] / ref[big]
        assert ratio.min() > 0 and np.ptp(ratio) < 1e-12 * abs(ratio.mean()), (l, m)


def test_solid_harmonics_p_order():
    """l = 1 pure order is m = -1, 0, +1 = (y, z, x)."""
    assert np.allclose(oracle.solid_transform(1), [[0, 1, 0], [0, 0, 1], [1, 0, 0]])


# ------------------------------------------------------------------- integrals
def _oracle_block(A, B, C, la, lb, lc, za, zb, zc, pure=0, **kw):
    xyz, aux, orb, trip = single_triplet(A, B, C, la, lb, lc, za, zb, zc, pure=pure, **kw)
    o, _ = oracle.eval_batch(xyz, aux, orb, trip, **{k: v for k, v in kw.items()
                                                     if k == "precision"})
    return o.reshape(block_shape(lc, la, lb, pure))


@pytest.mark.parametrize("same", [False, True])
def test_ssss_closed_form(same):
    """[00|0]^(0) = 2 pi^{5/2} / ((g + zc)^{1/2} g zc) exp(-za zb/g |AB|^2) F_0(rho |PC|^2),
    F_0(T) = (1/2) sqrt(pi/T) erf(sqrt T) (Section 2.5.2 at m = 0)."""
    rng = np.random.default_rng(502)  # own stream: independent of test order
    for _ in range(20):
        A, B, C = rng.uniform(-3, 3, (3, 3))
        if same:
            B = C = A
        za, zb, zc = np.exp(rng.uniform(np.log(0.05), np.log(100), 3))
        g = za + zb
        P = (za * A + zb * B) / g
        rho = g * zc / (g + zc)
        T = rho * np.sum((P - C) ** 2)
        F0 = 1.0 if T == 0 else 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))
        ref = 2 * math.pi ** 2.5 / (math.sqrt(g + zc) * g * zc) * \
            math.exp(-za * zb / g * np.sum((A - B) ** 2)) * F0
        val = _oracle_block(A, B, C, 0, 0, 0, za, zb, zc)[0, 0, 0]
        # exp(-x) carries the rounding of its argument as a relative error
        # of about x eps: the bar grows with the exponent of the overlap
        x = za * zb / g * np.sum((A - B) ** 2)
        assert abs(val - ref) <= (1e-14 + 4e-16 * x) * abs(ref)


@pytest.mark.parametrize("la,lb,lc", list(itertools.product(range(3), range(3), range(3))))
def test_primitive_vs_quadrature(la, lb, lc):
    rng = np.random.default_rng(100 * la + 10 * lb + lc)
    A, B, C = rng.uniform(-1.5, 1.5, (3, 3))
    za, zb, zc = np.exp(rng.uniform(np.log(0.2), np.log(5), 3))
    o = _oracle_block(A, B, C, la, lb, lc, za, zb, zc)
    q = primitive_block(A, B, C, la, lb, lc, za, zb, zc)
    assert np.abs(o - q).max() <= 1e-13 * np.abs(q).max()


@pytest.mark.parametrize("la,lb,lc", [(3, 0, 0), (0, 3, 1), (1, 1, 3), (3, 2, 2), (2, 3, 3),
                                      (4, 2, 4), (3, 3, 6), (4, 4, 6), (5, 5, 7)])
def test_primitive_vs_quadrature_f(la, lb, lc):
    rng = np.random.default_rng(7 + 100 * la + 10 * lb + lc)
    A, B, C = rng.uniform(-1.0, 1.0, (3, 3))
    za, zb, zc = np.exp(rng.uniform(np.log(0.3), np.log(3), 3))
    o = _oracle_block(A, B, C, la, lb, lc, za, zb, zc)
    q = primitive_block(A, B, C, la, lb, lc, za, zb, zc)
    assert np.abs(o - q).max() <= 5e-13 * np.abs(q).max()


def test_contracted_pure_vs_quadrature():
    """A contracted triplet with a pure ket: contraction and solid-harmonic
    projection applied to quadrature blocks by hand."""
    A, B, C = np.array([0.2, -0.1, 0.4]), np.array([-0.5, 0.6, 0.1]), np.array([0.3, 0.3, -0.7])
    za, zb, zc = [2.0, 0.5], [1.1, 0.3, 4.0], [0.9]
    ca, cb, cc = [0.4, 0.7], [0.2, 0.5, 0.9], [1.3]
    la, lb, lc = 1, 2, 2
    o = _oracle_block(A, B, C, la, lb, lc, za, zb, zc, pure=1, ca=ca, cb=cb, cc=cc)
    q = np.zeros(block_shape(lc, la, lb, 0))
    for (i, a), (j, b), (k, c) in itertools.product(enumerate(za), enumerate(zb), enumerate(zc)):
        q += ca[i] * cb[j] * cc[k] * primitive_block(A, B, C, la, lb, lc, a, b, c)
    # the projection is the defining step of the pure ket (Section 2.5.1)
    T = oracle.solid_transform(lc)
    assert np.allclose(o, np.einsum("pc,cab->pab", T, q), rtol=0, atol=1e-13 * np.abs(q).max())


@pytest.mark.parametrize("pure", [0, 1])
def test_bra_swap_symmetry(pure):
    rng = np.random.default_rng(40 + pure)  # own stream: independent of test order
    for la, lb, lc in [(0, 1, 2), (2, 1, 3), (3, 2, 4), (1, 3, 6)]:
        A, B, C = rng.uniform(-2, 2, (3, 3))
        za, zb, zc = [0.7, 3.1], [0.2, 1.4, 9.0], [1.1]
        x = _oracle_block(A, B, C, la, lb, lc, za, zb, zc, pure=pure)
        y = _oracle_block(B, A, C, lb, la, lc, zb, za, zc, pure=pure)
        assert np.abs(x - y.transpose(0, 2, 1)).max() <= 1e-13 * np.abs(x).max()


def test_translation_invariance():
    rng = np.random.default_rng(503)  # own stream: independent of test order
    for la, lb, lc in [(1, 1, 1), (2, 3, 4), (4, 4, 6)]:
        A, B, C = rng.uniform(-2, 2, (3, 3))
        s = rng.uniform(-10, 10, 3)
        za, zb, zc = [0.7, 3.1], [0.4], [1.1]
        x = _oracle_block(A, B, C, la, lb, lc, za, zb, zc, pure=1)
        y = _oracle_block(A + s, B + s, C + s, la, lb, lc, za, zb, zc, pure=1)
        assert np.abs(x - y).max() <= 1e-12 * np.abs(x).max()


def test_rotation_covariance_p():
    """Rotating every centre by R rotates each p index by R (Cartesian p)."""
    rng = np.random.default_rng(504)  # own stream: independent of test order
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    A, B, C = rng.uniform(-2, 2, (3, 3))
    za, zb, zc = [0.8], [1.7], [0.6]
    x = _oracle_block(A, B, C, 1, 1, 1, za, zb, zc)            # [c][a][b], Cartesian c
    y = _oracle_block(q @ A, q @ B, q @ C, 1, 1, 1, za, zb, zc)
    assert np.allclose(y, np.einsum("ci,aj,bk,ijk->cab", q, q, q, x), atol=1e-13)


def test_gamma_bilinear_identity_with_J():
    """sum_P gamma_P(D) d_P == sum_ab D_ab J_ab(d) for a non-symmetric D: gamma
    digests over the orbital pairs, J over the aux shells, in separate loops."""
    s = inputs.plain_dfj_system(seed=inputs.SEED_BASE + 71, natom=3)
    rng = np.random.default_rng(71)
    D = rng.normal(size=(s.orb.nbf, s.orb.nbf))
    d = rng.normal(size=s.aux.nbf)
    g = oracle.coulomb_gamma(s.xyz, s.aux, s.orb, D)
    J = oracle.coulomb_J(s.xyz, s.aux, s.orb, d)
    assert abs(g @ d - (D * J).sum()) <= 1e-12 * np.abs(g).max() * np.abs(d).sum()


def test_gamma_equals_block_contraction():
    """gamma against blocks of the batch entry point contracted with D by
    numpy (an orbital g shell and a Cartesian index order that a transposed D
    would break)."""
    rng = np.random.default_rng(72)
    xyz = rng.uniform(-1.5, 1.5, (2, 3))
    from paper_2210_03192_amd.inputs import _Builder
    ob, ab = _Builder(0), _Builder(1)
    for a, ls in ((0, (0, 1, 4)), (1, (2, 3))):
        for l in ls:
            ob.add(l, a, rng.uniform(0.3, 3.0, 2), rng.uniform(0.2, 1.0, 2))
    for a in (0, 1):
        for l in (0, 2, 5):
            ab.add(l, a, rng.uniform(0.2, 2.0, 1), [1.0])
    orb, aux = ob.build(), ab.build()
    D = rng.normal(size=(orb.nbf, orb.nbf))
    g = oracle.coulomb_gamma(xyz, aux, orb, D)
    trip = np.array([(P, a, b) for P in range(aux.nshell) for a in range(orb.nshell)
                     for b in range(orb.nshell)], np.int32)
    out, off = oracle.eval_batch(xyz, aux, orb, trip)
    ao, po = orb.offsets(), aux.offsets()
    ref = np.zeros(aux.nbf)
    for (P, a, b), o in zip(trip, off):
        nP, na, nb = aux.nfunc(P), orb.nfunc(a), orb.nfunc(b)
        blk = out[o:o + nP * na * nb].reshape(nP, na, nb)
        ref[po[P]:po[P + 1]] += np.einsum("pab,ab->p", blk, D[ao[a]:ao[a + 1], ao[b]:ao[b + 1]])
    np.testing.assert_allclose(g, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())


def _ss_closed(za, zb, R2):
    """Unnormalised (s_a|s_b) and F_1 of the two-centre integral."""
    from scipy.special import erf
    rho = za * zb / (za + zb)
    T = rho * R2
    F0 = 0.5 * math.sqrt(math.pi / T) * erf(math.sqrt(T))
    F1 = (F0 - math.exp(-T)) / (2 * T)
    pre = 2 * math.pi ** 2.5 / (za * zb * math.sqrt(za + zb))
    return pre * F0, pre, rho, F1


def test_metric_closed_forms():
    """(s|s) from F_0 by erf, (p_x|s) = 1/(2 zeta_p) d/dP_x (s|s) with
    dF_0/dT = -F_1 (Cartesian aux so the p components are x, y, z)."""
    from paper_2210_03192_amd.inputs import _Builder
    xyz = np.array([[0.0, 0.0, 0.0], [0.3, -0.7, 1.1]])
    za, zb = 0.8, 1.7
    b = _Builder(0)
    b.add(1, 0, [za], [1.0])
    b.add(0, 1, [zb], [1.0])
    aux = b.build()
    V = oracle.coulomb_metric(xyz, aux)
    cp, cs = aux.coefs
    R = xyz[0] - xyz[1]
    ss, pre, rho, F1 = _ss_closed(za, zb, R @ R)
    for x in range(3):
        px_s = cp * cs / (2 * za) * pre * (-F1) * 2 * rho * R[x]
        assert abs(V[x, 3] - px_s) <= 1e-13 * abs(V).max()
        assert abs(V[3, x] - px_s) <= 1e-13 * abs(V).max()
    b = _Builder(1)
    b.add(0, 0, [za], [1.0])
    b.add(0, 1, [zb], [1.0])
    aux = b.build()
    V = oracle.coulomb_metric(xyz, aux)
    c0, c1 = aux.coefs
    assert abs(V[0, 1] - c0 * c1 * ss) <= 1e-14 * abs(V[0, 1])
    # one centre: F_0(0) = 1
    assert abs(V[0, 0] - c0 * c0 * 2 * math.pi ** 2.5 / (za * za * math.sqrt(2 * za))) <= \
        1e-14 * V[0, 0]


def test_metric_symmetric_positive_definite():
    s = inputs.plain_dfj_system(seed=inputs.SEED_BASE + 91, natom=2)
    from paper_2210_03192_amd.inputs import _Builder
    rng = np.random.default_rng(91)
    b = _Builder(1)
    for a in range(2):
        for l in range(7):
            b.add(l, a, rng.uniform(0.3, 3.0, 1), [1.0])
    aux = b.build()
    V = oracle.coulomb_metric(s.xyz, aux)
    assert np.abs(V - V.T).max() <= 1e-13 * np.abs(V).max()
    assert np.linalg.eigvalsh(0.5 * (V + V.T)).min() > 0


def test_J_equals_block_contraction():
    s = inputs.plain_dfj_system()
    d = inputs.fitting_coefficients(s.aux.nbf, 7)
    J = oracle.coulomb_J(s.xyz, s.aux, s.orb, d)
    ao, po = s.orb.offsets(), s.aux.offsets()
    trip = np.array([(P, a, b) for a in range(s.orb.nshell) for b in range(s.orb.nshell)
                     for P in range(s.aux.nshell)], np.int32)
    out, off = oracle.eval_batch(s.xyz, s.aux, s.orb, trip)
    ref = np.zeros_like(J)
    for (P, a, b), o in zip(trip, off):
        na, nb, npP = s.orb.nfunc(a), s.orb.nfunc(b), s.aux.nfunc(P)
        blk = out[o:o + npP * na * nb].reshape(npP, na, nb)
        ref[ao[a]:ao[a] + na, ao[b]:ao[b] + nb] += np.einsum("pab,p->ab", blk, d[po[P]:po[P] + npP])
    assert np.allclose(J, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    pairs = np.array([[3, 1], [0, 0], [31, 17]], np.int32)
    blocks = oracle.coulomb_J_pairs(s.xyz, s.aux, s.orb, d, pairs)
    for (a, b), blk in zip(pairs, blocks):
        assert np.allclose(blk, J[ao[a]:ao[a + 1], ao[b]:ao[b + 1]], rtol=1e-14, atol=1e-14)


def _small_system():
    s = inputs.plain_dfj_system(seed=99, natom=3)
    return s, inputs.fitting_coefficients(s.aux.nbf, 3), inputs.symmetric_density(s.orb.nbf, 4)


def test_gradient_central_difference():
    s, d, G = _small_system()
    g = oracle.coulomb_J_grad(s.xyz, s.aux, s.orb, d, G)
    h = 1e-4
    fd = np.zeros_like(g)
    for X in range(len(s.xyz)):
        for i in range(3):
            vals = []
            for sgn in (1, -1):
                xyz = s.xyz.copy()
                xyz[X, i] += sgn * h
                vals.append(np.sum(G * oracle.coulomb_J(xyz, s.aux, s.orb, d)))
            fd[X, i] = (vals[0] - vals[1]) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-7 * np.abs(g).max()


def test_gradient_sums_to_zero():
    s, d, G = _small_system()
    g = oracle.coulomb_J_grad(s.xyz, s.aux, s.orb, d, G)
    assert np.abs(g.sum(0)).max() <= 1e-12 * np.abs(g).max()


def test_gradient_atom_mask():
    s, d, G = _small_system()
    g = oracle.coulomb_J_grad(s.xyz, s.aux, s.orb, d, G)
    m = np.zeros(len(s.xyz), np.uint8)
    m[1] = 1
    gm = oracle.coulomb_J_grad(s.xyz, s.aux, s.orb, d, G, atom_mask=m)
    assert np.allclose(gm[1], g[1], rtol=1e-13, atol=1e-14 * np.abs(g).max())


def test_long_double_build_agrees():
    rng = np.random.default_rng(505)  # own stream: independent of test order
    A, B, C = rng.uniform(-2, 2, (3, 3))
    x = _oracle_block(A, B, C, 3, 2, 5, [0.7, 3.1], [0.4, 12.0], [1.1], pure=1)
    xyz, aux, orb, trip = single_triplet(A, B, C, 3, 2, 5, [0.7, 3.1], [0.4, 12.0], [1.1], pure=1)
    y, _ = oracle.eval_batch(xyz, aux, orb, trip, precision="long")
    assert np.abs(x.ravel() - y).max() <= 1e-12 * np.abs(y).max()


def test_rejects_bad_arguments():
    xyz, aux, orb, trip = single_triplet([0, 0, 0], [1, 0, 0], [0, 1, 0], 0, 0, 0, 1.0, 1.0, 1.0)
    with pytest.raises(ValueError):
        oracle.eval_batch(xyz, aux, orb, np.array([[0, 0, 5]], np.int32))
    aux.nprim[0] = 0
    with pytest.raises(ValueError):
        oracle.eval_batch(xyz, aux, orb, trip)
