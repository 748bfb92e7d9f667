"""Pins of the oracle's shell-pair screening and masked J (NEXT row f2).

* the bound S_ab is recomputed from its definition with numpy (to 1e-12: the
  exponent argument, up to ~1e3 for distant pairs, scales the rounding);
* an all-ones mask gives J exactly; a random symmetric mask keeps exactly the
  blocks of its pairs and zeroes the others;
* screening a water dimer at tau = 1e-12 changes J by far less than the
  neglected pairs' bound would allow to matter (|dJ| <= 1e-8 max|J|).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2210_03192_amd import inputs


def _bound(xyz, orb):
    n = len(orb.l)
    S = np.zeros((n, n))
    for a in range(n):
        for b in range(n):
            A, B = xyz[orb.atom[a]], xyz[orb.atom[b]]
            ab2 = float((A - B) @ (A - B))
            best = 0.0
            for i in range(orb.nprim[a]):
                for j in range(orb.nprim[b]):
                    za, zb = orb.exps[orb.prim_off[a] + i], orb.exps[orb.prim_off[b] + j]
                    ca, cb = orb.coefs[orb.prim_off[a] + i], orb.coefs[orb.prim_off[b] + j]
                    g = za + zb
                    best = max(best, abs(ca * cb) * (math.pi / g) ** 1.5 * math.exp(-za * zb / g * ab2))
            S[a, b] = best
    return S


def test_screen_bound_and_mask():
    s = inputs.water_cluster(3, seed=inputs.SEED_BASE + 401)
    tau = 1e-6
    mask, S = oracle.screen_pairs(s.xyz, s.orb, tau)
    ref = _bound(s.xyz, s.orb)
    # exp of arguments up to ~1e3 carries |argument| x eps relative rounding
    np.testing.assert_allclose(S, ref, rtol=1e-12, atol=0)
    assert np.array_equal(mask, (ref >= tau).astype(np.uint8))
    assert np.array_equal(mask, mask.T)
    assert 0 < mask.sum() < mask.size


def test_masked_J_blocks():
    s = inputs.plain_dfj_system(seed=inputs.SEED_BASE + 402, natom=3)
    d = inputs.fitting_coefficients(s.aux.nbf, 403)
    J = oracle.coulomb_J(s.xyz, s.aux, s.orb, d)
    n = len(s.orb.l)
    np.testing.assert_array_equal(oracle.coulomb_J_masked(s.xyz, s.aux, s.orb, d,
                                                          np.ones((n, n), np.uint8)), J)
    rng = np.random.default_rng(404)
    m = rng.integers(0, 2, (n, n)).astype(np.uint8)
    m = np.maximum(m, m.T)
    Jm = oracle.coulomb_J_masked(s.xyz, s.aux, s.orb, d, m)
    off = s.orb.offsets()
    for a in range(n):
        for b in range(n):
            blk = (slice(off[a], off[a + 1]), slice(off[b], off[b + 1]))
            if m[a, b]:
                np.testing.assert_array_equal(Jm[blk], J[blk])
            else:
                assert not Jm[blk].any()


def test_screening_error_is_small():
    s = inputs.water_cluster(2, seed=inputs.SEED_BASE + 405)
    d = inputs.fitting_coefficients(s.aux.nbf, 406)
    mask, S = oracle.screen_pairs(s.xyz, s.orb, 1e-12)
    J = oracle.coulomb_J(s.xyz, s.aux, s.orb, d)
    Jm = oracle.coulomb_J_masked(s.xyz, s.aux, s.orb, d, mask)
    assert np.abs(Jm - J).max() <= 1e-8 * np.abs(J).max()


def test_masked_gradient_is_the_derivative_of_masked_J():
    """The oracle's gradient over a pair mask is the derivative of
    L = sum G_ab J_ab(masked): central differences of the masked J (h = 1e-4),
    and an all-ones mask gives the full gradient."""
    s = inputs.water_cluster(2, seed=inputs.SEED_BASE + 407)
    d = inputs.fitting_coefficients(s.aux.nbf, 408)
    G = inputs.symmetric_density(s.orb.nbf, 409)
    mask, _ = oracle.screen_pairs(s.xyz, s.orb, 1e-3)
    assert 0 < mask.sum() < mask.size
    n = len(s.orb.l)
    full = oracle.coulomb_J_grad(s.xyz, s.aux, s.orb, d, G)
    # (the oracle's threaded reduction order varies, so equal to rounding)
    np.testing.assert_allclose(
        oracle.coulomb_J_grad(s.xyz, s.aux, s.orb, d, G, pair_mask=np.ones((n, n), np.uint8)), full,
        rtol=1e-12, atol=1e-12 * np.abs(full).max())
    g = oracle.coulomb_J_grad(s.xyz, s.aux, s.orb, d, G, pair_mask=mask)
    h = 1e-4
    for at, ax in ((0, 0), (1, 2), (4, 1)):
        xp, xm = s.xyz.copy(), s.xyz.copy()
        xp[at, ax] += h
        xm[at, ax] -= h
        fd = ((G * oracle.coulomb_J_masked(xp, s.aux, s.orb, d, mask)).sum() -
              (G * oracle.coulomb_J_masked(xm, s.aux, s.orb, d, mask)).sum()) / (2 * h)
        assert abs(g[at, ax] - fd) <= 1e-6 * max(1.0, abs(fd))


# ---------------------------------------------------------------- Schwarz-type
def _random_system(seed, natom=3, kmax=3):
    from paper_2210_03192_amd.inputs import System, _Builder, _logu, random_atoms
    rng = np.random.default_rng(seed)
    xyz = random_atoms(rng, natom, 5.0, 1.2)
    ob, ab = _Builder(0), _Builder(1)
    for a in range(natom):
        for l in range(5):
            k = int(rng.integers(1, kmax + 1))
            ob.add(l, a, _logu(rng, 0.05, 60.0, k), rng.uniform(0.1, 1.0, k))
        for l in range(7):
            ab.add(l, a, _logu(rng, 0.05, 20.0, 1), [1.0])
    return System(xyz, ob.build(), ab.build(), "schwarz")


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_schwarz_bound_holds_for_every_integral(seed):
    """|(ab|P_m)| <= Q_ab Q_P for every triplet of a system with contracted
    s..g orbital shells and pure s..i aux shells (brute force over the
    oracle's McMurchie-Davidson integrals)."""
    s = _random_system(seed)
    Qab, QP = oracle.schwarz_bounds(s.xyz, s.aux, s.orb)
    trip = np.array([(P, a, b) for P in range(s.aux.nshell) for a in range(s.orb.nshell)
                     for b in range(s.orb.nshell)], np.int32)
    out, off = oracle.eval_batch(s.xyz, s.aux, s.orb, trip)
    worst = 0.0
    for (P, a, b), o in zip(trip, off):
        n = s.aux.nfunc(P) * s.orb.nfunc(a) * s.orb.nfunc(b)
        m = np.abs(out[o:o + n]).max()
        worst = max(worst, m / (Qab[a, b] * QP[P]))
    assert worst <= 1.0 + 1e-12, worst


def test_schwarz_bound_exact_for_one_centre_s_functions():
    """For s functions the envelope is the function itself, so at one centre
    Q_ab^2 = (ab|ab): with a = b one s primitive (exponent z, coefficient c)
    and an aux s shell of exponent 2z and coefficient c^2 holding the pair's
    product, (ab|P) = Q_ab^2; and Q_P^2 = (P|P) from the metric."""
    from paper_2210_03192_amd.inputs import Basis
    z, c = 0.7, 1.3
    xyz = np.zeros((1, 3))
    orb = Basis(np.array([0], np.int32), np.array([1], np.int32), np.array([0], np.int64),
                np.array([0], np.int32), np.array([z]), np.array([c]), 0)
    aux = Basis(np.array([0], np.int32), np.array([1], np.int32), np.array([0], np.int64),
                np.array([0], np.int32), np.array([2 * z]), np.array([c * c]), 1)
    Qab, QP = oracle.schwarz_bounds(xyz, aux, orb)
    blk, _ = oracle.eval_batch(xyz, aux, orb, np.array([[0, 0, 0]], np.int32))
    assert abs(blk[0] - Qab[0, 0] ** 2) <= 1e-14 * blk[0]
    V = oracle.coulomb_metric(xyz, aux)
    assert abs(V[0, 0] - QP[0] ** 2) <= 1e-14 * V[0, 0]


def test_schwarz_mask_bounds_the_dropped_J_blocks():
    """Every J block of a pair the Schwarz mask drops is below tau in every
    element (the guarantee of the criterion), on a 4-water cluster."""
    s = inputs.water_cluster(4, seed=inputs.SEED_BASE + 77)
    d = inputs.fitting_coefficients(s.aux.nbf, 78)
    tau = 1e-10
    mask, Sd = oracle.screen_pairs_schwarz(s.xyz, s.aux, s.orb, d, tau)
    assert 0 < mask.mean() < 1 and np.array_equal(mask, mask.T)
    J = oracle.coulomb_J(s.xyz, s.aux, s.orb, d)
    Jm = oracle.coulomb_J_masked(s.xyz, s.aux, s.orb, d, mask)
    assert np.abs(J - Jm).max() <= tau
