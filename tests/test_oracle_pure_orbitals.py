"""Pins of the oracle's J over solid-harmonic orbital shells (NEXT row f4:
the bra transform after the HRR, Section 2.5.1).

* l <= 1: the real solid harmonics of s and p shells are the Cartesian
  functions themselves (p in the order y, z, x for m = -1, 0, 1), so J over a
  pure s/p basis is the Cartesian J with the p rows and columns permuted;
* rotation: with s-type fitting functions only, d is unchanged by a rotation
  of the molecule and each solid-harmonic shell turns by an orthogonal
  matrix, so the Frobenius norm of every J block (a, b) is unchanged; the
  Cartesian blocks of d, f, g shells do change (checked, so that the test
  would see a wrong or missing transform);
* J over pure shells is exactly symmetric.
"""
import numpy as np

import oracle
from paper_2210_03192_amd import inputs


def _system(ls, seed, natom=3):
    rng = np.random.default_rng(seed)
    xyz = inputs.random_atoms(rng, natom, 4.0, 1.5)
    ob, ab = inputs._Builder(0), inputs._Builder(1)
    for a in range(natom):
        for l in ls:
            ob.add(l, a, inputs._logu(rng, 0.2, 8.0, 2), rng.uniform(0.2, 1.0, 2))
        for _ in range(3):
            ab.add(0, a, inputs._logu(rng, 0.1, 5.0, 1), [1.0])
    orb = ob.build()
    return xyz, orb, ab.build()


def _pure(b):
    return inputs.Basis(b.l, b.nprim, b.prim_off, b.atom, b.exps, b.coefs, pure=1)


def test_sp_shells_are_permuted_cartesians():
    xyz, orb, aux = _system((0, 1, 1), 1101)
    d = inputs.fitting_coefficients(aux.nbf, 1102)
    Jc = oracle.coulomb_J(xyz, aux, orb, d)
    Jp = oracle.coulomb_J(xyz, aux, _pure(orb), d)
    perm = []
    for s, o in zip(orb.l, orb.offsets()[:-1]):
        perm += [o] if s == 0 else [o + 1, o + 2, o]
    np.testing.assert_array_equal(Jp.shape, Jc.shape)
    np.testing.assert_allclose(Jp, Jc[np.ix_(perm, perm)], rtol=1e-14, atol=1e-15 * abs(Jc).max())


def test_block_norms_invariant_under_rotation():
    xyz, orb, aux = _system((0, 1, 2, 3, 4), 1103, natom=2)
    d = inputs.fitting_coefficients(aux.nbf, 1104)
    R = inputs._random_rotation(np.random.default_rng(1105))
    xr = xyz @ R.T
    po = _pure(orb)
    Jp, Jpr = oracle.coulomb_J(xyz, aux, po, d), oracle.coulomb_J(xr, aux, po, d)
    Jc, Jcr = oracle.coulomb_J(xyz, aux, orb, d), oracle.coulomb_J(xr, aux, orb, d)
    np.testing.assert_allclose(Jp, Jp.T, rtol=0, atol=0)
    op, oc = po.offsets(), orb.offsets()
    n = orb.nshell
    changed = 0
    for a in range(n):
        for b in range(n):
            blk = lambda J, o: J[o[a]:o[a + 1], o[b]:o[b + 1]]
            na, nr = np.linalg.norm(blk(Jp, op)), np.linalg.norm(blk(Jpr, op))
            assert abs(na - nr) <= 1e-11 * max(na, 1e-300) + 1e-14 * abs(Jp).max(), (a, b, na, nr)
            ca, cr = np.linalg.norm(blk(Jc, oc)), np.linalg.norm(blk(Jcr, oc))
            if max(orb.l[a], orb.l[b]) >= 2 and abs(ca - cr) > 1e-6 * ca:
                changed += 1
    assert changed > 0



def test_gradient_is_the_derivative_of_pure_J():
    """With solid-harmonic orbital shells, the gradient of L = sum G_ab J_ab
    (G over the pure functions, non-symmetric) equals central differences
    of the oracle's pure J (h = 1e-4) on d, f and g shells; an s/p basis gives
    the Cartesian gradient of the permuted G."""
    xyz, orb, aux = _system((0, 1, 2, 3, 4), 1108, natom=2)
    po = _pure(orb)
    d = inputs.fitting_coefficients(aux.nbf, 1109)
    G = np.random.default_rng(1110).normal(size=(po.nbf, po.nbf))
    g = oracle.coulomb_J_grad(xyz, aux, po, d, G)
    h = 1e-4
    for at in range(2):
        for ax in range(3):
            xp, xm = xyz.copy(), xyz.copy()
            xp[at, ax] += h
            xm[at, ax] -= h
            fd = ((G * oracle.coulomb_J(xp, aux, po, d)).sum() -
                  (G * oracle.coulomb_J(xm, aux, po, d)).sum()) / (2 * h)
            assert abs(g[at, ax] - fd) <= 1e-6 * max(1.0, abs(fd)), (at, ax, g[at, ax], fd)

    xyz, orb, aux = _system((0, 1, 1), 1111)
    po = _pure(orb)
    d = inputs.fitting_coefficients(aux.nbf, 1112)
    G = np.random.default_rng(1113).normal(size=(po.nbf, po.nbf))
    perm = []
    for s, o in zip(orb.l, orb.offsets()[:-1]):
        perm += [o] if s == 0 else [o + 1, o + 2, o]
    Gc = np.zeros_like(G)
    Gc[np.ix_(perm, perm)] = G
    np.testing.assert_allclose(oracle.coulomb_J_grad(xyz, aux, po, d, G),
                               oracle.coulomb_J_grad(xyz, aux, orb, d, Gc), rtol=1e-12, atol=1e-13)


def test_gamma_is_the_adjoint_of_pure_J():
    """gamma_P = sum_ab (P|ab) D_ab over pure orbital functions satisfies
    sum_P gamma_P(D) d_P = sum_ab D_ab J_ab(d) with the pure J (pinned
    above), for a non-symmetric D and pure aux shells s..d; for s/p shells it
    equals the Cartesian gamma of the permuted D."""
    xyz, orb, aux = _system((0, 1, 2, 3), 1114, natom=2)
    auxp = inputs._Builder(1)
    rng = np.random.default_rng(1115)
    for a in range(2):
        for l in (0, 1, 2):
            auxp.add(l, a, inputs._logu(rng, 0.1, 5.0, 1), [1.0])
    aux = auxp.build()
    po = _pure(orb)
    d = inputs.fitting_coefficients(aux.nbf, 1116)
    D = rng.normal(size=(po.nbf, po.nbf))
    gam = oracle.coulomb_gamma(xyz, aux, po, D)
    J = oracle.coulomb_J(xyz, aux, po, d)
    lhs, rhs = float(gam @ d), float((D * J).sum())
    # both sides sum the same products in different orders: rounding of the sum of |terms|
    assert abs(lhs - rhs) <= 1e-12 * float((np.abs(D) * np.abs(J)).sum()), (lhs, rhs)

    xyz, orb, aux = _system((0, 1, 1), 1117)
    po = _pure(orb)
    D = np.random.default_rng(1118).normal(size=(po.nbf, po.nbf))
    perm = []
    for s, o in zip(orb.l, orb.offsets()[:-1]):
        perm += [o] if s == 0 else [o + 1, o + 2, o]
    Dc = np.zeros_like(D)
    Dc[np.ix_(perm, perm)] = D
    np.testing.assert_allclose(oracle.coulomb_gamma(xyz, aux, po, D),
                               oracle.coulomb_gamma(xyz, aux, orb, Dc), rtol=1e-13, atol=1e-14)
