"""DF-J over solid-harmonic orbital shells (NEXT row f4, first half): the
library's J with orb.pure = 1 against the oracle's, which transforms each
Cartesian block on both sides by its definition.

* orbital s..g shells (contracted s and p), pure aux s..i, three atoms;
* a water cluster (the element basis) with the orbital basis taken pure;
* the masked J over pure orbital shells: the kept blocks are the oracle's
  full-J blocks, the others zero; an all-ones mask gives the unmasked pure J
  bitwise.

Bar: the Cartesian J's bar, max(1e-11 |x|, 1e-13) per element, carried
through the linear transform: |x - x_ref| <= (|T_a| B_cart |T_b|^T)[r, c] with
B_cart = max(1e-11 |J_cart|, 1e-13) from the oracle's Cartesian J and
solid-harmonic tables.  A pure element sums up to (l+1)(l+2)/2 Cartesian
elements per side with coefficients up to a few, and the combinations cancel
(x^2 - y^2 and the like), so its error scales with those terms, not with the
(possibly much smaller) result.
"""
import numpy as np
import pytest

import oracle
from tests.gamma_bar import assert_gamma
from paper_2210_03192_amd import inputs
from paper_2210_03192_amd.inputs import Basis, System, _Builder, _logu, random_atoms
from tests.test_gpu_parity import GpuSystem, _torch

pytestmark = pytest.mark.gpu


def _pure(b):
    return Basis(b.l, b.nprim, b.prim_off, b.atom, b.exps, b.coefs, pure=1)


def _system(seed):
    rng = np.random.default_rng(seed)
    xyz = random_atoms(rng, 3, 4.0, 1.5)
    ob, ab = _Builder(1), _Builder(1)
    for a in range(3):
        for l, k in ((0, 3), (1, 2), (2, 1), (3, 1), (4, 1)):
            ob.add(l, a, _logu(rng, 0.2, 20.0, k), rng.uniform(0.2, 1.0, k))
        for l in range(7):
            ab.add(l, a, _logu(rng, 0.1, 10.0, 1), [1.0])
    return System(xyz, ob.build(), ab.build(), "pure-orbitals")


def _cartesian(b):
    return Basis(b.l, b.nprim, b.prim_off, b.atom, b.exps, b.coefs, pure=0)


def _bound(xyz, aux, orb, d, mask=None):
    """|T| max(1e-11 |J_cart|, 1e-13) |T|^T over the block-diagonal
    solid-harmonic transform T."""
    cart = _cartesian(orb)
    Jc = oracle.coulomb_J(xyz, aux, cart, d)
    B = np.maximum(1e-11 * np.abs(Jc), 1e-13)
    op, oc = orb.offsets(), cart.offsets()
    if mask is not None:
        for a in range(orb.nshell):
            for b in range(orb.nshell):
                if not mask[a, b]:
                    B[oc[a]:oc[a + 1], oc[b]:oc[b + 1]] = 1e-13
    T = np.zeros((orb.nbf, cart.nbf))
    for s, l in enumerate(orb.l):
        T[op[s]:op[s + 1], oc[s]:oc[s + 1]] = oracle.solid_transform(int(l))
    return np.abs(T) @ B @ np.abs(T).T


def _assert_pure_parity(J, ref, bound, what):
    err = np.abs(J - ref)
    bad = err > bound
    if bad.any():
        i = np.unravel_index(int(np.argmax(err / bound)), err.shape)
        raise AssertionError(f"{what}: {int(bad.sum())}/{err.size} elements outside the bar; "
                             f"worst {i}: got {J[i]!r}, oracle {ref[i]!r}, |err| {err[i]:.3e}, "
                             f"bar {bound[i]:.3e}")


def _check(s, seed):
    assert s.orb.pure == 1
    d = inputs.fitting_coefficients(s.aux.nbf, seed)
    print(f"pure-orbital J: {s.name} nao={s.orb.nbf} naux={s.aux.nbf}", flush=True)
    J = GpuSystem(s.xyz, s.aux, s.orb).coulomb_J(d)
    assert J.shape == (s.orb.nbf, s.orb.nbf)
    ref = oracle.coulomb_J(s.xyz, s.aux, s.orb, d)
    _assert_pure_parity(J, ref, _bound(s.xyz, s.aux, s.orb, d), "J (pure orbitals)")
    assert np.array_equal(J, J.T)


def test_J_pure_orbital_s_to_g():
    _check(_system(inputs.SEED_BASE + 1201), inputs.SEED_BASE + 1202)


def test_J_pure_orbital_water_cluster():
    s = inputs.water_cluster(4, seed=inputs.SEED_BASE + 1203)
    _check(System(s.xyz, _pure(s.orb), s.aux, "water4-pure"), inputs.SEED_BASE + 1204)


def test_masked_J_pure_orbitals():
    torch = _torch()
    from paper_2210_03192_amd import df3c
    s = inputs.water_cluster(4, seed=inputs.SEED_BASE + 1205)
    orb = _pure(s.orb)
    d = inputs.fitting_coefficients(s.aux.nbf, inputs.SEED_BASE + 1206)
    mask, _ = oracle.screen_pairs(s.xyz, s.orb, 1e-4)
    assert 0 < mask.sum() < mask.size
    ref = oracle.coulomb_J(s.xyz, s.aux, orb, d)
    off = orb.offsets()
    for a in range(orb.nshell):
        for b in range(orb.nshell):
            if not mask[a, b]:
                ref[off[a]:off[a + 1], off[b]:off[b + 1]] = 0.0
    g = GpuSystem(s.xyz, s.aux, orb)
    dd = torch.as_tensor(d, device="cuda")
    m = torch.as_tensor(mask, device="cuda")
    J = df3c.coulomb_J_masked(g.xyz, g.aux, g.orb, dd, m)
    ones = torch.ones_like(m)
    assert torch.equal(df3c.coulomb_J_masked(g.xyz, g.aux, g.orb, dd, ones),
                       df3c.coulomb_J(g.xyz, g.aux, g.orb, dd))
    torch.cuda.synchronize()
    J = J.cpu().numpy()
    assert J.shape == ref.shape
    _assert_pure_parity(J, ref, _bound(s.xyz, s.aux, orb, d, mask),
                        "masked J (pure orbitals)")


def _grad_system(seed):
    rng = np.random.default_rng(seed)
    xyz = random_atoms(rng, 3, 4.0, 1.5)
    ob, ab = _Builder(1), _Builder(1)
    for a in range(3):
        for l, k in ((0, 3), (1, 2), (2, 2), (3, 1)):
            ob.add(l, a, _logu(rng, 0.2, 20.0, k), rng.uniform(0.2, 1.0, k))
        for l in range(6):
            ab.add(l, a, _logu(rng, 0.1, 10.0, 1), [1.0])
    return System(xyz, ob.build(), ab.build(), "pure-orbital-gradient")


def test_gradient_pure_orbitals():
    """The J gradient over pure s..f orbital shells (G non-symmetric) against
    the oracle's, to 1e-10 of max|grad| like the Cartesian gradient; the
    masked gradient under an all-ones mask is the same bitwise."""
    torch = _torch()
    from paper_2210_03192_amd import df3c
    s = _grad_system(inputs.SEED_BASE + 1207)
    d = inputs.fitting_coefficients(s.aux.nbf, inputs.SEED_BASE + 1208)
    G = np.random.default_rng(inputs.SEED_BASE + 1209).normal(size=(s.orb.nbf, s.orb.nbf))
    print(f"pure-orbital gradient: nao={s.orb.nbf} naux={s.aux.nbf}", flush=True)
    ref = oracle.coulomb_J_grad(s.xyz, s.aux, s.orb, d, G)
    g = GpuSystem(s.xyz, s.aux, s.orb)
    dd = torch.as_tensor(d, device="cuda")
    Gd = torch.as_tensor(G, device="cuda")
    got = df3c.coulomb_J_grad(g.xyz, g.aux, g.orb, dd, Gd)
    ones = torch.ones((s.orb.nshell, s.orb.nshell), dtype=torch.uint8, device="cuda")
    gm = df3c.coulomb_J_grad_masked(g.xyz, g.aux, g.orb, dd, Gd, ones)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max(), np.abs(got - ref).max()
    assert np.array_equal(gm.cpu().numpy(), got)


def _assert_gamma(g, s, D, what):
    assert_gamma(g, s.xyz, s.aux, s.orb, D, what)


def test_gamma_and_autograd_pure_orbitals():
    """gamma = (P|ab) D over pure orbital functions (D non-symmetric) against
    the oracle, then the autograd of L = sum G J(xyz, d): dL/dd = gamma(G) and
    dL/dxyz = the pure-orbital gradient, both against the oracle."""
    torch = _torch()
    from paper_2210_03192_amd import df3c
    s = _grad_system(inputs.SEED_BASE + 1210)
    print(f"pure-orbital gamma: nao={s.orb.nbf} naux={s.aux.nbf}", flush=True)
    g = GpuSystem(s.xyz, s.aux, s.orb)
    D = np.random.default_rng(inputs.SEED_BASE + 1211).normal(size=(s.orb.nbf, s.orb.nbf))
    gam = df3c.coulomb_gamma(g.xyz, g.aux, g.orb, torch.as_tensor(D, device="cuda"))
    _assert_gamma(gam.cpu().numpy(), s, D, "gamma (pure orbitals)")

    dn = inputs.fitting_coefficients(s.aux.nbf, inputs.SEED_BASE + 1212)
    Gn = np.random.default_rng(inputs.SEED_BASE + 1213).normal(size=(s.orb.nbf, s.orb.nbf))
    d = torch.as_tensor(dn, device="cuda").requires_grad_(True)
    x = g.xyz.clone().requires_grad_(True)
    L = (torch.as_tensor(Gn, device="cuda") * df3c.J(x, d, g.aux, g.orb)).sum()
    L.backward()
    _assert_gamma(d.grad.cpu().numpy(), s, Gn, "dL/dd (pure orbitals)")
    gref = oracle.coulomb_J_grad(s.xyz, s.aux, s.orb, dn, Gn)
    assert np.abs(x.grad.cpu().numpy() - gref).max() <= 1e-10 * np.abs(gref).max()


@pytest.mark.parametrize("ls", [(0,), (1,), (2, 2)], ids=["one_s", "one_p", "two_d"])
def test_J_pure_orbital_degenerate_bases(ls):
    """The smallest bases: a lone s shell (nao 1), a lone p shell, two d
    shells on one atom (no s or p orbital class at all)."""
    rng = np.random.default_rng(inputs.SEED_BASE + 1214 + len(ls))
    xyz = random_atoms(rng, 2, 3.0, 1.5)
    ob, ab = _Builder(1), _Builder(1)
    for l in ls:
        ob.add(l, 0, _logu(rng, 0.3, 5.0, 2), rng.uniform(0.2, 1.0, 2))
    for a in range(2):
        for l in (0, 1, 2):
            ab.add(l, a, _logu(rng, 0.1, 5.0, 1), [1.0])
    _check(System(xyz, ob.build(), ab.build(), "pure-" + "".join(map(str, ls))),
           inputs.SEED_BASE + 1218)


def test_J_pure_orbital_120_atoms_sampled_pairs():
    """J over pure orbital shells of the 120-atom water cluster (the DF-J
    benchmark workload, nao 2320, in the launch configuration the benchmark
    times): the blocks of 10 close shell pairs (same atom or bonded
    neighbours) of every (l_a, l_b) class, d-d, f-d and f-f included, and 12
    random pairs against the oracle's Cartesian blocks carried through its
    solid-harmonic tables, with the Cartesian bar carried the same way.  At
    least 500 elements of the l >= 2 blocks must be >= 1e-2, where the
    relative part of the bar applies."""
    from tests.helpers import close_shell_pairs
    s = inputs.dfj_120_system()
    orb = _pure(s.orb)
    d = inputs.fitting_coefficients(s.aux.nbf, inputs.SEED_BASE + 13)
    print(f"pure-orbital J: 120 atoms nao={orb.nbf}", flush=True)
    J = GpuSystem(s.xyz, s.aux, orb).coulomb_J(d)
    assert np.array_equal(J, J.T)
    n = orb.nshell
    rng = np.random.default_rng(4)
    rnd = np.stack([rng.integers(0, n, 12), rng.integers(0, n, 12)], 1)
    rnd[0] = [0, 0]
    rnd[1] = [n - 1, 0]
    pairs = np.concatenate([close_shell_pairs(s.orb, s.xyz, 41, per_class=10), rnd])
    blocks = oracle.coulomb_J_pairs(s.xyz, s.aux, s.orb, d, pairs)
    op = orb.offsets()
    n_rel_high_l = 0
    for (a, b), blk in zip(pairs, blocks):
        Ta = oracle.solid_transform(int(orb.l[a]))
        Tb = oracle.solid_transform(int(orb.l[b]))
        ref = Ta @ blk @ Tb.T
        bound = np.abs(Ta) @ np.maximum(1e-11 * np.abs(blk), 1e-13) @ np.abs(Tb).T
        got = J[op[a]:op[a + 1], op[b]:op[b + 1]]
        err = np.abs(got - ref)
        assert (err <= bound).all(), (a, b, float(err.max()), float(bound.min()))
        if min(orb.l[a], orb.l[b]) >= 2:
            n_rel_high_l += int((np.abs(ref) >= 1e-2).sum())
    print(f"pure-orbital J: {len(pairs)} pairs, {n_rel_high_l} l>=2 elements >= 1e-2")
    assert n_rel_high_l >= 500, n_rel_high_l