"""GPU parity of the J-gradient (backward) kernel.

Checks (tolerances of the differentiable workload): against the oracle's
explicit three-centre gradient to 1e-10 relative (max norm), against central
finite differences of the library's own J (h = 1e-4 bohr) to 1e-7 relative,
zero net force, bitwise reproducibility, and the torch.autograd.Function.
"""
import numpy as np
import pytest

import oracle
from paper_2210_03192_amd import inputs

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dev(s):
    torch = _torch()
    from paper_2210_03192_amd import df3c
    xyz = torch.as_tensor(s.xyz, dtype=torch.float64, device="cuda")
    return df3c, xyz, df3c.DeviceBasis.from_basis(s.aux), df3c.DeviceBasis.from_basis(s.orb)


def _rel_inf(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("which", ["plain3", "water2"])
def test_grad_vs_oracle(which):
    torch = _torch()
    if which == "plain3":
        s = inputs.plain_dfj_system(seed=99, natom=3)
    else:
        s = inputs.water_cluster(2, seed=inputs.SEED_BASE + 55)
    d = inputs.fitting_coefficients(s.aux.nbf, 3)
    G = inputs.symmetric_density(s.orb.nbf, 4)
    G[0, 1] += 0.37  # a non-symmetric G as well
    ref = oracle.coulomb_J_grad(s.xyz, s.aux, s.orb, d, G)
    df3c, xyz, aux, orb = _dev(s)
    g = df3c.coulomb_J_grad(xyz, aux, orb, torch.as_tensor(d, device="cuda"),
                            torch.as_tensor(G, device="cuda")).cpu().numpy()
    assert _rel_inf(g, ref) <= 1e-10, _rel_inf(g, ref)
    assert np.abs(g.sum(0)).max() <= 1e-10 * np.abs(g).max()


def test_grad_vs_finite_differences_60_atoms():
    """20 waters (60 atoms); central differences of L = sum G J on 8 atoms."""
    torch = _torch()
    s = inputs.grad_60_system()
    d = torch.as_tensor(inputs.fitting_coefficients(s.aux.nbf, 5), device="cuda")
    G = torch.as_tensor(inputs.symmetric_density(s.orb.nbf, 6), device="cuda")
    df3c, xyz, aux, orb = _dev(s)
    g = df3c.coulomb_J_grad(xyz, aux, orb, d, G).cpu().numpy()
    assert np.abs(g.sum(0)).max() <= 1e-10 * np.abs(g).max()
    h = 1e-4
    rng = np.random.default_rng(0)
    atoms = rng.choice(len(s.xyz), 8, replace=False)
    fd = np.zeros((len(atoms), 3))
    for k, X in enumerate(atoms):
        for i in range(3):
            vals = []
            for sgn in (1.0, -1.0):
                x2 = xyz.clone()
                x2[X, i] += sgn * h
                vals.append(float((G * df3c.coulomb_J(x2, aux, orb, d)).sum()))
            fd[k, i] = (vals[0] - vals[1]) / (2 * h)
    err = np.abs(g[atoms] - fd).max() / np.abs(g).max()
    assert err <= 1e-7, err


def test_grad_bitwise_reproducible():
    torch = _torch()
    s = inputs.water_cluster(3, seed=inputs.SEED_BASE + 56)
    d = torch.as_tensor(inputs.fitting_coefficients(s.aux.nbf, 7), device="cuda")
    G = torch.as_tensor(inputs.symmetric_density(s.orb.nbf, 8), device="cuda")
    df3c, xyz, aux, orb = _dev(s)
    g1 = df3c.coulomb_J_grad(xyz, aux, orb, d, G).cpu().numpy()
    g2 = df3c.coulomb_J_grad(xyz, aux, orb, d, G).cpu().numpy()
    assert np.array_equal(g1, g2)


def test_autograd_function():
    torch = _torch()
    s = inputs.plain_dfj_system(seed=101, natom=4)
    dn = inputs.fitting_coefficients(s.aux.nbf, 9)
    Gn = inputs.symmetric_density(s.orb.nbf, 10)
    df3c, xyz, aux, orb = _dev(s)
    x = xyz.clone().requires_grad_(True)
    d = torch.as_tensor(dn, device="cuda")
    Gt = torch.as_tensor(Gn, device="cuda")
    J = df3c.J(x, d, aux, orb)
    L = (Gt * J).sum()
    L.backward()
    ref = oracle.coulomb_J_grad(s.xyz, s.aux, s.orb, dn, Gn)
    assert _rel_inf(x.grad.cpu().numpy(), ref) <= 1e-10
    Jref = oracle.coulomb_J(s.xyz, s.aux, s.orb, dn)
    assert np.abs(J.detach().cpu().numpy() - Jref).max() <= 1e-11 * np.abs(Jref).max() + 1e-13


def test_grad_rejects_bad_atom_index():
    torch = _torch()
    s = inputs.plain_dfj_system(seed=99, natom=3)
    df3c, xyz, aux, orb = _dev(s)
    d = torch.zeros(s.aux.nbf, dtype=torch.float64, device="cuda")
    G = torch.zeros((s.orb.nbf, s.orb.nbf), dtype=torch.float64, device="cuda")
    with pytest.raises(df3c.DF3CError):
        df3c.coulomb_J_grad(xyz[:2].contiguous(), aux, orb, d, G)


def _golden_rows(path):
    atoms, rows = [], []
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            x = line.split()
            atoms.append(int(x[0]))
            rows.append([float(v) for v in x[1:4]])
    return np.array(atoms), np.array(rows)


def test_grad_60_atoms_vs_oracle_rows():
    """The differentiable workload at full size (60-atom water cluster, the
    launch the benchmark times) against the oracle's explicit three-centre
    gradient rows of six atoms (tests/golden/grad60_atoms.txt, written by
    tests/golden/make_grad60_golden.py from the oracle alone): 1e-10 of the
    largest oracle row element."""
    import os
    torch = _torch()
    s = inputs.grad_60_system()
    d = torch.as_tensor(inputs.fitting_coefficients(s.aux.nbf, 5), device="cuda")
    G = torch.as_tensor(inputs.symmetric_density(s.orb.nbf, 6), device="cuda")
    df3c, xyz, aux, orb = _dev(s)
    g = df3c.coulomb_J_grad(xyz, aux, orb, d, G).cpu().numpy()
    atoms, ref = _golden_rows(os.path.join(os.path.dirname(__file__), "golden",
                                           "grad60_atoms.txt"))
    assert len(atoms) >= 4
    err = np.abs(g[atoms] - ref).max() / np.abs(ref).max()
    print(f"60-atom gradient vs oracle rows of atoms {atoms.tolist()}: {err:.3g}")
    assert err <= 1e-10, err


@pytest.mark.parametrize("which", ["s_to_g", "contracted_s_to_g"])
def test_grad_g_orbital_shells_vs_oracle(which):
    """Orbital shells up to g (the raised bra reaches h): the gradient against
    the oracle's explicit three-centre gradient to 1e-10 of its max norm, and
    zero net force."""
    torch = _torch()
    from tests.test_gpu_j_engines import _contracted_system, _system
    if which == "s_to_g":
        s = _system(inputs.SEED_BASE + 57, range(7), 1)
    else:
        s = _contracted_system(inputs.SEED_BASE + 58)
    d = inputs.fitting_coefficients(s.aux.nbf, 59)
    G = inputs.symmetric_density(s.orb.nbf, 60)
    G[1, 4] -= 0.29  # not symmetric
    ref = oracle.coulomb_J_grad(s.xyz, s.aux, s.orb, d, G)
    df3c, xyz, aux, orb = _dev(s)
    g = df3c.coulomb_J_grad(xyz, aux, orb, torch.as_tensor(d, device="cuda"),
                            torch.as_tensor(G, device="cuda")).cpu().numpy()
    err = _rel_inf(g, ref)
    print(f"g-shell gradient ({which}): {err:.3g}")
    assert err <= 1e-10, err
    assert np.abs(g.sum(0)).max() <= 1e-10 * np.abs(g).max()


def test_grad_batched_molecules():
    """Four molecules of uneven size in one call: every molecule's gradient
    rows equal its single-molecule gradient bitwise, the smallest two match the
    oracle to 1e-10, and a shell whose atom lies outside its molecule's range
    is rejected."""
    torch = _torch()
    from paper_2210_03192_amd import df3c
    systems = [inputs.water_cluster(n, seed=inputs.SEED_BASE + 60 + n) for n in (3, 1, 5, 2)]
    b = inputs.concat_systems(systems)
    mol_atom = np.concatenate([[0], np.cumsum([len(s.xyz) for s in systems])]).astype(np.int32)
    d = inputs.fitting_coefficients(b.aux.nbf, 61)
    Gs = [inputs.symmetric_density(s.orb.nbf, 62 + k) for k, s in enumerate(systems)]
    Gflat = np.concatenate([g.ravel() for g in Gs])
    xyz = torch.as_tensor(b.xyz, device="cuda")
    aux = df3c.DeviceBasis.from_basis(b.aux)
    orb = df3c.DeviceBasis.from_basis(b.orb)
    g = df3c.coulomb_J_grad_batched(xyz, aux, orb, b.mol_orb, b.mol_aux, mol_atom,
                                    torch.as_tensor(d, device="cuda"),
                                    torch.as_tensor(Gflat, device="cuda")).cpu().numpy()
    po = b.aux.offsets()
    for m, s in enumerate(systems):
        dm = d[po[b.mol_aux[m]]:po[b.mol_aux[m + 1]]]
        df, sx, sa, so = _dev(s)
        single = df.coulomb_J_grad(sx, sa, so, torch.as_tensor(dm, device="cuda"),
                                   torch.as_tensor(Gs[m], device="cuda")).cpu().numpy()
        rows = g[mol_atom[m]:mol_atom[m + 1]]
        assert np.array_equal(rows, single), m
        if len(s.xyz) <= 6:
            ref = oracle.coulomb_J_grad(s.xyz, s.aux, s.orb, dm, Gs[m])
            assert _rel_inf(rows, ref) <= 1e-10, m
    # molecule ranges that cut a molecule's shells off their atoms
    bad = mol_atom.copy()
    bad[1] -= 1
    with pytest.raises(df3c.DF3CError):
        df3c.coulomb_J_grad_batched(xyz, aux, orb, b.mol_orb, b.mol_aux, bad,
                                    torch.as_tensor(d, device="cuda"),
                                    torch.as_tensor(Gflat, device="cuda"))
