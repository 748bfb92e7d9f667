"""GPU parity of the two-centre metric V_PQ = (P|Q) and of the density-fitting
chain D -> gamma = (P|ab) D -> d = V^-1 gamma -> J(d).

Bar for V: element-wise |x - x_ref| <= max(1e-11 |x_ref|, 1e-13)
against the oracle (long-double oracle for elements outside); V is exactly
symmetric.  The fitted Coulomb energy E = gamma^T V^-1 gamma / 2 of a
well-conditioned fitting basis agrees with the oracle's chain to 1e-10.
"""
import numpy as np
import pytest

import oracle
from paper_2210_03192_amd import inputs
from tests.test_gpu_j_engines import _system

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _gpu(s):
    torch = _torch()
    from paper_2210_03192_amd import df3c
    xyz = torch.as_tensor(s.xyz, dtype=torch.float64, device="cuda")
    return df3c, xyz, df3c.DeviceBasis.from_basis(s.aux), df3c.DeviceBasis.from_basis(s.orb)


@pytest.mark.parametrize("which", ["pure_s_to_i", "cartesian", "water2"])
def test_metric_vs_oracle(which):
    if which == "pure_s_to_i":
        s = _system(inputs.SEED_BASE + 92, range(7), 1)
    elif which == "cartesian":
        s = _system(inputs.SEED_BASE + 93, (0, 1, 1), 0)
    else:
        s = inputs.water_cluster(2, seed=inputs.SEED_BASE + 94)
    df3c, xyz, aux, orb = _gpu(s)
    V = df3c.coulomb_metric(xyz, aux).cpu().numpy()
    assert np.array_equal(V, V.T)
    ref = oracle.coulomb_metric(s.xyz, s.aux)
    atol = 1e-13
    bad = np.abs(V - ref) > np.maximum(1e-11 * np.abs(ref), atol)
    if bad.any():
        ref = oracle.coulomb_metric(s.xyz, s.aux, precision="long")
        bad = np.abs(V - ref) > np.maximum(1e-11 * np.abs(ref), atol)
    assert not bad.any(), (int(bad.sum()), np.abs(V - ref).max())


def test_density_fitting_chain():
    """Three atoms, orbital s..g, one pure aux shell per l = 0..6 per atom:
    cond(V) ~ 5e2, so the fitted energy is determined to ~1e-13 by inputs
    accurate to 1e-15 (a random-exponent water dimer with 518 aux functions
    has cond(V) ~ 1e15 and no stable fit)."""
    torch = _torch()
    s = _system(inputs.SEED_BASE + 95, range(7), 1)
    df3c, xyz, aux, orb = _gpu(s)
    D = inputs.symmetric_density(s.orb.nbf, 96)
    g = df3c.coulomb_gamma(xyz, aux, orb, torch.as_tensor(D, device="cuda")).cpu().numpy()
    V = df3c.coulomb_metric(xyz, aux).cpu().numpy()
    d = np.linalg.solve(V, g)
    J = df3c.coulomb_J(xyz, aux, orb, torch.as_tensor(d, device="cuda")).cpu().numpy()
    g0 = oracle.coulomb_gamma(s.xyz, s.aux, s.orb, D)
    V0 = oracle.coulomb_metric(s.xyz, s.aux)
    d0 = np.linalg.solve(V0, g0)
    E, E0 = 0.5 * g @ d, 0.5 * g0 @ d0
    assert abs(E - E0) <= 1e-10 * abs(E0)
    # the fitted J reproduces the energy: E = sum_ab D_ab J_ab / 2
    assert abs(0.5 * (D * J).sum() - E) <= 1e-9 * abs(E)
