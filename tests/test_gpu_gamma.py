"""GPU parity of the adjoint digestion gamma_P = sum_ab (P|ab) D_ab and of the
autograd gradient with respect to the fitting coefficients.

Bar: element-wise |x - x_ref| <= max(1e-11 |x_ref|, 1e-13) against the oracle
(long-double oracle for elements outside); the bar carried through the sum
over shell pairs, sum_ab |D_ab| max(1e-11 |(P|ab)|, 1e-13), is reported beside
it (tests/gamma_bar.py).  The register engine, the MFMA classes and the
per-triplet pipeline all contribute to these systems.
"""
import numpy as np
import pytest

import oracle
from tests.gamma_bar import assert_gamma
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


def _assert_gamma(g, s, D, what):
    assert_gamma(g, s.xyz, s.aux, s.orb, D, what)


@pytest.mark.parametrize("which", ["plain3", "s_to_g_pure", "s_to_g_cartesian", "water2"])
def test_gamma_vs_oracle(which):
    torch = _torch()
    if which == "plain3":
        s = inputs.plain_dfj_system(seed=inputs.SEED_BASE + 81, natom=3)
    elif which == "s_to_g_pure":
        s = _system(inputs.SEED_BASE + 82, range(7), 1)
    elif which == "s_to_g_cartesian":
        s = _system(inputs.SEED_BASE + 83, (0, 1, 1), 0)
    else:
        s = inputs.water_cluster(2, seed=inputs.SEED_BASE + 84)
    D = np.random.default_rng(85).normal(size=(s.orb.nbf, s.orb.nbf))  # not symmetric
    df3c, xyz, aux, orb = _gpu(s)
    g = df3c.coulomb_gamma(xyz, aux, orb, torch.as_tensor(D, device="cuda")).cpu().numpy()
    _assert_gamma(g, s, D, which)


def test_gamma_reproducible_and_bilinear_with_J():
    """Bitwise reproducible; sum_P gamma_P(D) d_P equals sum_ab D_ab J_ab(d)
    with the library's own J (60-atom water cluster)."""
    torch = _torch()
    s = inputs.grad_60_system()
    df3c, xyz, aux, orb = _gpu(s)
    D = torch.as_tensor(inputs.symmetric_density(s.orb.nbf, 86), device="cuda")
    d = torch.as_tensor(inputs.fitting_coefficients(s.aux.nbf, 87), device="cuda")
    g1 = df3c.coulomb_gamma(xyz, aux, orb, D)
    g2 = df3c.coulomb_gamma(xyz, aux, orb, D)
    assert torch.equal(g1, g2)
    J = df3c.coulomb_J(xyz, aux, orb, d)
    lhs, rhs = float(g1 @ d), float((D * J).sum())
    assert abs(lhs - rhs) <= 1e-11 * float(g1.abs().sum() * d.abs().max())


def test_autograd_gradient_wrt_d():
    torch = _torch()
    s = inputs.plain_dfj_system(seed=inputs.SEED_BASE + 88, natom=4)
    df3c, xyz, aux, orb = _gpu(s)
    dn = inputs.fitting_coefficients(s.aux.nbf, 89)
    Gn = np.random.default_rng(90).normal(size=(s.orb.nbf, s.orb.nbf))
    d = torch.as_tensor(dn, device="cuda").requires_grad_(True)
    x = xyz.clone().requires_grad_(True)
    L = (torch.as_tensor(Gn, device="cuda") * df3c.J(x, d, aux, orb)).sum()
    L.backward()
    _assert_gamma(d.grad.cpu().numpy(), s, Gn, "dL/dd")
    gref = oracle.coulomb_J_grad(s.xyz, s.aux, s.orb, dn, Gn)
    assert np.abs(x.grad.cpu().numpy() - gref).max() <= 1e-10 * np.abs(gref).max()
