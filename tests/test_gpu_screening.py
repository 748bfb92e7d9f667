"""GPU parity of the screened DF-J (NEXT row f2): J over a shell-pair mask.

* the same mask (computed by the oracle) into both sides: GPU vs oracle masked
  J, bar max(1e-11 |ref|, 1e-13 max|ref|) (long-double oracle for outliers);
* an all-ones mask reproduces the unmasked GPU J bitwise;
* the library's mask equals the oracle's except for pairs whose bound lies
  within 1e-9 (relative) of tau, where the two rounding paths may disagree;
* 120-atom water cluster at tau = 1e-12: the screened J differs from the full
  J by at most 1e-7 max|J| (measured 2.8e-8: the overlap bound leaves out the
  Coulomb factor and the sum over ~5e3 fitting functions), with a fraction of
  the pairs kept.
"""
import numpy as np
import pytest

import oracle
from paper_2210_03192_amd import inputs
from tests.test_gpu_parity import assert_parity

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
    return torch, df3c, xyz, df3c.DeviceBasis.from_basis(s.aux), df3c.DeviceBasis.from_basis(s.orb)


@pytest.mark.parametrize("n_w,tau", [(3, 1e-4), (4, 1e-8)])
def test_masked_J_vs_oracle(n_w, tau):
    s = inputs.water_cluster(n_w, seed=inputs.SEED_BASE + 410 + n_w)
    torch, df3c, xyz, aux, orb = _gpu(s)
    mask, _ = oracle.screen_pairs(s.xyz, s.orb, tau)
    assert 0 < mask.sum() < mask.size
    d = inputs.fitting_coefficients(s.aux.nbf, 415)
    J = df3c.coulomb_J_masked(xyz, aux, orb, torch.as_tensor(d, device="cuda"),
                              torch.as_tensor(mask, device="cuda")).cpu().numpy()
    ref = oracle.coulomb_J_masked(s.xyz, s.aux, s.orb, d, mask)
    assert np.array_equal(J, J.T)
    try:
        assert_parity(J, ref, what="masked J")
    except AssertionError:
        assert_parity(J, oracle.coulomb_J_masked(s.xyz, s.aux, s.orb, d, mask, precision="long"),
                      what="masked J (long-double oracle)")


def test_all_ones_mask_is_plain_J():
    s = inputs.water_cluster(5, seed=inputs.SEED_BASE + 420)
    torch, df3c, xyz, aux, orb = _gpu(s)
    d = torch.as_tensor(inputs.fitting_coefficients(s.aux.nbf, 421), device="cuda")
    ones = torch.ones((orb.nshell, orb.nshell), dtype=torch.uint8, device="cuda")
    assert torch.equal(df3c.coulomb_J_masked(xyz, aux, orb, d, ones), df3c.coulomb_J(xyz, aux, orb, d))


def test_library_mask_matches_oracle():
    s = inputs.water_cluster(6, seed=inputs.SEED_BASE + 430)
    torch, df3c, xyz, aux, orb = _gpu(s)
    for tau in (1e-3, 1e-8, 1e-12):
        m_gpu = df3c.screen_pairs(xyz, orb, tau).cpu().numpy()
        m_ref, S = oracle.screen_pairs(s.xyz, s.orb, tau)
        near = np.abs(S - tau) <= 1e-9 * tau
        assert np.array_equal(m_gpu[~near], m_ref[~near])
        assert np.array_equal(m_gpu, m_gpu.T)


def test_screened_J_error_water120():
    s = inputs.dfj_120_system()
    torch, df3c, xyz, aux, orb = _gpu(s)
    d = torch.as_tensor(inputs.fitting_coefficients(s.aux.nbf, 1), device="cuda")
    mask = df3c.screen_pairs(xyz, orb, 1e-12)
    kept = float(mask.double().mean())
    assert 0.05 < kept < 0.95
    J = df3c.coulomb_J(xyz, aux, orb, d)
    Js = df3c.coulomb_J_masked(xyz, aux, orb, d, mask)
    assert float((Js - J).abs().max()) <= 1e-7 * float(J.abs().max())


def test_masked_gradient_vs_oracle():
    """Gradient of the screened L over the oracle's mask against the oracle's
    masked gradient (the gradient bar: 1e-10 relative in the max norm); an
    all-ones mask gives the unscreened GPU gradient bitwise."""
    s = inputs.water_cluster(3, seed=inputs.SEED_BASE + 440)
    torch, df3c, xyz, aux, orb = _gpu(s)
    mask, _ = oracle.screen_pairs(s.xyz, s.orb, 1e-4)
    assert 0 < mask.sum() < mask.size
    dn = inputs.fitting_coefficients(s.aux.nbf, 441)
    Gn = inputs.symmetric_density(s.orb.nbf, 442)
    d = torch.as_tensor(dn, device="cuda")
    G = torch.as_tensor(Gn, device="cuda")
    g = df3c.coulomb_J_grad_masked(xyz, aux, orb, d, G, torch.as_tensor(mask, device="cuda"))
    ref = oracle.coulomb_J_grad(s.xyz, s.aux, s.orb, dn, Gn, pair_mask=mask)
    assert np.abs(g.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()
    ones = torch.ones((orb.nshell, orb.nshell), dtype=torch.uint8, device="cuda")
    assert torch.equal(df3c.coulomb_J_grad_masked(xyz, aux, orb, d, G, ones),
                       df3c.coulomb_J_grad(xyz, aux, orb, d, G))


# ---------------------------------------------------------------- Schwarz-type
@pytest.mark.parametrize("n_w,tau", [(3, 1e-6), (5, 1e-10)])
def test_schwarz_mask_matches_oracle_and_masked_J(n_w, tau):
    """The library's Schwarz-type mask equals the oracle's except for pairs
    whose bound Q_ab S_d lies within 1e-9 (relative) of tau; J over the
    oracle's mask matches the oracle's masked J at the element bar."""
    s = inputs.water_cluster(n_w, seed=inputs.SEED_BASE + 430 + n_w)
    torch, df3c, xyz, aux, orb = _gpu(s)
    dn = inputs.fitting_coefficients(s.aux.nbf, 431 + n_w)
    d = torch.as_tensor(dn, device="cuda")
    m_gpu = df3c.screen_pairs_schwarz(xyz, aux, orb, d, tau).cpu().numpy()
    m_ref, Sd = oracle.screen_pairs_schwarz(s.xyz, s.aux, s.orb, dn, tau)
    Qab, _ = oracle.schwarz_bounds(s.xyz, s.aux, s.orb)
    near = np.abs(Qab * Sd - tau) <= 1e-9 * tau
    assert np.array_equal(m_gpu, m_gpu.T)
    assert np.array_equal(m_gpu[~near], m_ref[~near])
    assert 0 < m_ref.mean() < 1
    J = df3c.coulomb_J_masked(xyz, aux, orb, d, torch.as_tensor(m_ref, device="cuda"))
    ref = oracle.coulomb_J_masked(s.xyz, s.aux, s.orb, dn, m_ref)
    assert_parity(J.cpu().numpy(), ref, what="Schwarz-masked J")


def test_schwarz_screened_J_error_below_tau_120_atoms():
    """120-atom water cluster: every element of a dropped pair's J block is
    below tau (the guarantee of the criterion), checked on the library's full
    J; the screened J equals the full J elsewhere to rounding."""
    s = inputs.dfj_120_system()
    torch, df3c, xyz, aux, orb = _gpu(s)
    d = torch.as_tensor(inputs.fitting_coefficients(s.aux.nbf, 1), device="cuda")
    J = df3c.coulomb_J(xyz, aux, orb, d)
    for tau in (1e-10, 1e-12):
        mask = df3c.screen_pairs_schwarz(xyz, aux, orb, d, tau)
        Jm = df3c.coulomb_J_masked(xyz, aux, orb, d, mask)
        ao = torch.as_tensor(s.orb.offsets(), device="cuda")
        # AO-level mask
        sh = torch.repeat_interleave(torch.arange(s.orb.nshell, device="cuda"),
                                     (ao[1:] - ao[:-1]).long())
        keep = mask[sh][:, sh].bool()
        dropped = float(J[~keep].abs().max()) if (~keep).any() else 0.0
        kept_dev = float((J - Jm)[keep].abs().max())
        print(f"tau {tau:g}: kept {float(mask.double().mean()):.3f}, max dropped |J| "
              f"{dropped:.3g}, kept deviation {kept_dev:.3g}")
        assert dropped <= tau
        assert kept_dev <= 1e-13 * float(J.abs().max())
        assert float(Jm[~keep].abs().max()) == 0.0
