"""GPU parity of the density-fitting solve d = V^{-1} gamma (the library's
FP64 Cholesky, df3c_fit_solve) and of the whole fit (gamma, metric, solve)
against the oracle's chain; at the 60-atom size by the factorisation's and
the solve's backward errors (properties that hold at any size)."""
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


def _spd(n, seed, cond_shift=1.0):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, n))
    return X @ X.T / n + cond_shift * np.eye(n), rng.normal(size=n)


@pytest.mark.parametrize("n", [1, 7, 64, 130, 517])
def test_fit_solve_random_spd(n):
    """Ragged sizes around the 64-wide block columns: the factor equals the
    oracle's Cholesky factor, the solution the oracle's, both at 1e-12."""
    torch = _torch()
    from paper_2210_03192_amd import df3c
    V, g = _spd(n, 400 + n)
    Vd = torch.as_tensor(V, device="cuda").contiguous()
    x = df3c.fit_solve(Vd, torch.as_tensor(g, device="cuda"))
    L = np.tril(Vd.cpu().numpy())
    U = np.triu(Vd.cpu().numpy())
    Lref = np.linalg.cholesky(V)
    assert np.abs(L - Lref).max() <= 1e-12 * np.abs(Lref).max()
    assert np.array_equal(U, L.T)
    d0 = oracle.fit_coefficients(V, g)
    assert np.abs(x.cpu().numpy() - d0).max() <= 1e-12 * np.abs(d0).max()


def test_fit_solve_rejects_non_positive_definite():
    torch = _torch()
    from paper_2210_03192_amd import df3c
    V, g = _spd(70, 9)
    V[40, 40] = -1.0
    with pytest.raises(df3c.DF3CError):
        df3c.fit_solve(torch.as_tensor(V, device="cuda"), torch.as_tensor(g, device="cuda"))
    # positive diagonal, indefinite: the pivot of row 11 is 1 - 2^2 = -3
    W = np.eye(100)
    W[10, 11] = W[11, 10] = 2.0
    with pytest.raises(df3c.DF3CError):
        df3c.fit_solve(torch.as_tensor(W, device="cuda"),
                       torch.as_tensor(np.ones(100), device="cuda"))


def test_density_fit_chain_matches_oracle():
    """Three atoms, orbital s..g, one pure aux shell of every l = 0..6 per atom
    (cond(V) ~ 5e2): gamma, V and d = V^{-1} gamma all from the library equal
    the oracle's chain, d to 1e-10, and so does the fitted energy
    gamma . d / 2."""
    torch = _torch()
    from paper_2210_03192_amd import df3c
    s = _system(inputs.SEED_BASE + 95, range(7), 1)
    xyz = torch.as_tensor(s.xyz, device="cuda")
    aux = df3c.DeviceBasis.from_basis(s.aux)
    orb = df3c.DeviceBasis.from_basis(s.orb)
    D = inputs.symmetric_density(s.orb.nbf, 96)
    Dd = torch.as_tensor(D, device="cuda")
    d = df3c.density_fit(xyz, aux, orb, Dd).cpu().numpy()
    g0 = oracle.coulomb_gamma(s.xyz, s.aux, s.orb, D)
    d0 = oracle.fit_coefficients(oracle.coulomb_metric(s.xyz, s.aux), g0)
    assert np.abs(d - d0).max() <= 1e-10 * np.abs(d0).max()
    E, E0 = 0.5 * g0 @ d, 0.5 * g0 @ d0
    assert abs(E - E0) <= 1e-10 * abs(E0)


def test_fit_60_atom_metric_backward_errors():
    """The metric of the 60-atom water cluster (5180 aux functions; its
    random-exponent basis makes cond(V) ~ 1e15): the factorisation passes the
    pivot test, V = L L^T to n 1e-16 of max|V| and the solve's residual
    |V d - gamma| <= 1e-13 |V| |d| (backward stable), whatever the
    conditioning."""
    torch = _torch()
    from paper_2210_03192_amd import df3c
    s = inputs.grad_60_system()
    xyz = torch.as_tensor(s.xyz, device="cuda")
    aux = df3c.DeviceBasis.from_basis(s.aux)
    orb = df3c.DeviceBasis.from_basis(s.orb)
    V = df3c.coulomb_metric(xyz, aux)
    V0 = V.cpu().numpy()
    g = df3c.coulomb_gamma(xyz, aux, orb,
                           torch.as_tensor(inputs.symmetric_density(s.orb.nbf, 97), device="cuda"))
    g0 = g.cpu().numpy()
    print(f"fit: n = {len(g0)}", flush=True)
    x = df3c.fit_solve(V, g).cpu().numpy()
    L = np.tril(V.cpu().numpy())
    vmax = np.abs(V0).max()
    assert np.abs(L @ L.T - V0).max() <= 1e-16 * len(g0) * vmax
    res = np.abs(V0 @ x - g0).max()
    assert res <= 1e-13 * vmax * np.abs(x).max(), res
