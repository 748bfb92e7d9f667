"""DF-J of every orbital angular momentum the library builds (s..g) against the
oracle: the register engine (small classes), the MFMA engine (whole-wave teams,
up to (6,4,4)) and the per-triplet pipeline all contribute to these J
matrices.  Pure aux shells s..i, and a Cartesian aux basis (l <= 1, where the
ket needs no transform) as the second case.

Bar: element-wise |x - x_ref| <= max(1e-11 |x_ref|, 1e-13); elements outside
are adjudicated by the long-double build of the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2210_03192_amd import inputs
from paper_2210_03192_amd.inputs import System, _Builder, _logu, random_atoms
from tests.test_gpu_parity import GpuSystem, assert_parity

pytestmark = pytest.mark.gpu


def _system(seed, aux_ls, aux_pure):
    """Three atoms; orbital s (K=3), p (K=2), d, f, g per atom; one aux shell
    per l in aux_ls per atom (uncontracted)."""
    rng = np.random.default_rng(seed)
    xyz = random_atoms(rng, 3, 4.0, 1.5)
    ob, ab = _Builder(0), _Builder(aux_pure)
    for a in range(3):
        for l, k in ((0, 3), (1, 2), (2, 1), (3, 1), (4, 1)):
            ob.add(l, a, _logu(rng, 0.2, 20.0, k), rng.uniform(0.2, 1.0, k))
        for l in aux_ls:
            ab.add(l, a, _logu(rng, 0.1, 10.0, 1), [1.0])
    return System(xyz, ob.build(), ab.build(), "j-engines")


def _check(s, seed):
    d = inputs.fitting_coefficients(s.aux.nbf, seed)
    J = GpuSystem(s.xyz, s.aux, s.orb).coulomb_J(d)
    assert np.array_equal(J, J.T)
    ref = oracle.coulomb_J(s.xyz, s.aux, s.orb, d)
    try:
        assert_parity(J, ref, what="J")
    except AssertionError:
        ref_ld = oracle.coulomb_J(s.xyz, s.aux, s.orb, d, precision="long")
        assert_parity(J, ref_ld, what="J (long-double oracle)")


def test_J_orbital_s_to_g_pure_aux_s_to_i():
    _check(_system(inputs.SEED_BASE + 61, range(7), 1), inputs.SEED_BASE + 62)


def test_J_orbital_s_to_g_cartesian_aux():
    _check(_system(inputs.SEED_BASE + 63, (0, 1, 1), 0), inputs.SEED_BASE + 64)
