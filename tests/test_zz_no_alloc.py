"""df3c_coulomb_J_noalloc: the DF-J entry point that allocates nothing (its
workspace is the library's own device array).  Called through the C ABI;
every result is compared with df3c_coulomb_J's (the same kernels: bitwise)
and with the oracle at the element bar, on two calls in a row, the second
with a smaller input, and a too-large input is rejected before any device
work."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2210_03192_amd import inputs
from tests.test_gpu_parity import GpuSystem, assert_parity

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _noalloc(df3c, g, d, J, status, stream):
    L = df3c.lib()
    P = ctypes.c_void_p
    L.df3c_coulomb_J_noalloc.argtypes = [P, ctypes.c_int32, P, P, P, P, P, ctypes.c_uint32, P]
    sa, so = g.aux.struct(), g.orb.struct()
    return L.df3c_coulomb_J_noalloc(df3c._ptr(g.xyz), int(g.xyz.shape[0]), ctypes.byref(sa),
                                    ctypes.byref(so), df3c._ptr(d), df3c._ptr(J),
                                    df3c._ptr(status), 0, df3c._stream(stream))


def test_noalloc_J_matches_coulomb_J_twice():
    torch = _torch()
    from paper_2210_03192_amd import df3c
    systems = [inputs.plain_dfj_system(), inputs.plain_dfj_system(seed=inputs.SEED_BASE + 330,
                                                                  natom=3)]
    stream = torch.cuda.Stream()
    status = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    for k, s in enumerate(systems):  # the second input is smaller
        g = GpuSystem(s.xyz, s.aux, s.orb)
        dn = inputs.fitting_coefficients(s.aux.nbf, inputs.SEED_BASE + 331 + k)
        d = torch.as_tensor(dn, device="cuda")
        J = torch.full((s.orb.nbf, s.orb.nbf), np.nan, dtype=torch.float64, device="cuda")
        with torch.cuda.stream(stream):
            rc = _noalloc(df3c, g, d, J, status, stream)
        assert rc == 0, rc
        stream.synchronize()
        assert int(status.item()) == 0
        ref = df3c.coulomb_J(g.xyz, g.aux, g.orb, d)
        torch.cuda.synchronize()
        assert torch.equal(J, ref), k
        assert_parity(J.cpu().numpy(), oracle.coulomb_J(s.xyz, s.aux, s.orb, dn),
                      what=f"no-allocation J, call {k}")


def test_noalloc_J_rejects_inputs_beyond_its_array():
    """Solid-harmonic orbital shells of the 120-atom cluster need the
    Cartesian J (54 MB) in the workspace: beyond the array, rejected before
    any device work."""
    torch = _torch()
    from paper_2210_03192_amd import df3c
    s = inputs.dfj_120_system()
    orb = inputs.Basis(s.orb.l, s.orb.nprim, s.orb.prim_off, s.orb.atom, s.orb.exps,
                       s.orb.coefs, pure=1)
    g = GpuSystem(s.xyz, s.aux, orb)
    d = torch.zeros(s.aux.nbf, dtype=torch.float64, device="cuda")
    J = torch.empty((orb.nbf, orb.nbf), dtype=torch.float64, device="cuda")
    assert _noalloc(df3c, g, d, J, None, None) == -3
