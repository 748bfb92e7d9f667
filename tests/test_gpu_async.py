"""Asynchronous, capture-safe calls (DF3C_ASYNC): the shell lists are planned
on the device and the calls only enqueue kernels, so DF-J can be captured
into a HIP graph and replayed; device-side argument checks leave their status
in the workspace.  Every result is compared with the oracle or, bitwise, with
the synchronous call."""
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


def test_coulomb_J_captured_in_a_graph_matches_oracle():
    """df3c_coulomb_J with DF3C_ASYNC captured into a HIP graph (torch's
    capture stream), replayed four times with eager work and a changed d in
    between; every replay equals the eager call bitwise and the oracle at the
    element bar."""
    torch = _torch()
    from paper_2210_03192_amd import df3c
    s = inputs.plain_dfj_system()
    g = GpuSystem(s.xyz, s.aux, s.orb)
    nao = s.orb.nbf
    ds = [inputs.fitting_coefficients(s.aux.nbf, inputs.SEED_BASE + 300 + k) for k in range(2)]
    d = torch.as_tensor(ds[0], device="cuda")
    J = torch.empty((nao, nao), dtype=torch.float64, device="cuda")
    ws = torch.empty(df3c.coulomb_J_workspace(g.aux, g.orb), dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):  # warm-up on a side stream (kernel attributes)
        df3c.coulomb_J(g.xyz, g.aux, g.orb, d, J=J, ws=ws, flags=df3c.ASYNC, stream=side)
    side.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        df3c.coulomb_J(g.xyz, g.aux, g.orb, d, J=J, ws=ws, flags=df3c.ASYNC)
    for k in range(4):
        d.copy_(torch.as_tensor(ds[k % 2], device="cuda"))
        J.fill_(np.nan)
        graph.replay()
        torch.cuda.synchronize()
        got = J.cpu().numpy()
        eager = df3c.coulomb_J(g.xyz, g.aux, g.orb, d).cpu().numpy()
        assert np.array_equal(got, eager), k
        ref = oracle.coulomb_J(s.xyz, s.aux, s.orb, ds[k % 2])
        assert_parity(got, ref, what=f"replay {k}")
        assert df3c.workspace_status(ws) == 0


def test_async_calls_equal_synchronous_calls():
    """eval_batch (every class launched over device counts), J, the gradient
    and gamma with DF3C_ASYNC give the synchronous results bitwise; the masked
    J (launches sized for every candidate pair instead of the kept ones, so
    the aux shells of a pair may be split over other lane counts) to
    rounding."""
    torch = _torch()
    from paper_2210_03192_amd import df3c
    s = inputs.water_cluster(3, seed=inputs.SEED_BASE + 310)
    g = GpuSystem(s.xyz, s.aux, s.orb)
    rng = np.random.default_rng(311)
    trip = np.stack([rng.integers(0, s.aux.nshell, 700), rng.integers(0, s.orb.nshell, 700),
                     rng.integers(0, s.orb.nshell, 700)], 1).astype(np.int32)
    sizes = np.array([s.aux.nfunc(P) * s.orb.nfunc(a) * s.orb.nfunc(b) for P, a, b in trip])
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    t = torch.as_tensor(trip, device="cuda")
    o = torch.as_tensor(off, device="cuda")
    out0 = torch.zeros(int(sizes.sum()), dtype=torch.float64, device="cuda")
    out1 = torch.zeros_like(out0)
    df3c.eval_batch(g.xyz, g.aux, g.orb, t, o, out0)
    ws = torch.empty(df3c.eval_batch_workspace(len(trip)), dtype=torch.uint8, device="cuda")
    df3c.eval_batch(g.xyz, g.aux, g.orb, t, o, out1, ws=ws, flags=df3c.ASYNC)
    assert df3c.workspace_status(ws) == 0
    assert torch.equal(out0, out1)
    d = torch.as_tensor(inputs.fitting_coefficients(s.aux.nbf, 312), device="cuda")
    G = torch.as_tensor(inputs.symmetric_density(s.orb.nbf, 313), device="cuda")
    mask = df3c.screen_pairs(g.xyz, g.orb, 1e-8)
    pairs = [(df3c.coulomb_J, (d,)), (df3c.coulomb_J_masked, (d, mask)),
             (df3c.coulomb_J_grad, (d, G)), (df3c.coulomb_gamma, (G,))]
    for fn, args in pairs:
        a = fn(g.xyz, g.aux, g.orb, *args)
        b = fn(g.xyz, g.aux, g.orb, *args, flags=df3c.ASYNC)
        torch.cuda.synchronize()
        if fn is df3c.coulomb_J_masked:
            assert float((a - b).abs().max()) <= 1e-13 * float(a.abs().max()), fn.__name__
        else:
            assert torch.equal(a, b), fn.__name__


def test_device_checks_leave_status_in_workspace():
    """A bad atom index and an l that disagrees with l_host are caught on the
    device: the synchronous call raises, the asynchronous one leaves the
    status in its workspace and its kernels do nothing."""
    torch = _torch()
    from paper_2210_03192_amd import df3c
    s = inputs.plain_dfj_system(seed=inputs.SEED_BASE + 320, natom=3)
    g = GpuSystem(s.xyz, s.aux, s.orb)
    d = torch.as_tensor(inputs.fitting_coefficients(s.aux.nbf, 321), device="cuda")
    # atom index beyond natom (xyz cut to two atoms)
    xyz2 = g.xyz[:2].contiguous()
    with pytest.raises(df3c.DF3CError):
        df3c.coulomb_J(xyz2, g.aux, g.orb, d)
    ws = torch.empty(df3c.coulomb_J_workspace(g.aux, g.orb), dtype=torch.uint8, device="cuda")
    df3c.coulomb_J(xyz2, g.aux, g.orb, d, ws=ws, flags=df3c.ASYNC)
    assert df3c.workspace_status(ws) == -1
    # device l disagrees with l_host (same counts would pass; here a d shell
    # becomes an f shell on the device only)
    bad = df3c.DeviceBasis.from_basis(s.orb)
    l_dev = bad.l.clone()
    k = int(np.nonzero(s.orb.l == 2)[0][0])
    l_dev[k] = 3
    bad.l = l_dev
    with pytest.raises(df3c.DF3CError):
        df3c.coulomb_J(g.xyz, g.aux, bad, d)
    with pytest.raises(df3c.DF3CError):
        df3c.coulomb_J_grad(g.xyz, g.aux, bad, d,
                            torch.zeros((s.orb.nbf, s.orb.nbf), dtype=torch.float64,
                                        device="cuda"))
    # and the library still works after the failed calls
    J = df3c.coulomb_J(g.xyz, g.aux, g.orb, d).cpu().numpy()
    assert_parity(J, oracle.coulomb_J(s.xyz, s.aux, s.orb, d.cpu().numpy()), what="after errors")


def test_concurrent_host_threads_match_serial_calls():
    """Two host threads call DF-J, gamma and the gradient at the same time on
    their own streams (the calls fork their class groups onto the device's
    shared side streams under a lock): every result equals the one-thread
    result bitwise."""
    import threading
    torch = _torch()
    from paper_2210_03192_amd import df3c
    s = inputs.water_cluster(4, seed=inputs.SEED_BASE + 330)
    g = GpuSystem(s.xyz, s.aux, s.orb)
    ds = [torch.as_tensor(inputs.fitting_coefficients(s.aux.nbf, 331 + k), device="cuda")
          for k in range(2)]
    G = torch.as_tensor(inputs.symmetric_density(s.orb.nbf, 333), device="cuda")

    def calls(d, stream=None):
        return (df3c.coulomb_J(g.xyz, g.aux, g.orb, d, stream=stream),
                df3c.coulomb_gamma(g.xyz, g.aux, g.orb, G, stream=stream),
                df3c.coulomb_J_grad(g.xyz, g.aux, g.orb, d, G, stream=stream))
    ref = [calls(d) for d in ds]
    torch.cuda.synchronize()
    out, errs = [None, None], []

    def worker(k):
        try:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                res = [calls(ds[k], stream=st) for _ in range(3)]
            st.synchronize()
            out[k] = res
        except Exception as e:  # surfaced below
            errs.append(e)
    th = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errs, errs
    for k in range(2):
        for res in out[k]:
            for a, b in zip(res, ref[k]):
                assert torch.equal(a, b)
