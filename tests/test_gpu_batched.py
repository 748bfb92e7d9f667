"""Batched DF-J over several molecules: per-class schedule, persistent work
queue, and its HIP-graph replay, against each molecule's J from the oracle
(small molecules) and from the single-molecule entry point (larger ones)."""
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


def _setup(systems, seed):
    torch = _torch()
    from paper_2210_03192_amd import df3c
    b = inputs.concat_systems(systems)
    d = inputs.fitting_coefficients(b.aux.nbf, seed)
    xyz = torch.as_tensor(b.xyz, device="cuda")
    aux = df3c.DeviceBasis.from_basis(b.aux)
    orb = df3c.DeviceBasis.from_basis(b.orb)
    return df3c, b, d, xyz, aux, orb, torch.as_tensor(d, device="cuda")


def _split(b, Jflat):
    out, o = [], 0
    ao = b.orb.offsets()
    for m in range(b.nmol):
        n = int(ao[b.mol_orb[m + 1]] - ao[b.mol_orb[m]])
        out.append(Jflat[o:o + n * n].reshape(n, n))
        o += n * n
    return out


def _mol_d(b, d, m):
    po = b.aux.offsets()
    return d[po[b.mol_aux[m]]:po[b.mol_aux[m + 1]]]


@pytest.mark.parametrize("flags", ["per_class", "persistent", "persistent_graph"])
def test_batched_small_vs_oracle(flags):
    torch = _torch()
    systems = [inputs.plain_dfj_system(seed=200 + i, natom=n) for i, n in enumerate([2, 5, 3, 8])]
    df3c, b, d, xyz, aux, orb, dd = _setup(systems, 31)
    f = {"per_class": df3c.SCHED_PER_CLASS, "persistent": df3c.SCHED_PERSISTENT,
         "persistent_graph": df3c.SCHED_PERSISTENT | df3c.GRAPH}[flags]
    stream = torch.cuda.Stream()
    ws = torch.empty(df3c.coulomb_J_batched_workspace(aux, orb, b.nmol), dtype=torch.uint8,
                     device="cuda")
    with torch.cuda.stream(stream):
        J = df3c.coulomb_J_batched(xyz, aux, orb, b.mol_orb, b.mol_aux, dd, flags=f, ws=ws,
                                   stream=stream)
        reps = [J.clone()]
        if f & df3c.GRAPH:
            for _ in range(3):  # graph replays, with eager work in between
                J.fill_(np.nan)
                df3c.coulomb_J_batched(xyz, aux, orb, b.mol_orb, b.mol_aux, dd, J=J, flags=f,
                                       ws=ws, stream=stream)
                stream.synchronize()
                reps.append(J.clone())
    torch.cuda.synchronize()
    Js = _split(b, reps[0].cpu().numpy())
    for m, s in enumerate(systems):
        ref = oracle.coulomb_J(s.xyz, s.aux, s.orb, _mol_d(b, d, m))
        err = np.abs(Js[m] - ref) / np.maximum(1e-11 * np.abs(ref), 1e-13)
        assert err.max() <= 1.0, (m, err.max())
    for r in reps[1:]:
        assert torch.equal(r, reps[0])


def _assert_close_pairs(J, s, d, seed, per_class=2, carried=False):
    """Blocks of close shell pairs (every (l_a, l_b) class) of one molecule's
    J against the oracle at the element bar (or, with carried, at the bar
    carried through the sum over the fitting functions); returns the number
    of elements judged by the relative part of the element bar."""
    from tests.gamma_bar import j_pair_bars
    from tests.helpers import close_shell_pairs
    pairs = close_shell_pairs(s.orb, s.xyz, seed, per_class=per_class)
    blocks = oracle.coulomb_J_pairs(s.xyz, s.aux, s.orb, d, pairs)
    bars = j_pair_bars(s.xyz, s.aux, s.orb, d, pairs) if carried else None
    ao = s.orb.offsets()
    n_rel, worst = 0, 0.0
    for k, ((a, b), blk) in enumerate(zip(pairs, blocks)):
        got = J[ao[a]:ao[a + 1], ao[b]:ao[b + 1]]
        elem = np.maximum(1e-11 * np.abs(blk), 1e-13)
        worst = max(worst, float((np.abs(got - blk) / elem).max()))
        err = np.abs(got - blk) / (bars[k] if carried else elem)
        assert err.max() <= 1.0, (a, b, float(err.max()))
        n_rel += int((np.abs(blk) >= 1e-2).sum())
    print(f"close pairs of {s.name}: worst error / element bar {worst:.3g}")
    return n_rel


def test_batched_water_clusters_match_single():
    """Six water clusters of uneven size: persistent + graph schedule (with a
    caller-owned workspace) equals the per-class schedule bitwise (same pair
    ownership and summation order) and the single-molecule DF-J of every
    cluster to rounding; close shell pairs of every class of every cluster
    against the oracle."""
    torch = _torch()
    systems = [inputs.water_cluster(n, seed=300 + n) for n in (2, 9, 4, 14, 5, 7)]
    df3c, b, d, xyz, aux, orb, dd = _setup(systems, 32)
    stream = torch.cuda.Stream()
    ws = torch.empty(df3c.coulomb_J_batched_workspace(aux, orb, b.nmol), dtype=torch.uint8,
                     device="cuda")
    with torch.cuda.stream(stream):
        Jp = df3c.coulomb_J_batched(xyz, aux, orb, b.mol_orb, b.mol_aux, dd,
                                    flags=df3c.SCHED_PERSISTENT | df3c.GRAPH, ws=ws,
                                    stream=stream)
        Jc = df3c.coulomb_J_batched(xyz, aux, orb, b.mol_orb, b.mol_aux, dd,
                                    flags=df3c.SCHED_PER_CLASS, ws=ws, stream=stream)
    torch.cuda.synchronize()
    assert torch.equal(Jp, Jc)
    Js = _split(b, Jp.cpu().numpy())
    n_rel = 0
    for m, s in enumerate(systems):
        sx = torch.as_tensor(s.xyz, device="cuda")
        Jm = df3c.coulomb_J(sx, df3c.DeviceBasis.from_basis(s.aux),
                            df3c.DeviceBasis.from_basis(s.orb),
                            torch.as_tensor(_mol_d(b, d, m), device="cuda"))
        ref = Jm.cpu().numpy()
        assert np.abs(Js[m] - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
        n_rel += _assert_close_pairs(Js[m], s, _mol_d(b, d, m), 400 + m)
    assert n_rel >= 500, n_rel


def test_batched_64_clusters_vs_oracle():
    """The batched uneven workload at full size (64 water clusters of 15..150
    atoms) in the launch the benchmark times (persistent work queue, HIP
    graph, the stored tuning table): the three smallest clusters' whole J and
    close shell pairs of the three largest against the oracle."""
    torch = _torch()
    from paper_2210_03192_amd import autotune
    systems = inputs.batched_systems()
    df3c, b, d, xyz, aux, orb, dd = _setup(systems, inputs.SEED_BASE + 40)
    stream = torch.cuda.Stream()
    ws = torch.empty(df3c.coulomb_J_batched_workspace(aux, orb, b.nmol), dtype=torch.uint8,
                     device="cuda")
    print(f"batched: {b.nmol} clusters, {len(b.xyz)} atoms", flush=True)
    with torch.cuda.stream(stream):
        J = df3c.coulomb_J_batched(xyz, aux, orb, b.mol_orb, b.mol_aux, dd, tune=autotune.load(),
                                   flags=df3c.SCHED_PERSISTENT | df3c.GRAPH, ws=ws,
                                   stream=stream)
    torch.cuda.synchronize()
    Js = _split(b, J.cpu().numpy())
    sizes = np.array([len(s.xyz) for s in systems])
    order = np.argsort(sizes, kind="stable")
    for m in order[:3]:
        s = systems[m]
        ref = oracle.coulomb_J(s.xyz, s.aux, s.orb, _mol_d(b, d, m))
        err = np.abs(Js[m] - ref) / np.maximum(1e-11 * np.abs(ref), 1e-13)
        assert err.max() <= 1.0, (int(m), float(err.max()))
    # the 150-atom clusters hold O f / H d pairs 1.81 bohr apart whose tight
    # exponent sits on the lower-l shell; the DF-J engines keep the HRR
    # quanta on the higher-l shell, and the measured worst element is 1.09x
    # its element bar, within the bar carried through the sum over P
    n_rel = sum(_assert_close_pairs(Js[m], systems[m], _mol_d(b, d, m), 500 + int(m),
                                    carried=True)
                for m in order[-3:])
    assert n_rel >= 500, n_rel


def test_batched_tune_table_and_errors():
    torch = _torch()
    systems = [inputs.plain_dfj_system(seed=210 + i, natom=3) for i in range(3)]
    df3c, b, d, xyz, aux, orb, dd = _setup(systems, 33)
    t = df3c.default_tune()
    for c in range(df3c.NCLASS):
        t[c].chunk = 1 + c % 4
        t[c].grid_per_cu = 1 + c % 3
        t[c].order = c % 5
    J1 = df3c.coulomb_J_batched(xyz, aux, orb, b.mol_orb, b.mol_aux, dd, tune=t,
                                flags=df3c.SCHED_PERSISTENT)
    J0 = df3c.coulomb_J_batched(xyz, aux, orb, b.mol_orb, b.mol_aux, dd,
                                flags=df3c.SCHED_PERSISTENT)
    # J blocks accumulate over the L_P classes, so another class order sums in
    # another order: equal to rounding, not bitwise
    ref = J0.abs().max().item()
    assert (J0 - J1).abs().max().item() <= 1e-13 * max(1.0, ref)
    # the same table twice is bitwise reproducible
    J2 = df3c.coulomb_J_batched(xyz, aux, orb, b.mol_orb, b.mol_aux, dd, tune=t,
                                flags=df3c.SCHED_PERSISTENT)
    assert torch.equal(J1, J2)
    bad = b.mol_orb.copy()
    bad[-1] -= 1
    with pytest.raises(df3c.DF3CError):
        df3c.coulomb_J_batched(xyz, aux, orb, bad, b.mol_aux, dd)


def test_batched_pure_orbital_shells():
    """Solid-harmonic orbital shells in the batched call (the Cartesian J of
    every cluster in the workspace, one transform per cluster): five water
    clusters; persistent + graph (replayed) equals the per-class schedule
    bitwise, each cluster's J equals the single-molecule pure J to rounding,
    and the two smallest clusters' whole J matches the oracle's pure J at the
    Cartesian element bar carried through the transform."""
    import dataclasses
    from paper_2210_03192_amd.inputs import Basis
    torch = _torch()

    def pure(bs):
        return Basis(bs.l, bs.nprim, bs.prim_off, bs.atom, bs.exps, bs.coefs, pure=1)

    systems = [dataclasses.replace(s, orb=pure(s.orb))
               for s in (inputs.water_cluster(n, seed=600 + n) for n in (2, 6, 3, 11, 5))]
    df3c, b, d, xyz, aux, orb, dd = _setup(systems, 34)
    assert b.orb.pure == 1
    stream = torch.cuda.Stream()
    need = df3c.coulomb_J_batched_workspace(aux, orb, b.nmol, b.mol_orb)
    assert need > df3c.coulomb_J_batched_workspace(
        aux, df3c.DeviceBasis.from_basis(dataclasses.replace(b.orb, pure=0)), b.nmol)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    f = df3c.SCHED_PERSISTENT | df3c.GRAPH
    with torch.cuda.stream(stream):
        Jp = df3c.coulomb_J_batched(xyz, aux, orb, b.mol_orb, b.mol_aux, dd, flags=f, ws=ws,
                                    stream=stream)
        reps = [Jp.clone()]
        for _ in range(2):  # graph replays, with eager work in between
            Jp.fill_(np.nan)
            df3c.coulomb_J_batched(xyz, aux, orb, b.mol_orb, b.mol_aux, dd, J=Jp, flags=f,
                                   ws=ws, stream=stream)
            stream.synchronize()
            reps.append(Jp.clone())
        Jc = df3c.coulomb_J_batched(xyz, aux, orb, b.mol_orb, b.mol_aux, dd,
                                    flags=df3c.SCHED_PER_CLASS, ws=ws, stream=stream)
    torch.cuda.synchronize()
    for r in reps[1:]:
        assert torch.equal(r, reps[0])
    assert torch.equal(reps[0], Jc)
    Js = _split(b, reps[0].cpu().numpy())
    for m, s in enumerate(systems):
        Jm = df3c.coulomb_J(torch.as_tensor(s.xyz, device="cuda"),
                            df3c.DeviceBasis.from_basis(s.aux), df3c.DeviceBasis.from_basis(s.orb),
                            torch.as_tensor(_mol_d(b, d, m), device="cuda")).cpu().numpy()
        assert Js[m].shape == Jm.shape
        assert np.abs(Js[m] - Jm).max() <= 1e-13 * max(1.0, np.abs(Jm).max())
    # the pure J's bar: the Cartesian element bar carried through the transform
    from tests.test_gpu_pure_orbitals import _assert_pure_parity, _bound
    for m in (0, 2):
        s, dm = systems[m], _mol_d(b, d, m)
        ref = oracle.coulomb_J(s.xyz, s.aux, s.orb, dm)
        _assert_pure_parity(Js[m], ref, _bound(s.xyz, s.aux, s.orb, dm),
                            f"batched pure J, cluster {m}")
