"""Benchmark of the (P|ab) hot path on one MI355X.

Workload (one step): the per-class batches -- 1e5 shell triplets for each
class (L_P, l_a, l_b) in {(0,0,0), (2,1,1), (4,2,2), (6,3,3), (6,4,4)} and each
contraction degree K_a = K_b in {1, 3, 6} (K_P = 1), fresh centres per
triplet in a 20 bohr cube, exponents log-uniform in [0.05, 100], raw blocks
written to HBM.  value = contracted output integrals per second over the whole
step, inputs resident in HBM.  Also reported: per-batch integrals/s and the
DF-J wall time of the 8-atom and 120-atom systems.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "3-center integrals/s (FP64) per L class; DF-J and J-gradient ms vs plain"
PEAK_FP64 = 78.6e12       # FLOP/s: 256 CUs x 2.4 GHz x 128 FP64 FLOP/clk/CU
PEAK_HBM = 8.0e12         # B/s
# algorithmic FP64 FLOP per triplet of the per-class batches (operation-count
# model of the HGPA scheme: Boys, VRR1, contraction, CVRR2, transform, HRR)
MODEL_FLOP = {
    ((0, 0, 0), 1): 66, ((0, 0, 0), 3): 562, ((0, 0, 0), 6): 2236,
    ((2, 1, 1), 1): 756, ((2, 1, 1), 3): 3400, ((2, 1, 1), 6): 12300,
    ((4, 2, 2), 1): 8400, ((4, 2, 2), 3): 25000, ((4, 2, 2), 6): 82000,
    ((6, 3, 3), 1): 53000, ((6, 3, 3), 3): 131000, ((6, 3, 3), 6): 393000,
    ((6, 4, 4), 1): 131000, ((6, 4, 4), 3): 298000, ((6, 4, 4), 6): 863000,
}

# HBM bytes per launch of the dominant kernel from the FETCH_SIZE / WRITE_SIZE
# counter passes summarised under profiles/ (each scaled by the counter's
# reading for a copy of known size).  A figure holds only for the kernel
# sources it was measured with: SHA-256 over KERNEL_SOURCES, else traffic = null.
KERNEL_SOURCES = [os.path.join("paper_2210_03192_amd", "csrc", f)
                  for f in ("device.hpp", "tables.hpp", "kernels.hpp", "gen_tables.py",
                            "inst_lp6.hip")]
MEASURED_TRAFFIC = {
    "k_store<6,4,4> K=6": (8.586e9,
                           "9da0434dc324308a2041d1ec7201422ca91dd37135a6634f9af4b6c77c6a1dfb"),
}


def class_model_flop(LP, la, lb, K):
    """Operation-count model of one contracted triplet with K primitive triplets
    (the scheme as implemented: per primitive setup ~40 FLOP, Boys ~20 FLOP per
    m, 4 FMA per VRR1 item, one FMA per CVRR2 prerequisite; per triplet the
    CVRR2 combination, the sparse ket transform and the HRR at one FMA per term).
    Used for the DF-J and gradient legs; the per-class batches use MODEL_FLOP."""
    prim, fixed = _class_model(LP, la, lb)
    return prim * K + fixed


_MODEL_CACHE = {}


def _class_model(LP, la, lb):
    key = (LP, la, lb)
    if key not in _MODEL_CACHE:
        sys.path.insert(0, os.path.join(ROOT, "paper_2210_03192_amd", "csrc"))
        import gen_tables as gt
        g = gt.Geo(LP, la, la + lb)
        L = la + lb
        nnz = sum(1 for r in gt.solid(LP) for x in r if x != 0.0)
        ne = gt.offT(L + 1) - gt.offT(la)
        prim = 40 + 20 * (L + 1) + 8 * len(gt.vtab(L)) + 2 * g.NPI
        fixed = 2 * len(gt.combine(g)[1]) + 2 * nnz * ne + 2 * gt.hrr(la, lb)[0][-1] * (2 * LP + 1)
        _MODEL_CACHE[key] = (prim, fixed)
    return _MODEL_CACHE[key]


def system_model_flop(aux, orb, grad=False):
    """Model FLOP of DF-J over all (P, a >= b) triplets of a system (no
    screening); grad=True sums the four shifted classes of the derivative
    integrals instead."""
    from collections import Counter
    ko = Counter(zip(orb.l.tolist(), orb.nprim.tolist()))
    kp = Counter(zip(aux.l.tolist(), aux.nprim.tolist()))
    total = 0.0
    items = sorted(ko.items())
    for i, ((la, ka), na) in enumerate(items):
        for (lb, kb), nb in items[:i + 1]:
            npair = na * (na + 1) // 2 if (la, ka) == (lb, kb) else na * nb
            hi, lo = (la, lb) if la >= lb else (lb, la)
            for (lp, kc), npp in kp.items():
                K = ka * kb * kc
                if grad:
                    shifted = [(hi + 1, lo), (hi, lo + 1), (hi - 1, lo), (hi, lo - 1)]
                    f = sum(class_model_flop(lp, max(x, y), min(x, y), K)
                            for x, y in shifted if min(x, y) >= 0)
                else:
                    f = class_model_flop(lp, hi, lo, K)
                total += f * npair * npp
    return total


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--ntrip", type=int, default=100000)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-dfj", action="store_true")
    p.add_argument("--batched-nmol", type=int, default=64)
    p.add_argument("--dfj-only", default="",
                   help="profiling runs: only these DF-J legs (comma list of j120, gamma120, "
                        "grad60), no batched leg")
    p.add_argument("--only", default="",
                   help="profiling runs: only these per-class batches (comma list such as "
                        "P6a4b4K6); the printed line then covers that subset (config.subset)")
    p.add_argument("--copy-calibration-mib", type=int, default=0,
                   help="first run a plain device copy of this many MiB three times "
                        "(the reference kernel for hardware byte counters)")
    return p.parse_args()


def cpu_baseline(batches, budget_s=20.0):
    """The oracle on a bounded sample of every batch (same triplets), scaled to
    integrals/s of the whole per-class workload."""
    import oracle
    nthreads = os.cpu_count() or 1
    total_t, total_int = 0.0, 0
    per = budget_s / len(batches)
    desc = []
    for (cls, K), cb in batches.items():
        n = 8
        while True:
            t0 = time.perf_counter()
            oracle.eval_batch(cb.xyz, cb.aux, cb.orb, cb.trip[:n], nthreads=nthreads)
            dt = time.perf_counter() - t0
            if dt > per / 4 or n >= 4096:
                break
            n *= 4
        # time per integral of this batch, weighted by its share of the workload
        total_t += dt / (n * cb.block) * cb.nint
        total_int += cb.nint
        desc.append(f"{cls}K{K}:{n}")
    return {"value": total_int / total_t, "unit": "integrals/s", "cores": nthreads,
            "kind": "oracle",
            "sample": "first n triplets of each of the 15 per-class batches (" + ", ".join(desc) +
                      "), time scaled to 1e5 triplets per batch"}


def _time_ms(torch, fn, reps, stream=None):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps * 1e3


def dfj_legs(args, df3c, inputs, torch, dev):
    """DF-J wall times (device-resident inputs): single molecules, the batched
    uneven water clusters (per-class launches vs the tuned persistent queue in a
    HIP graph), and the J gradient."""
    out = {}
    legs = set(x for x in args.dfj_only.split(",") if x)
    want = lambda leg: not legs or leg in legs  # noqa: E731
    for name, sysf in (("plain_8atoms", inputs.plain_dfj_system),
                       ("water_120atoms", inputs.dfj_120_system)):
        if legs and not (name == "water_120atoms" and (legs & {"j120", "gamma120"})):
            continue
        s = sysf()
        d = torch.as_tensor(inputs.fitting_coefficients(s.aux.nbf, 1), device=dev)
        xyz = torch.as_tensor(s.xyz, device=dev)
        aux = df3c.DeviceBasis.from_basis(s.aux, dev)
        orb = df3c.DeviceBasis.from_basis(s.orb, dev)
        J = torch.empty((s.orb.nbf, s.orb.nbf), dtype=torch.float64, device=dev)
        wsj = torch.empty(df3c.coulomb_J_workspace(aux, orb), dtype=torch.uint8, device=dev)
        if want("j120"):
            out[f"dfj_ms_{name}"] = _time_ms(torch, lambda: df3c.coulomb_J(xyz, aux, orb, d, J=J,
                                                                            ws=wsj), 3)
        if legs:
            if "gamma120" in legs:
                D = torch.as_tensor(inputs.symmetric_density(s.orb.nbf, 2), device=dev)
                out["gamma_ms_water_120atoms"] = _time_ms(
                    torch, lambda: df3c.coulomb_gamma(xyz, aux, orb, D), 2)
            continue
        mf = system_model_flop(s.aux, s.orb)
        out[f"dfj_model_frac_{name}"] = mf / (out[f"dfj_ms_{name}"] * 1e-3) / PEAK_FP64
        if name == "plain_8atoms":
            # asynchronous calls (plan built on the device, no readback) back to
            # back, and the same call captured in a HIP graph and replayed
            out["dfj_ms_plain_8atoms_async"] = _time_ms(
                torch, lambda: df3c.coulomb_J(xyz, aux, orb, d, J=J, ws=wsj, flags=df3c.ASYNC), 50)
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                df3c.coulomb_J(xyz, aux, orb, d, J=J, ws=wsj, flags=df3c.ASYNC, stream=side)
            torch.cuda.current_stream().wait_stream(side)
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                df3c.coulomb_J(xyz, aux, orb, d, J=J, ws=wsj, flags=df3c.ASYNC)
            out["dfj_ms_plain_8atoms_graph"] = _time_ms(torch, graph.replay, 100)
            df3c.check_workspace(wsj, "8-atom DF-J (graph)")
        if name == "water_120atoms":
            # the fitting legs: gamma = (P|ab) D and the metric (P|Q)
            D = torch.as_tensor(inputs.symmetric_density(s.orb.nbf, 2), device=dev)
            gam = torch.empty(s.aux.nbf, dtype=torch.float64, device=dev)
            wsg = torch.empty(df3c.coulomb_gamma_workspace(aux, orb), dtype=torch.uint8,
                              device=dev)
            out["gamma_ms_water_120atoms"] = _time_ms(
                torch, lambda: df3c.coulomb_gamma(xyz, aux, orb, D, gamma=gam, ws=wsg), 2)
            out["gamma_model_frac_water_120atoms"] = mf / (
                out["gamma_ms_water_120atoms"] * 1e-3) / PEAK_FP64
            Vm = torch.empty((s.aux.nbf, s.aux.nbf), dtype=torch.float64, device=dev)
            out["metric_ms_water_120atoms"] = _time_ms(
                torch, lambda: df3c.coulomb_metric(xyz, aux, V=Vm), 3)
            # the fitting solve d = V^-1 gamma (Cholesky of the n = 10360 metric,
            # two triangular solves; the timed call includes restoring V, a
            # 0.86 GB device copy)
            V0 = Vm.clone()
            dfit = torch.empty_like(gam)
            wsf = torch.empty(df3c.lib().df3c_fit_solve_workspace(s.aux.nbf), dtype=torch.uint8,
                              device=dev)

            def fit():
                Vm.copy_(V0)
                df3c.fit_solve(Vm, gam, x=dfit, ws=wsf)
            out["fit_solve_ms_water_120atoms"] = _time_ms(torch, fit, 2)
            out["fit_solve_n_water_120atoms"] = s.aux.nbf
            out["fit_solve_tflops_water_120atoms"] = (s.aux.nbf ** 3 / 3) / (
                out["fit_solve_ms_water_120atoms"] * 1e-3) / 1e12
            # screened DF-J (pairs kept by the primitive overlap bound >= 1e-12):
            # the screening kernel and the masked J together
            tau = 1e-12
            mask = torch.empty((orb.nshell, orb.nshell), dtype=torch.uint8, device=dev)
            Js = torch.empty_like(J)
            wsm = torch.empty(df3c.coulomb_J_masked_workspace(aux, orb), dtype=torch.uint8,
                              device=dev)

            def screened():
                df3c.screen_pairs(xyz, orb, tau, mask=mask)
                df3c.coulomb_J_masked(xyz, aux, orb, d, mask, J=Js, ws=wsm)
            out["dfj_ms_water_120atoms_screened"] = _time_ms(torch, screened, 3)
            out["dfj_screened_tau"] = tau
            out["dfj_screened_pair_fraction"] = float(mask.double().mean())
            df3c.coulomb_J(xyz, aux, orb, d, J=J, ws=wsj)
            out["dfj_screened_max_dev_rel"] = float((Js - J).abs().max() / J.abs().max())
            # Schwarz-type screening (every dropped J element is below tau)
            for tau_s in (1e-10, 1e-12):
                def schwarz():
                    df3c.screen_pairs_schwarz(xyz, aux, orb, d, tau_s, mask=mask)
                    df3c.coulomb_J_masked(xyz, aux, orb, d, mask, J=Js, ws=wsm)
                key = f"dfj_ms_water_120atoms_schwarz_tau{tau_s:g}"
                out[key] = _time_ms(torch, schwarz, 3)
                out[key.replace("dfj_ms", "dfj_pair_fraction")] = float(mask.double().mean())
                out[key.replace("dfj_ms", "dfj_max_dev_abs")] = float((Js - J).abs().max())
            # solid-harmonic orbital shells: the same J plus the two-sided
            # transform of every block (nao 2l+1 per shell)
            sp = inputs.Basis(s.orb.l, s.orb.nprim, s.orb.prim_off, s.orb.atom, s.orb.exps,
                              s.orb.coefs, pure=1)
            orbp = df3c.DeviceBasis.from_basis(sp, dev)
            Jp = torch.empty((sp.nbf, sp.nbf), dtype=torch.float64, device=dev)
            wsp = torch.empty(df3c.coulomb_J_workspace(aux, orbp), dtype=torch.uint8, device=dev)
            out["dfj_ms_water_120atoms_pure_orbitals"] = _time_ms(
                torch, lambda: df3c.coulomb_J(xyz, aux, orbp, d, J=Jp, ws=wsp), 3)
            out["dfj_pure_orbitals_nao"] = sp.nbf
    if legs and "grad60" not in legs:
        return out
    # J gradient, 60 atoms
    s = inputs.grad_60_system()
    d = torch.as_tensor(inputs.fitting_coefficients(s.aux.nbf, 5), device=dev)
    G = torch.as_tensor(inputs.symmetric_density(s.orb.nbf, 6), device=dev)
    xyz = torch.as_tensor(s.xyz, device=dev)
    aux = df3c.DeviceBasis.from_basis(s.aux, dev)
    orb = df3c.DeviceBasis.from_basis(s.orb, dev)
    if legs:
        out["grad_ms_water_60atoms"] = _time_ms(
            torch, lambda: df3c.coulomb_J_grad(xyz, aux, orb, d, G), 1)
        return out
    out["dfj_ms_water_60atoms"] = _time_ms(torch, lambda: df3c.coulomb_J(xyz, aux, orb, d), 2)
    out["grad_ms_water_60atoms"] = _time_ms(
        torch, lambda: df3c.coulomb_J_grad(xyz, aux, orb, d, G), 1)
    out["dfj_model_frac_water_60atoms"] = system_model_flop(s.aux, s.orb) / (
        out["dfj_ms_water_60atoms"] * 1e-3) / PEAK_FP64
    out["grad_model_frac_water_60atoms"] = system_model_flop(s.aux, s.orb, grad=True) / (
        out["grad_ms_water_60atoms"] * 1e-3) / PEAK_FP64
    # screened J gradient (same criterion and threshold as the screened DF-J):
    # the screening kernel and the masked gradient together
    tau = 1e-12
    mask = torch.empty((orb.nshell, orb.nshell), dtype=torch.uint8, device=dev)
    gs = torch.empty((len(s.xyz), 3), dtype=torch.float64, device=dev)
    wsg = torch.empty(df3c.coulomb_J_grad_masked_workspace(aux, orb, len(s.xyz)),
                      dtype=torch.uint8, device=dev)

    def screened_grad():
        df3c.screen_pairs(xyz, orb, tau, mask=mask)
        df3c.coulomb_J_grad_masked(xyz, aux, orb, d, G, mask, grad=gs, ws=wsg)
    out["grad_ms_water_60atoms_screened"] = _time_ms(torch, screened_grad, 2)
    out["grad_screened_pair_fraction"] = float(mask.double().mean())
    g = df3c.coulomb_J_grad(xyz, aux, orb, d, G)
    out["grad_screened_max_dev_rel"] = float((gs - g).abs().max() / g.abs().max())

    def schwarz_grad():
        df3c.screen_pairs_schwarz(xyz, aux, orb, d, 1e-10, mask=mask)
        df3c.coulomb_J_grad_masked(xyz, aux, orb, d, G, mask, grad=gs, ws=wsg)
    out["grad_ms_water_60atoms_schwarz_tau1e-10"] = _time_ms(torch, schwarz_grad, 2)
    out["grad_pair_fraction_water_60atoms_schwarz_tau1e-10"] = float(mask.double().mean())
    out["grad_max_dev_rel_water_60atoms_schwarz_tau1e-10"] = float(
        (gs - g).abs().max() / g.abs().max())
    # J gradient over solid-harmonic orbital shells (G over the pure functions,
    # pulled back to the Cartesian blocks before the same engines)
    sp = inputs.Basis(s.orb.l, s.orb.nprim, s.orb.prim_off, s.orb.atom, s.orb.exps, s.orb.coefs,
                      pure=1)
    orbp = df3c.DeviceBasis.from_basis(sp, dev)
    Gp = torch.as_tensor(inputs.symmetric_density(sp.nbf, 6), device=dev)
    wsp = torch.empty(df3c.coulomb_J_grad_workspace(aux, orbp, len(s.xyz)), dtype=torch.uint8,
                      device=dev)
    gp = torch.empty((len(s.xyz), 3), dtype=torch.float64, device=dev)
    out["grad_ms_water_60atoms_pure_orbitals"] = _time_ms(
        torch, lambda: df3c.coulomb_J_grad(xyz, aux, orbp, d, Gp, grad=gp, ws=wsp), 2)
    # batched uneven clusters
    if args.batched_nmol > 0:
        from paper_2210_03192_amd import autotune
        b = inputs.concat_systems(inputs.batched_systems(args.batched_nmol))
        db = torch.as_tensor(inputs.fitting_coefficients(b.aux.nbf, 7), device=dev)
        xb = torch.as_tensor(b.xyz, device=dev)
        ab = df3c.DeviceBasis.from_basis(b.aux, dev)
        ob = df3c.DeviceBasis.from_basis(b.orb, dev)
        st = torch.cuda.Stream()
        ws = torch.empty(df3c.coulomb_J_batched_workspace(ab, ob, b.nmol), dtype=torch.uint8,
                         device=dev)
        off = b.orb.offsets()
        nao = off[b.mol_orb[1:]] - off[b.mol_orb[:-1]]
        Jb = torch.empty(int((nao * nao).sum()), dtype=torch.float64, device=dev)
        tuned = autotune.load()

        def run(flags, tune=None):
            with torch.cuda.stream(st):
                df3c.coulomb_J_batched(xb, ab, ob, b.mol_orb, b.mol_aux, db, J=Jb, tune=tune,
                                       flags=flags, ws=ws, stream=st)
        out["batched_nmol"] = b.nmol
        out["batched_natoms"] = int(len(b.xyz))
        out["batched_dfj_ms_per_class"] = _time_ms(torch, lambda: run(df3c.SCHED_PER_CLASS), 1)
        out["batched_dfj_ms_persistent_graph"] = _time_ms(
            torch, lambda: run(df3c.SCHED_PERSISTENT | df3c.GRAPH), 1)
        if tuned is not None:
            out["batched_dfj_ms_persistent_graph_tuned"] = _time_ms(
                torch, lambda: run(df3c.SCHED_PERSISTENT | df3c.GRAPH, tuned), 1)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the per-GPU share of a "
              "sharded run is the single-GPU workload", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2210_03192_amd import df3c, inputs
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    df3c.init()

    batches, gpu = {}, {}
    maxout = 0
    only = set(x for x in args.only.split(",") if x)
    for cls in inputs.PER_CLASS_CLASSES:
        for K in inputs.PER_CLASS_K:
            if only and f"P{cls[0]}a{cls[1]}b{cls[2]}K{K}" not in only:
                continue
            cb = inputs.class_batch(*cls, K, args.ntrip)
            batches[(cls, K)] = cb
            gpu[(cls, K)] = dict(
                xyz=torch.as_tensor(cb.xyz, device=dev),
                aux=df3c.DeviceBasis.from_basis(cb.aux, dev),
                orb=df3c.DeviceBasis.from_basis(cb.orb, dev),
                trip=torch.as_tensor(cb.trip, device=dev),
                off=torch.as_tensor(cb.out_off, device=dev))
            maxout = max(maxout, cb.nint)
    out = torch.empty(maxout, dtype=torch.float64, device=dev)
    ws = torch.empty(df3c.eval_batch_workspace(args.ntrip), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    keys = list(gpu)

    def step():
        for key in keys:
            g = gpu[key]
            df3c.eval_batch(g["xyz"], g["aux"], g["orb"], g["trip"], g["off"], out, ws=ws,
                            stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # every eval_batch of a per-class batch launches exactly one class kernel; the
    # library brackets it with HIP events on the launch stream
    df3c.timing_read()
    df3c.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    df3c.timing_enable(False)
    rec_t = [r for r in df3c.timing_read() if r[0] == df3c.KERNEL_STORE]
    if len(rec_t) != len(keys) * args.steps:
        raise RuntimeError(f"expected {len(keys) * args.steps} timed launches, got {len(rec_t)}")
    times = {key: [] for key in keys}
    for i, (_, cls_id, ms) in enumerate(rec_t):
        key = keys[i % len(keys)]
        assert cls_id == df3c.class_index(*key[0])
        times[key].append(ms)
    ms_step = wall / args.steps * 1e3
    nint = sum(cb.nint for cb in batches.values())
    per_class = {}
    dom_key, dom_ms = None, 0.0
    for key, ev in times.items():
        ms = float(np.mean(ev))
        cb = batches[key]
        per_class[f"P{key[0][0]}a{key[0][1]}b{key[0][2]}_K{key[1]}"] = {
            "ms": ms, "integrals_per_s": cb.nint / (ms * 1e-3),
            "model_tflops": MODEL_FLOP[key] * cb.ntrip / (ms * 1e-3) / 1e12}
        if ms > dom_ms:
            dom_key, dom_ms = key, ms
    cbd = batches[dom_key]
    flop = MODEL_FLOP[dom_key] * cbd.ntrip
    ach = flop / (dom_ms * 1e-3)
    kname = f"k_store<{dom_key[0][0]},{dom_key[0][1]},{dom_key[0][2]}> K={dom_key[1]}"
    traffic = None
    if kname in MEASURED_TRAFFIC and MEASURED_TRAFFIC[kname][1] == kernel_sources_sha256():
        traffic = MEASURED_TRAFFIC[kname][0]
    roof = {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
            "frac": ach / PEAK_FP64, "traffic": traffic, "traffic_unit": "B per launch",
            "kernel": kname,
            "kernel_ms": dom_ms, "model_flop_per_triplet": MODEL_FLOP[dom_key],
            "triplets_per_launch": cbd.ntrip,
            "hbm_write_GBps": cbd.nint * 8 / (dom_ms * 1e-3) / 1e9}

    extra = {}
    if not args.no_dfj:
        extra.update(dfj_legs(args, df3c, inputs, torch, dev))
    rec = {"metric": METRIC, "value": nint / (ms_step * 1e-3), "unit": "integrals/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "per-class batches: 1e5 triplets x (L_P,l_a,l_b) in "
                                  "{(0,0,0),(2,1,1),(4,2,2),(6,3,3),(6,4,4)} x K_a=K_b in {1,3,6}",
                      "ntrip_per_batch": args.ntrip, "integrals_per_step": nint,
                      **({"subset": args.only} if args.only else {})},
           "roofline": roof, "per_class": per_class, **extra}
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(batches)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
