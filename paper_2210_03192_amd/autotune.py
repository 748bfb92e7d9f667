"""Autotuner of the persistent batched DF-J schedule.

For every class (L_P, l_a, l_b) present in a workload, the tuner runs that class
alone (all other classes disabled in the tuning table) with each candidate
(chunk, grid_per_cu) pair -- chunk = consecutive shell pairs a team takes per
queue grab, grid_per_cu = persistent workgroups per CU -- times it with HIP
events on the stream it runs on, and keeps the fastest.  Classes are then
ordered longest first so the long classes start early.  The table is stored as
JSON keyed by the GPU architecture and loaded by the benchmark.

Usage: python -m paper_2210_03192_amd.autotune [--nmol 16] [--out FILE]
"""
import argparse
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PATH = os.path.join(HERE, "tune", "gfx950_batched_J.json")
CHUNKS = (1, 2, 4, 8)
GRIDS = (1, 2, 4, 8)


def class_name(c):
    return f"P{c // 25}a{(c // 5) % 5}b{c % 5}"


def load(path=DEFAULT_PATH):
    """ClassTune table from a JSON file, or None if the file does not exist."""
    from . import df3c
    if not os.path.exists(path):
        return None
    data = json.load(open(path))
    t = df3c.default_tune()
    for c in range(df3c.NCLASS):
        e = data["classes"].get(class_name(c))
        if e:
            t[c].chunk, t[c].grid_per_cu, t[c].order = e["chunk"], e["grid_per_cu"], e["order"]
    return t


def tune(batch, reps=3, verbose=True):
    import torch

    from . import df3c
    dev = torch.device("cuda")
    d = torch.as_tensor(np.random.default_rng(0).normal(size=batch.aux.nbf), device=dev)
    xyz = torch.as_tensor(batch.xyz, device=dev)
    aux = df3c.DeviceBasis.from_basis(batch.aux, dev)
    orb = df3c.DeviceBasis.from_basis(batch.orb, dev)
    stream = torch.cuda.Stream()
    ws = torch.empty(df3c.coulomb_J_batched_workspace(aux, orb, batch.nmol), dtype=torch.uint8,
                     device=dev)
    off = batch.orb.offsets()
    nao = off[batch.mol_orb[1:]] - off[batch.mol_orb[:-1]]
    J = torch.empty(int((nao * nao).sum()), dtype=torch.float64, device=dev)
    # classes present: l of the shells of every molecule
    present = set()
    for m in range(batch.nmol):
        lo = set(int(l) for l in batch.orb.l[batch.mol_orb[m]:batch.mol_orb[m + 1]])
        lp = set(int(l) for l in batch.aux.l[batch.mol_aux[m]:batch.mol_aux[m + 1]])
        for P in lp:
            for a in lo:
                for b in lo:
                    if b <= a:
                        present.add(df3c.class_index(P, a, b))
    result = {}
    for c in sorted(present):
        best = None
        for ch in CHUNKS:
            for gr in GRIDS:
                t = df3c.default_tune()
                for k in range(df3c.NCLASS):
                    t[k].enabled = 0
                t[c] = df3c.ClassTune(ch, gr, 1, 0)
                with torch.cuda.stream(stream):
                    df3c.coulomb_J_batched(xyz, aux, orb, batch.mol_orb, batch.mol_aux, d, J=J,
                                           tune=t, flags=df3c.SCHED_PERSISTENT, ws=ws,
                                           stream=stream)
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    for _ in range(reps):
                        df3c.coulomb_J_batched(xyz, aux, orb, batch.mol_orb, batch.mol_aux, d,
                                               J=J, tune=t, flags=df3c.SCHED_PERSISTENT, ws=ws,
                                               stream=stream)
                    e1.record(stream)
                stream.synchronize()
                ms = e0.elapsed_time(e1) / reps
                if best is None or ms < best[0]:
                    best = (ms, ch, gr)
        result[c] = best
        if verbose:
            print(f"{class_name(c)}: chunk {best[1]} grid/CU {best[2]}  {best[0]:.3f} ms",
                  flush=True)
    ranked = sorted(result, key=lambda c: -result[c][0])
    classes = {class_name(c): {"chunk": result[c][1], "grid_per_cu": result[c][2],
                               "order": i, "ms": result[c][0]} for i, c in enumerate(ranked)}
    return {"arch": "gfx950", "workload": f"{batch.nmol} water clusters", "classes": classes}


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--nmol", type=int, default=16)
    p.add_argument("--out", default=DEFAULT_PATH)
    args = p.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    from . import df3c, inputs
    df3c.init()
    batch = inputs.concat_systems(inputs.batched_systems(args.nmol))
    table = tune(batch)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
