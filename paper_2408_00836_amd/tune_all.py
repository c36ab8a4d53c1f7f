"""Tune and cache the schedules of the standard workloads on this GPU:
tile sizes of the 8-, 16-, 24- and 32-qubit lattices (the 32-qubit torus
timed on two layers) and the work items and lanes of the 256-instance
batch.  Writes the cache that `Hubbard` and `Batch` read
($HUBVQE_TUNE_CACHE, else tune_cache.json next to this module).

    python -m paper_2408_00836_amd.tune_all [--skip-32q] [--out PATH]
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np
import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--skip-32q", action="store_true")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the 256-instance batch (lattice entries already cached)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    from . import tune, workloads as W
    from .model import Batch, Hubbard
    path = args.out or tune.cache_path()
    dev = torch.device("cuda:0")
    cfgs = [] if args.batch_only else [W.config1(), W.config2(1.0), W.config3()]
    if not args.skip_32q and not args.batch_only:
        cfgs.append(W.config5())
    for w in cfgs:
        m = Hubbard(w.nx, w.ny, tuned=False, **w.kwargs())
        th = torch.tensor(w.theta, dtype=torch.float64, device=dev)
        proxy = 2 if w.n_qubits >= 32 else None
        ent = tune.autotune(m, th, proxy_layers=proxy, reps=2, path=path)
        print(f"[tune] {w.name}: best {ent['best']} over {len(ent['table'])} candidates",
              flush=True)
        del m
        torch.cuda.empty_cache()
    ws = W.batch(256)
    # every lattice kind of the batch (U-only and general diagonal) on its
    # own first instance
    seen = set()
    for w in ([] if args.batch_only else ws):
        key = (w.nx, w.ny, w.general)
        if key in seen or w.n_qubits <= 12:   # up to 12 qubits: one tile, nothing to choose
            continue
        seen.add(key)
        m = Hubbard(w.nx, w.ny, tuned=False, **w.kwargs())
        th = torch.tensor(w.theta, dtype=torch.float64, device=dev)
        ent = tune.autotune(m, th, reps=2, path=path)
        print(f"[tune] batch kind {w.nx}x{w.ny} general={w.general}: best {ent['best']}",
              flush=True)
        del m
    models = [Hubbard(w.nx, w.ny, **w.kwargs(), tuned=False) for w in ws]
    b = Batch(models, [w.layers for w in ws], tuned=False)
    theta = torch.tensor(np.concatenate([w.theta for w in ws]), dtype=torch.float64, device=dev)
    ent = tune.autotune_batch(b, theta, reps=3, path=path)
    print(f"[tune] batch of 256: best (items, lanes, member tiles) = {ent['best']}",
          flush=True)
    print(f"[tune] wrote {os.path.abspath(path)}", flush=True)


if __name__ == "__main__":
    sys.exit(main())
