#!/usr/bin/env python3
"""Benchmark of the Hubbard HVA state-vector path on one MI355X.

Workload (default): 4x4 periodic Hubbard, t=1, U=8, half filling from the
checkerboard state, 16 Hamiltonian-variational layers x 5 parameters = 80,
32 qubits (complex128 state 64 GiB; psi and lambda 128 GiB in HBM).  One step
= one energy + adjoint-gradient evaluation (E and all 80 dE/dtheta).

Printed (one JSON line): evaluations/s, the roofline of the dominant kernel
(measured live with HIP events on the launch stream), H|psi> GB/s, the
finite-difference plain form on the same GPU, and the oracle's CPU rate.

    python bench.py [--steps K] [--warmup W] [--config c5|c3|c2]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pick_workload(name):
    from paper_2408_00836_amd import workloads as W
    return {"c5": W.config5, "c3": W.config3, "c2": lambda: W.config2(4.0),
            "c1": W.config1}[name]()


def oracle_work_units(w):
    """Full-vector loops the oracle's energy_grad performs, times 2^n (its cost
    model: every term, diagonal or inner product is one loop over all
    amplitudes)."""
    from oracle.model import make_model
    om = make_model(w.nx, w.ny, **w.kwargs())
    per = om.params_per_layer
    nb = len(om.bonds)
    slots = om.bond_slot()
    terms = [2 * sum(1 for s in slots if s == g) for g in range(1, per)]
    fwd = w.layers * (1 + sum(terms))
    ham = 1 + 2 * nb + 1
    rev = w.layers * (3 * (1 + sum(terms)) + per)
    return (fwd + ham + rev) * float(1 << om.nqubits)


def cpu_baseline(target):
    """Oracle energy+adjoint gradient of the 2x6 ladder (24 qubits, 60 params)
    on the host cores, scaled to the target workload by the ratio of oracle
    work units (full-vector loops x 2^n)."""
    import numpy as np
    from oracle import core as oc
    from oracle.model import make_model
    from paper_2408_00836_amd import workloads as W
    sample = W.config3()
    om = make_model(sample.nx, sample.ny, **sample.kwargs())
    cores = oc.threads()
    t0 = time.perf_counter()
    E, g = oc.energy_grad(om, sample.theta, sample.layers)
    dt = time.perf_counter() - t0
    scale = oracle_work_units(sample) / oracle_work_units(target)
    return {"value": scale / dt, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": (f"one oracle energy+adjoint-gradient of the 2x6 ladder "
                       f"(24 qubits, 60 params) took {dt:.2f} s on {cores} threads; "
                       f"scaled by oracle work units (24q/32q = {scale:.3e}) to the "
                       f"benchmark workload"),
            "sample_seconds": dt, "sample_E": E, "finite": bool(np.isfinite(g).all())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c5", choices=["c5", "c3", "c2", "c1"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fd", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the state-vector kernels run on one device; see DESIGN.md for how "
              "it would shard).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2408_00836_amd import abi
    from paper_2408_00836_amd.model import Hubbard

    dev = torch.device("cuda:0")
    w = pick_workload(args.config)
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    th = torch.tensor(w.theta, dtype=torch.float64, device=dev)
    L, P, n = w.layers, w.n_params, w.n_qubits
    dim = 1 << n
    n_fwd = len(abi.hubbard_plan_dump(m.handle, L, 0))
    n_ham = len(abi.hubbard_plan_dump(m.handle, L, 1))
    n_rev = len(abi.hubbard_plan_dump(m.handle, L, 2))
    n_exp = len(abi.hubbard_plan_dump(m.handle, L, 3))
    log(f"[bench] {w.name}: passes fwd={n_fwd} ham={n_ham} rev={n_rev} exp={n_exp}")

    abi.hubbard_set_timing(m.handle, True)
    E = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty(P, dtype=torch.float64, device=dev)
    for i in range(args.warmup):
        m.energy_grad(th, E, g)
        torch.cuda.synchronize()
        log(f"[bench] warmup {i + 1}/{args.warmup} E={E.item():.12f}")

    fwd_ms = ham_ms = rev_ms = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        m.energy_grad(th, E, g)
        f, h_, r = abi.hubbard_phase_ms(m.handle)   # waits for this step's last event
        fwd_ms += f
        ham_ms += h_
        rev_ms += r
        log(f"[bench] step {i + 1}/{args.steps}: fwd {f:.1f} ms, H {h_:.1f} ms, rev {r:.1f} ms")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = (t1 - t0) / args.steps
    evals_per_s = 1.0 / sec
    E_val = E.item()

    # per-launch averages and algorithmic bytes
    fwd_avg = fwd_ms / (args.steps * max(n_fwd, 1))
    rev_avg = rev_ms / (args.steps * max(n_rev, 1))
    fwd_gbs = 32.0 * dim / (fwd_avg * 1e-3) / 1e9
    rev_gbs = 64.0 * dim / (rev_avg * 1e-3) / 1e9
    if rev_ms >= fwd_ms:
        dom = dict(kernel="k_reverse", bytes=64.0 * dim, ms=rev_avg, gbs=rev_gbs)
    else:
        dom = dict(kernel="k_forward", bytes=32.0 * dim, ms=fwd_avg, gbs=fwd_gbs)

    # H|psi>: matrix-free application into the lambda buffer
    psi, lam = m.workspace_views(L)
    hps = []
    for _ in range(3):
        m.apply_h(psi, lam)
        _, hm, _ = abi.hubbard_phase_ms(m.handle)
        hps.append(hm)
    h_ms = min(hps)
    h_gbs = 32.0 * dim / (h_ms * 1e-3) / 1e9
    log(f"[bench] H|psi>: {h_ms:.1f} ms over {n_ham} passes -> {h_gbs:.0f} GB/s algorithmic")

    # finite-difference plain form: 2P+1 energy evaluations per gradient,
    # one instance per launch sequence, same library
    fd = None
    if not args.no_fd:
        ts = []
        for i in range(2):
            torch.cuda.synchronize()
            a = time.perf_counter()
            m.energy(th, E)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - a)
            log(f"[bench] energy-only eval {i + 1}/2: {ts[-1] * 1e3:.1f} ms")
        t_e = min(ts)
        fd_rate = 1.0 / ((2 * P + 1) * t_e)
        fd = {"evals_per_s": fd_rate, "energy_eval_ms": t_e * 1e3, "energy_evals_per_grad": 2 * P + 1,
              "speedup_adjoint_vs_fd": evals_per_s / fd_rate,
              "note": "central FD h=1e-5: 2P+1 energy evaluations per gradient, each timed "
                      "as one energy() call (forward passes + expectation passes)"}

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host (bounded sample)")
        cpu = cpu_baseline(w)

    out = {
        "metric": "energy+adjoint-grad evals/s vs FD plain form; H|psi> HBM GB/s at 32 qubits",
        "value": evals_per_s,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic (seeded theta; lattice model has no data)",
        "config": {"workload": w.name, "lattice": f"{w.nx}x{w.ny}",
                   "periodic": [w.periodic_x, w.periodic_y], "U": w.U, "qubits": n,
                   "layers": L, "params": P, "passes": {"fwd": n_fwd, "ham": n_ham,
                                                        "rev": n_rev, "exp": n_exp}},
        "roofline": {"bound": "hbm", "kernel": dom["kernel"], "achieved": dom["gbs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom["gbs"] / HBM_PEAK_GBS,
                     "traffic": None, "avg_launch_ms": dom["ms"],
                     "bytes_per_launch": dom["bytes"]},
        "kernels": {"k_forward": {"avg_ms": fwd_avg, "GBs": fwd_gbs, "launches_per_step": n_fwd},
                    "k_reverse": {"avg_ms": rev_avg, "GBs": rev_gbs, "launches_per_step": n_rev},
                    "phase_ms_per_step": {"forward": fwd_ms / args.steps,
                                          "hamiltonian": ham_ms / args.steps,
                                          "reverse": rev_ms / args.steps}},
        "hpsi": {"ms": h_ms, "algorithmic_GBs": h_gbs, "frac": h_gbs / HBM_PEAK_GBS,
                 "passes": n_ham},
        "fd_plain": fd,
        "cpu_baseline": cpu,
        "E": E_val,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
