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


def kernel_source_hash():
    """sha256 over the HIP sources, plan and headers the full-vector pass
    kernels come from (every source but the sector form's own file)."""
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2408_00836_amd", "csrc")
    for name in sorted(os.listdir(src)):
        if name.endswith((".hip", ".cpp", ".hpp")) and name != "sector.hip":
            with open(os.path.join(src, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def traffic_bytes(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, calibrated against a
    plain copy), or None when no summary exists or the kernel sources have
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_k_pass_4x4_32q.md")
    try:
        with open(path) as f:
            lines = f.read().splitlines()
    except OSError:
        return None
    kv = {}
    for ln in lines:
        if ln.startswith("- ") and ": " in ln:
            k, v = ln[2:].split(": ", 1)
            kv[k.strip()] = v.strip().strip("`")
    if kv.get("source_sha256") != kernel_source_hash() or kv.get("workload") != workload:
        return None
    val = kv.get(f"traffic_bytes_per_launch {kernel}")
    return float(val) if val else None


def batch_bench(torch, dev, reps=3):
    """The batched path on 256 uneven instances (8-20 qubits, own U, disorder,
    V and 2-10 layers each): one energy+gradient evaluation of all instances
    as an eager launch sequence and as a graph replay, against one
    energy_grad call per instance on the same GPU (the plain form)."""
    import numpy as np
    from paper_2408_00836_amd import workloads as W
    from paper_2408_00836_amd.model import Batch, Hubbard
    ws = W.batch(256)
    models = [Hubbard(w.nx, w.ny, **w.kwargs()) for w in ws]
    b = Batch(models, [w.layers for w in ws])
    tiles_src = sorted({m.tiles_source for m in models})
    theta = torch.tensor(np.concatenate([w.theta for w in ws]), dtype=torch.float64, device=dev)
    ths = [theta[o:o + w.n_params].contiguous() for o, w in zip(b.offsets, ws)]

    def best_of(fn):
        fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return best

    t_eager = best_of(lambda: b.energy_grad(theta))
    b.capture(theta)
    t_graph = best_of(lambda: b.replay(theta))

    def per_instance():
        for m, th in zip(models, ths):
            m.energy_grad(th)
    t_calls = best_of(per_instance)
    n = len(ws)
    return {"workload": "256 uneven instances: chains of 4-10 sites, 2x2..3x3 (8-20 qubits), "
                        "U~U(1,8), t/eps disorder, V=0.5 on odd instances, 2-10 layers",
            "evals_per_s": n / t_graph, "ms_per_batch_graph": t_graph * 1e3,
            "ms_per_batch_eager": t_eager * 1e3, "ms_per_instance_calls": t_calls * 1e3,
            "evals_per_s_instance_calls": n / t_calls, "speedup_vs_instance_calls": t_calls / t_graph,
            "qubits": sorted({w.n_qubits for w in ws}),
            "config": {"work_items": b.config[0], "lanes": b.config[1],
                       "source": b.config_source, "instance_tiles": tiles_src}}


def sector_bench(torch, dev, w, reps=3):
    """The particle-number sector form of the same workload: energy+gradient
    evaluations on the C(Ns,N_dn) x C(Ns,N_up) sector amplitudes (the circuit
    state's only nonzero ones), and H on a sector vector.  Algorithmic bytes
    per evaluation: every row pass reads and writes its vectors once (the
    forward one vector, the reverse two), every transpose reads and writes
    them once, H reads psi and writes phi in both layouts."""
    import numpy as np
    from paper_2408_00836_amd.model import Hubbard
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    nu, nd = m.sector_dims()
    dim = nu * nd
    th = torch.tensor(w.theta, dtype=torch.float64, device=dev)
    E = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty(w.n_params, dtype=torch.float64, device=dev)
    m.sector_energy_grad(th, E, g)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = time.perf_counter()
        m.sector_energy_grad(th, E, g)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - a)
    t = min(ts)
    psi = m.sector_state(th)
    phi = torch.empty_like(psi)
    m.sector_apply_h(psi, phi)
    torch.cuda.synchronize()
    hs = []
    for _ in range(reps):
        a = time.perf_counter()
        m.sector_apply_h(psi, phi)
        torch.cuda.synchronize()
        hs.append(time.perf_counter() - a)
    th_ = min(hs)
    L = w.layers
    passes = L + 1 if L else 0
    vec = 16.0 * dim
    # forward: passes x 2 vec + L transposes x 2 vec; H: 2 row passes (psi
    # read, phi written) + 2 transposes + the transpose-add (3 vec); reverse:
    # passes x 4 vec (the last one reads only: 2) + L transposes of psi and
    # lambda (4 vec each)
    fwd = passes * 2 + L * 2
    ham = 2 * 2 + 2 + 3
    rev = (passes * 4 - 2) + L * 4
    alg = (fwd + ham + rev) * vec
    # the reference ground state of the same model (sector Lanczos from the
    # default start; one H application and a host synchronisation per step)
    torch.cuda.synchronize()
    a = time.perf_counter()
    lz = m.sector_lanczos(max_iter=600, tol=1e-9)
    torch.cuda.synchronize()
    t_lz = time.perf_counter() - a
    return {"workload": w.name + ", sector form", "sector_dims": [nu, nd],
            "amplitudes": dim, "bytes_per_vector": vec,
            "evals_per_s": 1.0 / t, "ms_per_eval": t * 1e3,
            "E": float(E.item()), "row_passes_per_sweep": passes, "transposes_per_sweep": L,
            "algorithmic_bytes_per_eval": alg, "algorithmic_GBs": alg / t / 1e9,
            "frac_of_hbm_peak": alg / t / 1e9 / HBM_PEAK_GBS,
            "hpsi_ms": th_ * 1e3, "hpsi_algorithmic_GBs": 2 * vec / th_ / 1e9,
            "hpsi_bytes_moved_GBs": (2 * 2 + 2 + 3) * vec / th_ / 1e9,
            "lanczos": {"E0": lz["E0"], "E0_per_site": lz["E0"] / (w.nx * w.ny),
                        "iters": lz["iters"], "ritz_residual": lz["residual"], "seconds": t_lz}}


def general_diagonal_leg(torch, dev, reps=5):
    """The 24-qubit disordered ladder with on-site energies and V (the
    general diagonal's kernels): energy+gradient evaluations/s and each
    pass kind's launch-averaged HBM rate (algorithmic bytes as for the
    benchmark workload) as a fraction of the peak."""
    from paper_2408_00836_amd import abi, workloads as W
    from paper_2408_00836_amd.model import Hubbard
    w = W.config3()
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    th = torch.tensor(w.theta, dtype=torch.float64, device=dev)
    E = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty(w.n_params, dtype=torch.float64, device=dev)
    n_fwd = len(abi.hubbard_plan_dump(m.handle, w.layers, 0))
    n_rev = len(abi.hubbard_plan_dump(m.handle, w.layers, 2))
    n_ham = len(abi.hubbard_plan_dump(m.handle, w.layers, 1))
    abi.hubbard_set_timing(m.handle, True)
    m.energy_grad(th, E, g)
    torch.cuda.synchronize()
    kt = {mode: [0.0, 0] for mode in ("forward", "reverse", "hamiltonian")}
    ts = []
    for _ in range(reps):
        a = time.perf_counter()
        m.energy_grad(th, E, g)
        abi.hubbard_phase_ms(m.handle)   # waits for the call's last event
        ts.append(time.perf_counter() - a)
        for mode in kt:
            ms, cnt = abi.hubbard_kernel_ms(m.handle, abi.KERNEL_MODES[mode])
            kt[mode][0] += ms
            kt[mode][1] += cnt
    abi.hubbard_set_timing(m.handle, False)
    vec = 16.0 * (1 << w.n_qubits)
    nvec = {"forward": (2.0 * n_fwd - 1.0) / n_fwd, "reverse": (4.0 * n_rev - 2.0) / n_rev,
            "hamiltonian": (2.0 + 3.0 * (n_ham - 1)) / n_ham}
    kinds = {}
    for mode, (tot, cnt) in kt.items():
        avg = tot / max(cnt, 1)
        gbs = nvec[mode] * vec / (avg * 1e-3) / 1e9
        kinds[mode] = {"kernel": f"hv::k_pass<{abi.KERNEL_MODES[mode]}, true, true, 1, false, 0>",
                       "avg_ms": avg, "launches": cnt // reps, "GBs": gbs,
                       "frac": gbs / HBM_PEAK_GBS}
    t = min(ts)
    # the same evaluation in the particle-number sector form
    m.sector_energy_grad(th, E, g)
    torch.cuda.synchronize()
    ss = []
    for _ in range(reps):
        a = time.perf_counter()
        m.sector_energy_grad(th, E, g)
        torch.cuda.synchronize()
        ss.append(time.perf_counter() - a)
    ts_ = min(ss)
    return {"workload": w.name, "qubits": w.n_qubits, "evals_per_s": 1.0 / t,
            "ms_per_eval": t * 1e3, "E": float(E.item()), "passes": kinds,
            "sector": {"dims": list(m.sector_dims()), "evals_per_s": 1.0 / ts_,
                       "ms_per_eval": ts_ * 1e3}}


def copy_reference(torch, dev, gib=8, reps=3):
    """Bandwidth of a plain device copy (torch elementwise kernel, `gib` GiB
    read + `gib` GiB written): the practical HBM ceiling for an in-place
    read-modify-write stream on this GPU, and the calibration launch for the
    FETCH_SIZE/WRITE_SIZE counters."""
    n = (gib << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        torch.mul(src, 1.0, out=dst)
        b.record(s)
        b.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes": 2.0 * (gib << 30), "ms": best,
            "GBs": 2.0 * (gib << 30) / (best * 1e-3) / 1e9,
            "kernel": "torch mul(src, 1.0, out=dst), float64"}


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


def host_facts():
    """CPU model, hardware threads and RAM of the host (Linux /proc)."""
    model, ram = "unknown", None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for ln in f:
                if ln.startswith("MemTotal"):
                    ram = round(int(ln.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "ram_gib": ram}


def cpu_baseline(target):
    """The oracle (plain C, complex128, all 2^n amplitudes) timed on the host:
    one energy+adjoint gradient of the 2x6 ladder (24 qubits, 12 layers, 60
    params) on all host threads, and the same lattice with one layer on one
    thread.  The benchmark workload (32 qubits) needs 192 GiB and hours of
    the oracle, so its rate is extrapolated from the all-threads sample by
    the ratio of oracle work units (full-vector loops x 2^n) and flagged as
    such."""
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
    one = W.Workload(sample.name + ", 1 layer", sample.nx, sample.ny, False, False, sample.U, 1,
                     sample.params_per_layer, sample.theta[:sample.params_per_layer],
                     sample.t, sample.V, sample.eps)
    oc.set_threads(1)
    try:
        t1 = time.perf_counter()
        oc.energy_grad(om, one.theta, 1)
        dt1 = time.perf_counter() - t1
    finally:
        oc.set_threads(cores)
    u_sample, u_one, u_target = (oracle_work_units(x) for x in (sample, one, target))
    return {"value": u_sample / u_target / dt, "unit": "evals/s", "cores": cores,
            "kind": "oracle", "extrapolated": True,
            "sample": (f"oracle energy+adjoint gradient of the 2x6 ladder (24 qubits, 60 params) "
                       f"measured at {dt:.2f} s on {cores} threads; value scaled to the "
                       f"benchmark workload by oracle work units (x{u_sample / u_target:.3e})"),
            "measured": {
                "c3_all_threads": {"evals_per_s": 1.0 / dt, "seconds": dt, "threads": cores},
                "c3_one_thread": {"evals_per_s": u_one / u_sample / dt1,
                                  "sample_seconds": dt1, "threads": 1,
                                  "sample": "same ladder, 1 layer (5 params), scaled to 12 "
                                            "layers by oracle work units"}},
            "host": host_facts(), "sample_E": E, "finite": bool(np.isfinite(g).all())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c5", choices=["c5", "c3", "c2", "c1"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fd", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-sector", action="store_true")
    ap.add_argument("--no-general", action="store_true",
                    help="skip the 24-qubit general-diagonal leg")
    ap.add_argument("--sector-only", action="store_true",
                    help="time only the sector form (profiling runs)")
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
    if args.sector_only:
        sec = sector_bench(torch, dev, w)
        print(json.dumps({"sector": sec}), flush=True)
        return
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    th = torch.tensor(w.theta, dtype=torch.float64, device=dev)
    L, P, n = w.layers, w.n_params, w.n_qubits
    dim = 1 << n
    n_fwd = len(abi.hubbard_plan_dump(m.handle, L, 0))
    n_ham = len(abi.hubbard_plan_dump(m.handle, L, 1))
    n_rev = len(abi.hubbard_plan_dump(m.handle, L, 2))
    n_exp = len(abi.hubbard_plan_dump(m.handle, L, 3))
    tiles = m.tiles()
    log(f"[bench] {w.name}: tiles {tiles} ({m.tiles_source}); passes fwd={n_fwd} "
        f"ham={n_ham} rev={n_rev} exp={n_exp}")

    abi.hubbard_set_timing(m.handle, True)
    E = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty(P, dtype=torch.float64, device=dev)
    for i in range(args.warmup):
        m.energy_grad(th, E, g)
        torch.cuda.synchronize()
        log(f"[bench] warmup {i + 1}/{args.warmup} E={E.item():.12f}")

    fwd_ms = ham_ms = rev_ms = 0.0
    # per kernel mode: [summed launch ms, launches] over the timed steps
    kt = {mode: [0.0, 0] for mode in abi.KERNEL_MODES}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        m.energy_grad(th, E, g)
        f, h_, r = abi.hubbard_phase_ms(m.handle)   # waits for this step's last event
        fwd_ms += f
        ham_ms += h_
        rev_ms += r
        for mode, code in abi.KERNEL_MODES.items():
            ms, cnt = abi.hubbard_kernel_ms(m.handle, code)
            kt[mode][0] += ms
            kt[mode][1] += cnt
        log(f"[bench] step {i + 1}/{args.steps}: fwd {f:.1f} ms, H {h_:.1f} ms, rev {r:.1f} ms")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = (t1 - t0) / args.steps
    evals_per_s = 1.0 / sec
    E_val = E.item()

    # per-launch averages (events around each launch, on the launch stream)
    # and algorithmic bytes, averaged over the launches of a step: a forward
    # pass reads and writes psi once (the first only writes: it starts from
    # |b0>), a reverse pass psi and lambda (the last only reads them)
    gen = "true" if w.general else "false"   # the diagonal's kernel variant
    vec = 16.0 * dim
    kernels = {}
    # the first H pass reads psi and writes phi, later ones also read phi
    ham_vec = (2.0 + 3.0 * (n_ham - 1)) / max(n_ham, 1)
    fwd_vec = (2.0 * n_fwd - 1.0) / max(n_fwd, 1)
    rev_vec = (4.0 * n_rev - 2.0) / max(n_rev, 1)
    for mode, nvec in (("forward", fwd_vec), ("reverse", rev_vec), ("hamiltonian", ham_vec)):
        tot, cnt = kt[mode]
        if cnt == 0:
            continue
        avg = tot / cnt
        # kernel template: <mode, general diagonal, full tiles, tiles per
        # iteration, from the start state, op kinds> (the first forward pass
        # of a step is the one launch of the <..., true, 0> variant; op kinds
        # 0: hopping terms and diagonal sub-terms, the HVA circuit)
        nt = 2 if (mode == "forward" and not w.general) else 1
        kernels[mode] = {"kernel": f"hv::k_pass<{abi.KERNEL_MODES[mode]}, {gen}, true, {nt}, false, 0>",
                         "avg_ms": avg, "launches_per_step": cnt // args.steps,
                         "bytes_per_launch": nvec * vec,
                         "GBs": nvec * vec / (avg * 1e-3) / 1e9}
    dom = max(kernels.values(), key=lambda k: k["avg_ms"] * k["launches_per_step"])

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

    copy = copy_reference(torch, dev)
    log(f"[bench] plain copy: {copy['GBs']:.0f} GB/s")

    sector = None
    if not args.no_sector:
        log("[bench] sector form")
        sector = sector_bench(torch, dev, w)
        log(f"[bench] sector: {sector['ms_per_eval']:.1f} ms per evaluation")

    general = None
    if not args.no_general:
        log("[bench] general diagonal: 24-qubit ladder with disorder, eps and V")
        general = general_diagonal_leg(torch, dev)
        log(f"[bench] general diagonal: {general['ms_per_eval']:.2f} ms per evaluation")

    batch = None
    if not args.no_batch:
        log("[bench] batch of 256 uneven instances")
        batch = batch_bench(torch, dev)
        log(f"[bench] batch: {batch['ms_per_batch_graph']:.1f} ms per batch (graph), "
            f"{batch['ms_per_instance_calls']:.1f} ms as one call per instance")

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
                                                        "rev": n_rev, "exp": n_exp},
                   "tiles": {"fwd_k": tiles[0], "rev_k": tiles[1], "c": tiles[2],
                             "source": m.tiles_source}},
        "roofline": {"bound": "hbm", "kernel": dom["kernel"], "achieved": dom["GBs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom["GBs"] / HBM_PEAK_GBS,
                     "traffic": traffic_bytes(dom["kernel"], w.name),
                     "avg_launch_ms": dom["avg_ms"], "bytes_per_launch": dom["bytes_per_launch"]},
        "kernels": dict(kernels, phase_ms_per_step={"forward": fwd_ms / args.steps,
                                                    "hamiltonian": ham_ms / args.steps,
                                                    "reverse": rev_ms / args.steps}),
        "copy_reference": copy,
        "batch": batch,
        "sector": sector,
        "general_diagonal": general,
        "hpsi": {"ms": h_ms, "algorithmic_GBs": h_gbs, "frac": h_gbs / HBM_PEAK_GBS,
                 "passes": n_ham},
        "fd_plain": fd,
        "cpu_baseline": cpu,
        "E": E_val,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
