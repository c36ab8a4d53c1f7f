"""The VQE driver on the GPU (hubbard_vqe, Sec. 2.1): one start against the
same optimiser driven by the oracle's evaluations on the host; ten starts in
lockstep (one batched launch per round) with the U = 0 warm start, every
returned point checked with the oracle, and the best energy against the
variational bound and the Lanczos ground energy (error per site)."""
import json
import os
import sys

import numpy as np
import pytest
import torch

from oracle import core as oc
from oracle.model import make_model
from paper_2408_00836_amd import abi, vqe, workloads as W
from paper_2408_00836_amd.model import Hubbard

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                   "sector_ground_energies.json")))


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def host_run(om, L, x0):
    opt = abi.Lbfgs(x0)
    x, st = opt.start, 0
    while st == 0:
        st, x = opt.tell(*oc.energy_grad(om, x, L))
    return opt.result(), x


def test_vqe_single_start_matches_oracle_driven_run(gpu):
    w = W.config1()
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    om = make_model(w.nx, w.ny, **w.kwargs())
    x0 = W.vqe_starts(w.n_params, 1, seed=3)
    th, res = m.vqe(x0, w.layers)
    r = res[0]
    ref, x_ref = host_run(om, w.layers, x0[0])
    say(f"[vqe] GPU {r}, oracle-driven {ref}")
    assert abs(r["E"] - ref["E"]) <= 1e-9
    x = th.cpu().numpy()[0]
    E_chk, g_chk = oc.energy_grad(om, x, w.layers)
    assert abs(E_chk - r["E"]) <= 1e-12 * max(1.0, abs(E_chk))
    assert abs(np.linalg.norm(g_chk) - r["grad_norm"]) <= 1e-9
    assert r["why"] in ("energy tolerance", "gradient tolerance")


def test_vqe_ten_starts_lockstep_config2(gpu):
    w = W.config2(4.0)
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    om = make_model(w.nx, w.ny, **w.kwargs())
    E0 = m.lanczos()["E0"]
    assert abs(E0 - GOLD["config2_chain8_U4"]["E0"]) <= 1e-9
    say("[vqe] config 2, ten starts, U = 0 warm start")
    out = vqe.run(m, w.layers, n_starts=10, seed=0, E_ref=E0)
    res = out["results"]
    say(f"[vqe] best E {out['E']!r} (start {out['best']}), E0 {E0!r}, "
        f"error per site {out['delta_per_site']:.4f}; steps {[r['steps'] for r in res]}")
    assert len(res) == 10 and len(out["warm_results"]) == 10
    assert all(r["why"] in ("energy tolerance", "gradient tolerance") for r in res)
    assert out["E"] >= E0 - 1e-12 and out["delta_per_site"] >= 0.0
    for i in (out["best"], 0, 9):
        E_chk = oc.energy(om, out["thetas"][i], w.layers)
        assert abs(E_chk - res[i]["E"]) <= 1e-12 * max(1.0, abs(E_chk)), i
    # the lockstep run of start 0 and a run of start 0 alone reach the same minimum
    free = m.noninteracting()
    th_w, _ = free.vqe(W.vqe_starts(w.n_params, 10, 0)[:1], w.layers)
    _, res1 = m.vqe(th_w.cpu().numpy(), w.layers)
    assert abs(res1[0]["E"] - res[0]["E"]) <= 1e-6
