"""Single-state energy and gradient under HIP graph capture: after a first
call has uploaded the tables, energy and energy_grad only launch kernels, so a captured
graph replayed with new parameters in place must give bitwise the eager
results (reductions run in a fixed order), with eager work and
synchronisation between the replays."""
import sys

import numpy as np
import pytest
import torch

from oracle import core as oc
from oracle.model import make_model
from paper_2408_00836_amd import workloads as W
from paper_2408_00836_amd.model import Hubbard

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


# 16 qubits (plain vector layout), 22 qubits (psi and lambda interleaved in
# 2^20-amplitude blocks)
CASES = [dict(nx=1, ny=8, layers=3, seed=81, U=4.0, V=0.0),
         dict(nx=1, ny=11, layers=2, seed=82, U=3.0, V=0.4)]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_energy_grad_graph_replay(gpu, case):
    c = CASES[case]
    w = W.random_instance(c["nx"], c["ny"], c["layers"], 3, c["seed"], U=c["U"],
                          disorder=0.1, eps_width=0.3, V=c["V"])
    say(f"[capture] case {case}: {w.n_qubits} qubits, {w.layers} layers")
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    th = torch.tensor(w.theta, dtype=torch.float64, device=gpu)
    E_out = torch.empty(1, dtype=torch.float64, device=gpu)
    g_out = torch.empty(th.numel(), dtype=torch.float64, device=gpu)
    E_only = torch.empty(1, dtype=torch.float64, device=gpu)
    m.energy_grad(th, E_out, g_out)            # uploads tables, allocates the workspace
    torch.cuda.synchronize()
    m.energy(th, E_only)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        m.energy_grad(th, E_out, g_out)
    graph_e = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph_e):
        m.energy(th, E_only)
    rng = np.random.default_rng(c["seed"])
    om = make_model(w.nx, w.ny, **w.kwargs())
    for rep in range(3):
        new = w.theta + rng.uniform(-0.1, 0.1, th.numel())
        th.copy_(torch.tensor(new, dtype=torch.float64, device=gpu))
        graph.replay()
        graph_e.replay()
        torch.cuda.synchronize()
        Eg, gg, E1 = E_out.clone(), g_out.clone(), E_only.clone()
        Ee, ge = m.energy_grad(th.clone())     # eager, own outputs
        E1e = m.energy(th.clone())
        torch.cuda.synchronize()
        assert torch.equal(Eg, Ee) and torch.equal(gg, ge), rep
        assert torch.equal(E1, E1e), rep
        assert abs(E1.item() - Eg.item()) <= 1e-12 * max(1.0, abs(Eg.item()))
        if rep == 0:
            E_ref, g_ref = oc.energy_grad(om, new, w.layers)
            assert abs(Eg.item() - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
            assert np.max(np.abs(gg.cpu().numpy() - g_ref)) <= 1e-8
