"""The NP ansatz (Eq. (8), Sec. 2.2.1) on the GPU against the oracle:
energies, adjoint gradients and amplitudes (the library applies R_z as the
phase gate, i.e. R_z up to a known global phase), the reduction to the HVA
circuit with tied parameters, a batch mixing both ansaetze, and the
paper's 32-qubit NP workload (4x4 open, U = 2, 12 layers, 1568 parameters)
by symmetry and finite differences."""
import sys

import numpy as np
import pytest
import torch

from oracle import core as oc
from oracle.model import make_model
from paper_2408_00836_amd import abi, workloads as W
from paper_2408_00836_amd.model import Batch, Hubbard

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


CASES = {
    "2x2_U4": (2, 2, dict(U=4.0), 2),
    "1x8_U8": (1, 8, dict(U=8.0), 3),
    "2x3_general": (2, 3, dict(U=4.0, t=1.0 + 0.1 * np.arange(7), V=np.full(7, 0.5),
                               eps=np.linspace(-0.4, 0.4, 6)), 2),
    "1x6_periodic": (1, 6, dict(periodic_y=True, U=2.0), 2),
}


@pytest.mark.parametrize("key", sorted(CASES))
def test_np_energy_grad_and_state_vs_oracle(gpu, key):
    nx, ny, kw, L = CASES[key]
    m = Hubbard(nx, ny, ansatz="np", **kw)
    om = make_model(nx, ny, **kw)
    P = oc.np_n_params(om, L)
    assert m.n_params(L) == P
    th = np.random.default_rng(40).uniform(-0.4, 0.4, P)
    tdev = torch.tensor(th, dtype=torch.float64, device="cuda")
    say(f"[np] {key}: {P} parameters")
    E, g = m.energy_grad(tdev)
    E_ref, g_ref = oc.np_energy_grad(om, th, L)
    assert abs(E.item() - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
    assert np.max(np.abs(g.cpu().numpy() - g_ref)) <= 1e-8
    assert abs(m.energy(tdev).item() - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
    # amplitudes: the oracle's exact R_z adds the global phase prod exp(-i th_q / 2)
    psi = m.ansatz(tdev).cpu().numpy()
    phase = np.exp(-0.5j * np.sum(th[:om.nqubits]))
    assert np.max(np.abs(psi * phase - oc.np_ansatz(om, th, L))) <= 1e-10


def test_np_tied_parameters_equal_hva(gpu):
    w = W.config1()
    hva = Hubbard(w.nx, w.ny, **w.kwargs())
    npm = Hubbard(w.nx, w.ny, ansatz="np", **w.kwargs())
    om = make_model(w.nx, w.ny, **w.kwargs())
    per = om.params_per_layer
    slots = om.bond_slot()
    th = np.zeros(npm.n_params(w.layers))
    k = om.nqubits
    for l in range(w.layers):
        for i in range(om.nsites):
            th[k + 1] = -w.theta[l * per] * om.U
            k += 2
        for g in range(1, om.ngroups + 1):
            for b, s in enumerate(slots):
                if s == g:
                    for _ in (0, 1):
                        th[k] = w.theta[l * per + g] * om.t[b]
                        k += 2
    E_np = npm.energy(torch.tensor(th, dtype=torch.float64, device="cuda")).item()
    E_hva = hva.energy(torch.tensor(w.theta, dtype=torch.float64, device="cuda")).item()
    assert abs(E_np - E_hva) <= 1e-12 * max(1.0, abs(E_hva))


def test_batch_mixing_np_and_hva(gpu):
    specs = [(2, 2, dict(U=4.0), 2, "np"), (1, 6, dict(U=2.0), 3, "hva"),
             (2, 3, dict(U=3.0, V=np.full(7, 0.3)), 2, "np"), (1, 8, dict(U=8.0), 2, "np")]
    models = [Hubbard(nx, ny, ansatz=a, **kw) for nx, ny, kw, L, a in specs]
    layers = [L for *_, L, _ in specs]
    rng = np.random.default_rng(41)
    ths = [rng.uniform(-0.3, 0.3, m.n_params(L)) for m, L in zip(models, layers)]
    b = Batch(models, layers)
    E, g = b.energy_grad(torch.tensor(np.concatenate(ths), dtype=torch.float64, device="cuda"))
    E, g = E.cpu().numpy(), g.cpu().numpy()
    for i, ((nx, ny, kw, L, a), th) in enumerate(zip(specs, ths)):
        om = make_model(nx, ny, **kw)
        E_ref, g_ref = (oc.np_energy_grad(om, th, L) if a == "np" else
                        oc.energy_grad(om, th, L))
        o = b.offsets[i]
        assert abs(E[i] - E_ref) <= 1e-12 * max(1.0, abs(E_ref)), i
        assert np.max(np.abs(g[o:o + th.size] - g_ref)) <= 1e-8, i


def test_np_4x4_open_32q(gpu):
    """The paper's 32-qubit NP workload: 4x4 open, U/t = 2, 12 layers
    (12 * 128 + 32 = 1568 parameters): E(theta) = E(-theta), zero R_z
    gradient entries, and central differences for a hopping rotation and a
    pair phase (about 30 s on MI355X)."""
    m = Hubbard(4, 4, U=2.0, ansatz="np")
    L = 12
    P = m.n_params(L)
    assert P == 1568
    th = torch.tensor(W.vqe_starts(P, 1, seed=5)[0] * 30.0, dtype=torch.float64, device="cuda")
    say("[np 32q] energy_grad(theta), energy(-theta)")
    E1, g1 = m.energy_grad(th)
    E1, g1 = E1.item(), g1.cpu().numpy()
    assert abs(E1 - m.energy(-th).item()) <= 1e-12 * max(1.0, abs(E1))
    assert np.max(np.abs(g1[:32])) <= 1e-12
    say("[np 32q] central differences")
    h = 1e-5
    for k in (32 + 2 * 16 + 4, 32 + 11 * 128 + 127):
        tp, tm = th.clone(), th.clone()
        tp[k] += h
        tm[k] -= h
        fd = (m.energy(tp).item() - m.energy(tm).item()) / (2 * h)
        assert abs(fd - g1[k]) < 1e-8, (k, fd, g1[k])
