"""Krylov ground state (hubbard_lanczos) and overlaps (hubbard_overlap) on the
GPU against the oracle: sector ground energies from dense / sparse
diagonalisation of the oracle's H (tests/golden/sector_ground_energies.json),
ground-state fidelity against the oracle's eigenvector, exact zeros outside
the sector, overlaps against the oracle's compensated inner product."""
import json
import os
import sys

import numpy as np
import pytest
import torch

from oracle import core as oc
from oracle import dense as od
from oracle.model import make_model
from paper_2408_00836_amd import abi, workloads as W
from paper_2408_00836_amd.model import Hubbard

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                   "sector_ground_energies.json")))


def say(*a):
    print(*a, file=sys.stderr, flush=True)


CASES = {
    "config1_2x2_U4": W.config1,
    "config2_chain8_U1": lambda: W.config2(1.0),
    "config2_chain8_U4": lambda: W.config2(4.0),
    "config2_chain8_U8": lambda: W.config2(8.0),
    "config3_ladder_2x6": W.config3,
}


@pytest.mark.parametrize("key", sorted(CASES))
def test_lanczos_sector_ground_energy(gpu, key):
    w = CASES[key]()
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    say(f"[lanczos] {w.name}")
    r = m.lanczos(want_state=True)
    E0 = GOLD[key]["E0"]
    say(f"[lanczos] E0 = {r['E0']!r} (oracle {E0!r}), {r['iters']} steps, "
        f"residual {r['residual']:.1e}")
    assert abs(r["E0"] - E0) <= 1e-9 * max(1.0, abs(E0))
    assert r["residual"] <= 1e-10 * max(1.0, abs(E0))
    gs = r["state"]
    # unit norm, H gs = E0 gs, and nothing outside the start state's sector
    assert abs(m.overlap(gs, gs).item() - 1.0) <= 1e-12
    hg = m.apply_h(gs)
    assert torch.linalg.vector_norm(hg - r["E0"] * gs).item() <= 1e-8
    om = make_model(w.nx, w.ny, **w.kwargs())
    up, dn = om.neel_sites()
    ns = om.nsites
    if om.nqubits <= 16:
        x = gs.cpu().numpy()
        pop_up = np.array([bin(b & ((1 << ns) - 1)).count("1") for b in range(x.size)])
        pop_dn = np.array([bin(b >> ns).count("1") for b in range(x.size)])
        out = (pop_up != len(up)) | (pop_dn != len(dn))
        assert np.all(x[out] == 0.0)
        # fidelity with the oracle's eigenvector (dense / sparse eigh)
        wref, vref = od.sector_ground_state(om, len(up), len(dn), k=2)
        assert abs(wref[0] - r["E0"]) <= 1e-9 * max(1.0, abs(E0))
        if wref[1] - wref[0] > 1e-6:   # nondegenerate: the state is unique up to phase
            F = abs(np.vdot(vref[:, 0], x)) ** 2
            assert F >= 1.0 - 1e-10, F


def test_vqe_state_fidelity_and_bound(gpu):
    """Config 2's diagnostic: fidelity of the circuit state with the Lanczos
    ground state, and the variational bound E(theta) >= E0."""
    w = W.config2(4.0)
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    th = torch.tensor(w.theta, dtype=torch.float64, device="cuda")
    psi = m.ansatz(th)
    r = m.lanczos(want_state=True)
    F = abs(m.overlap(psi, r["state"]).item()) ** 2
    om = make_model(w.nx, w.ny, **w.kwargs())
    x = oc.ansatz(om, w.theta, w.layers)
    _, vref = od.sector_ground_state(om, 4, 4, k=1)
    F_ref = abs(np.vdot(x, vref[:, 0])) ** 2
    assert abs(F - F_ref) <= 1e-10
    assert m.energy(th).item() >= r["E0"] - 1e-12
    # the circuit keeps the checkerboard start's total-spin weights and the
    # ground state is a singlet: F <= the start's singlet weight 1 / (N/2 + 1)
    assert F <= 1.0 / (w.nx * w.ny // 2 + 1) + 1e-12


def test_overlap_matches_oracle(gpu):
    w = W.config3()
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    a = torch.randn(m.dim, dtype=torch.complex128, device="cuda", generator=g)
    b = torch.randn(m.dim, dtype=torch.complex128, device="cuda", generator=g)
    got = m.overlap(a, b).item()
    ref = oc.inner(a.cpu().numpy(), b.cpu().numpy())
    scale = float(torch.linalg.vector_norm(a) * torch.linalg.vector_norm(b))
    assert abs(got - ref) <= 1e-13 * scale
    # reproducible: the same sum in the same order
    assert m.overlap(a, b).item() == got


def test_lanczos_errors(gpu):
    w = W.config1()
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    z = torch.zeros(m.dim, dtype=torch.complex128, device="cuda")
    with pytest.raises(abi.HubbardError) as e:
        m.lanczos(z)
    assert e.value.status == abi.HUBBARD_ERR_ARG
