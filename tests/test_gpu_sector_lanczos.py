"""Sector-form Lanczos (hubbard_sector_lanczos) on the GPU: ground energies
against the oracle's sector diagonalisation (tests/golden/
sector_ground_energies.json), against the full-vector Lanczos on a 24-qubit
ladder with disorder and V, and at 32 qubits against the free-fermion closed
form (U = 0: twice the sum of the 8 lowest eigenvalues of the 4x4 torus's
hopping matrix) and the eigen-equation H x = E0 x at U = 8."""
import json
import os
import sys

import numpy as np
import pytest
import torch

from oracle import sector as osec
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


def norm(x):
    return torch.linalg.vector_norm(x).item()


@pytest.mark.parametrize("key", sorted(CASES))
def test_sector_lanczos_ground_energy(gpu, key):
    w = CASES[key]()
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    r = m.sector_lanczos(want_state=True)
    E0 = GOLD[key]["E0"]
    say(f"[sector lanczos] {w.name}: E0 = {r['E0']!r} (oracle {E0!r}), {r['iters']} steps, "
        f"residual {r['residual']:.1e}")
    assert abs(r["E0"] - E0) <= 1e-9 * max(1.0, abs(E0))
    assert r["residual"] <= 1e-10 * max(1.0, abs(E0))
    gs = r["state"]
    assert abs(norm(gs) - 1.0) <= 1e-12
    assert norm(m.sector_apply_h(gs) - r["E0"] * gs) <= 1e-8


def test_sector_lanczos_matches_full_vector(gpu):
    """Same start state in both forms: the same ground energy and state (the
    24-qubit ladder with bond disorder, on-site energies and V)."""
    w = W.config3()
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    om = make_model(w.nx, w.ny, **w.kwargs())
    th = torch.tensor(np.random.default_rng(5).uniform(-0.4, 0.4, m.n_params(2)),
                      dtype=torch.float64, device=gpu)
    rs = m.sector_lanczos(m.sector_state(th), want_state=True)
    rf = m.lanczos(m.ansatz(th), want_state=True)
    say(f"[sector lanczos] ladder: sector {rs['E0']!r} ({rs['iters']} steps), full "
        f"{rf['E0']!r} ({rf['iters']} steps)")
    assert abs(rs["E0"] - rf["E0"]) <= 1e-10 * max(1.0, abs(rf["E0"]))
    # the full state restricted to the sector (the oracle's position map)
    idx = torch.tensor(osec.indices(om).astype(np.int64), device=gpu)
    full_in_sector = rf["state"][idx]
    F = abs(torch.vdot(full_in_sector, rs["state"]).item()) ** 2
    assert F >= 1.0 - 1e-9, F


def hopping_ground_energy(nx, ny, n_up, n_dn):
    """Free fermions on the periodic nx x ny torus with t = 1: the sum of the
    lowest one-particle energies -2 cos(2 pi kx / nx) - 2 cos(2 pi ky / ny)."""
    e = np.sort([-2 * np.cos(2 * np.pi * kx / nx) - 2 * np.cos(2 * np.pi * ky / ny)
                 for kx in range(nx) for ky in range(ny)])
    return float(e[:n_up].sum() + e[:n_dn].sum())


def test_sector_lanczos_32q_free_fermions(gpu):
    w = W.config5()
    kw = dict(w.kwargs(), U=0.0)
    m = Hubbard(w.nx, w.ny, **kw)
    r = m.sector_lanczos(max_iter=300, tol=1e-10)
    E0 = hopping_ground_energy(4, 4, 8, 8)
    say(f"[sector lanczos 32q] U=0: E0 = {r['E0']!r} (closed form {E0!r}), {r['iters']} steps")
    assert abs(r["E0"] - E0) <= 1e-9 * abs(E0)


def test_sector_lanczos_32q_U8(gpu):
    """The 4x4 periodic U=8 ground state: H x = E0 x, and the variational
    bound against the benchmark circuit's energy."""
    w = W.config5()
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    r = m.sector_lanczos(max_iter=600, tol=1e-9, want_state=True)
    gs = r["state"]
    hres = norm(m.sector_apply_h(gs) - r["E0"] * gs)
    th = torch.tensor(w.theta, dtype=torch.float64, device=gpu)
    E_circ, _ = m.sector_energy_grad(th)
    say(f"[sector lanczos 32q] U=8: E0 = {r['E0']!r} ({r['E0'] / 16:.10f} per site), "
        f"{r['iters']} steps, Ritz residual {r['residual']:.1e}, ||H x - E0 x|| {hres:.1e}")
    assert r["residual"] <= 1e-9 * abs(r["E0"])
    assert hres <= 1e-7
    assert abs(norm(gs) - 1.0) <= 1e-12
    assert E_circ.item() >= r["E0"]


def test_sector_lanczos_errors(gpu):
    m = Hubbard(2, 2, U=4.0)
    z = torch.zeros(36, dtype=torch.complex128, device=gpu)
    with pytest.raises(abi.HubbardError) as e:
        m.sector_lanczos(z)
    assert e.value.status == abi.HUBBARD_ERR_ARG
    with pytest.raises(ValueError):
        m.sector_lanczos(torch.zeros(35, dtype=torch.complex128, device=gpu))
