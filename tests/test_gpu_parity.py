"""GPU parity: the gfx950 library (called through its C ABI) against the oracle.

Bars: amplitudes max-abs <= 1e-10, energy |dE| <= 1e-12 max(1, |E|),
gradient max-abs <= 1e-8 (complex128 throughout).  Integer/structural
results (zero amplitudes outside the sector) are checked exactly.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import core as oc
from oracle.model import make_model
from paper_2408_00836_amd import abi, workloads as W
from paper_2408_00836_amd.model import EnergyGrad, Hubbard

pytestmark = pytest.mark.gpu

AMP_TOL = 1e-10
GRAD_TOL = 1e-8


def e_tol(E):
    return 1e-12 * max(1.0, abs(E))


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def build(w, tiles=None):
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    if tiles:
        m.set_tiles(*tiles)
    om = make_model(w.nx, w.ny, **w.kwargs())
    return m, om


def th_dev(w, dev):
    return torch.tensor(w.theta, dtype=torch.float64, device=dev)


def compare_all(w, dev, tiles=None, check_amps=True):
    say(f"[parity] {w.name} tiles={tiles}")
    m, om = build(w, tiles)
    assert m.params_per_layer == om.params_per_layer
    th = th_dev(w, dev)
    if check_amps:
        psi = m.ansatz(th)
        torch.cuda.synchronize()
        ref = oc.ansatz(om, w.theta, w.layers)
        err = np.max(np.abs(psi.cpu().numpy() - ref))
        assert err <= AMP_TOL, f"amplitude error {err}"
        # H|psi> on the circuit state
        hp = m.apply_h(psi)
        torch.cuda.synchronize()
        href = oc.ham_apply(om, ref)
        herr = np.max(np.abs(hp.cpu().numpy() - href))
        assert herr <= AMP_TOL * max(1.0, np.max(np.abs(href))), f"H psi error {herr}"
    E_ref, g_ref = oc.energy_grad(om, w.theta, w.layers)
    E1 = m.energy(th).item()
    assert abs(E1 - E_ref) <= e_tol(E_ref), (E1, E_ref)
    E2, g = m.energy_grad(th)
    E2 = E2.item()
    g = g.cpu().numpy()
    assert abs(E2 - E_ref) <= e_tol(E_ref), (E2, E_ref)
    gerr = np.max(np.abs(g - g_ref))
    assert gerr <= GRAD_TOL, f"gradient error {gerr}"
    return m, om, th


def test_config1_2x2(gpu):
    compare_all(W.config1(), gpu)


@pytest.mark.parametrize("U", [1.0, 4.0, 8.0])
def test_config2_chain8(gpu, U):
    import json
    import os
    w = W.config2(U)
    m, om, th = compare_all(w, gpu)
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "sector_ground_energies.json")))
    E0 = gold[f"config2_chain8_U{U:g}"]["E0"]
    assert m.energy(th).item() >= E0 - 1e-12   # variational bound


FD_CONFIGS = {"c1": W.config1, "c2": lambda: W.config2(4.0), "c3": W.config3}


@pytest.mark.parametrize("cfg", sorted(FD_CONFIGS))
def test_adjoint_vs_gpu_fd(gpu, cfg):
    """The plain form's accuracy: central finite differences of the GPU energy
    (h = 1e-5, one energy() call per evaluation) against the oracle's adjoint
    gradient, and the GPU adjoint against both (configs 1, 2 and 3)."""
    w = FD_CONFIGS[cfg]()
    say(f"[fd] {w.name}: {2 * w.n_params} energy evaluations")
    m, om = build(w)
    th = th_dev(w, gpu)
    _, g = m.energy_grad(th)
    g = g.cpu().numpy()
    h = 1e-5
    fd = np.zeros_like(g)
    for k in range(th.numel()):
        tp, tm = th.clone(), th.clone()
        tp[k] += h
        tm[k] -= h
        fd[k] = (m.energy(tp).item() - m.energy(tm).item()) / (2 * h)
    _, g_ref = oc.energy_grad(om, w.theta, w.layers)
    assert np.max(np.abs(fd - g_ref)) < 1e-8
    assert np.max(np.abs(g - fd)) < 1e-8


def test_config3_ladder_24q(gpu):
    """Full 24-qubit config: disorder, eps and V exercise the general diagonal."""
    compare_all(W.config3(), gpu)


MULTI_TILE = [
    # (workload, tiles): small tiles force many tiles per pass and odd layouts
    (W.random_instance(2, 3, 3, 5, 31, U=4.0, disorder=0.1, eps_width=0.5, V=0.5), (6, 6, 2)),
    (W.random_instance(3, 3, 2, 5, 32, U=8.0, disorder=0.1, eps_width=0.5, V=0.5), (8, 7, 3)),
    (W.random_instance(1, 6, 3, 3, 33, periodic_y=True, U=2.0, disorder=0.2), (5, 5, 1)),
    (W.random_instance(2, 4, 2, 5, 34, periodic_y=True, U=4.0), (9, 8, 4)),
    (W.random_instance(4, 2, 2, 5, 35, periodic_x=True, U=4.0, eps_width=0.3), (7, 7, 0)),
    (W.random_instance(1, 9, 2, 3, 36, U=3.0, disorder=0.1, eps_width=0.2, V=0.3), None),
    (W.random_instance(2, 5, 2, 5, 37, U=6.0, disorder=0.1), (12, 11, 4)),
]


@pytest.mark.parametrize("case", range(len(MULTI_TILE)))
def test_multi_tile_layouts(gpu, case):
    w, tiles = MULTI_TILE[case]
    compare_all(w, gpu, tiles)


def test_edge_cases(gpu):
    # zero layers: E = D(b0) = sum eps + sum V; no gradient entries
    w = W.random_instance(2, 3, 0, 5, 41, U=4.0, eps_width=0.5, V=0.5)
    m, om = build(w)
    th = torch.zeros(0, dtype=torch.float64, device=gpu)
    E = m.energy(th).item()
    assert abs(E - (np.sum(w.eps) + np.sum(w.V))) < 1e-12
    # a single site: two qubits, no bonds, only the diagonal slot
    w1 = W.random_instance(1, 1, 2, 1, 42, U=3.0, eps_width=0.5)
    compare_all(w1, gpu)
    # one bond
    compare_all(W.random_instance(1, 2, 3, 2, 43, U=5.0, disorder=0.3), gpu)
    # U = 0 and theta = 0: gradient exactly the time-reversal zero
    w2 = W.random_instance(2, 2, 2, 3, 44, U=0.0)
    m2, _ = build(w2)
    E, g = m2.energy_grad(torch.zeros(6, dtype=torch.float64, device=gpu))
    assert np.max(np.abs(g.cpu().numpy())) < 1e-14
    # user-supplied groups (each bond its own group, reversed order)
    w3 = W.random_instance(1, 4, 2, 4, 45, U=4.0, disorder=0.1)
    m3 = Hubbard(1, 4, groups=[2, 1, 0], **w3.kwargs())
    om3 = make_model(1, 4, groups=[2, 1, 0], **w3.kwargs())
    th3 = th_dev(w3, gpu)
    E3, g3 = m3.energy_grad(th3)
    E3r, g3r = oc.energy_grad(om3, w3.theta, w3.layers)
    assert abs(E3.item() - E3r) < e_tol(E3r)
    assert np.max(np.abs(g3.cpu().numpy() - g3r)) < GRAD_TOL


def test_sector_and_norm_exact(gpu):
    w = W.random_instance(3, 3, 3, 5, 51, U=4.0, disorder=0.1, eps_width=0.5, V=0.5)
    m, om = build(w)
    psi = m.ansatz(th_dev(w, gpu)).cpu().numpy()
    up, dn = om.neel_sites()
    b = np.arange(psi.size)
    nu = sum((b >> s) & 1 for s in range(9))
    nd = sum((b >> (s + 9)) & 1 for s in range(9))
    out = (nu != len(up)) | (nd != len(dn))
    assert np.all(psi[out] == 0.0)
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-13


def test_hamiltonian_apply_random_vector(gpu):
    w = W.config3()
    m, om = build(w)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(m.dim) + 1j * rng.standard_normal(m.dim)
    vt = torch.from_numpy(v).to(gpu)
    out = m.apply_h(vt).cpu().numpy()
    ref = oc.ham_apply(om, v)
    assert np.max(np.abs(out - ref)) < 1e-10 * np.max(np.abs(ref))


def test_autograd_function(gpu):
    w = W.config1()
    m, om = build(w)
    th = th_dev(w, gpu).requires_grad_(True)
    E = EnergyGrad.apply(th, m)
    (2.5 * E).backward()
    _, g_ref = oc.energy_grad(om, w.theta, w.layers)
    assert np.max(np.abs(th.grad.cpu().numpy() - 2.5 * g_ref)) < 1e-8


def test_deterministic_reductions(gpu):
    w = W.config2(4.0)
    m, _ = build(w)
    th = th_dev(w, gpu)
    E1, g1 = m.energy_grad(th)
    E1, g1 = E1.clone(), g1.clone()
    E2, g2 = m.energy_grad(th)
    assert torch.equal(E1, E2) and torch.equal(g1, g2)


def test_workspace_too_small_is_an_error(gpu):
    w = W.config1()
    m, _ = build(w)
    th = th_dev(w, gpu)
    E = torch.empty(1, dtype=torch.float64, device=gpu)
    g = torch.empty(6, dtype=torch.float64, device=gpu)
    ws = torch.empty(100, dtype=torch.uint8, device=gpu)
    with pytest.raises(abi.HubbardError) as e:
        abi.energy_grad(m.handle, th.data_ptr(), 2, E.data_ptr(), g.data_ptr(), ws.data_ptr(),
                        ws.numel(), 0)
    assert e.value.status == abi.HUBBARD_ERR_SIZE
