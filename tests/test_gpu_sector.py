"""GPU parity of the particle-number sector form (sector_ansatz_apply,
sector_hamiltonian_apply, sector_energy_grad) against the oracle.

The oracle side is oracle.sector (plain C loops over the sector's amplitudes,
pinned to the full-space oracle bit for bit in test_oracle_sector.py) and,
for energies and gradients, the full-space oracle itself.  At 32 qubits the
references are the stored oracle values of the 4x4 periodic benchmark
circuit (tests/golden/c5_4x4_periodic_U8.json).

Bars: amplitudes max-abs <= 1e-10, |dE| <= 1e-12 max(1, |E|), gradient
max-abs <= 1e-8.  The sector vector's element order is the oracle's
(r_dn * C(Ns, N_up) + r_up), so amplitudes compare element by element.
"""
import json
import os
import sys

import numpy as np
import pytest
import torch

from oracle import core as oc
from oracle import sector as osec
from oracle.model import make_model
from paper_2408_00836_amd import abi, workloads as W
from paper_2408_00836_amd.model import Hubbard

pytestmark = pytest.mark.gpu

AMP_TOL = 1e-10
GRAD_TOL = 1e-8
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "c5_4x4_periodic_U8.json")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def e_tol(E):
    return 1e-12 * max(1.0, abs(E))


CASES = {
    "c1": W.config1,
    "c2": lambda: W.config2(4.0),
    "c3": W.config3,
    # odd site count: N_up = 3, N_dn = 2, a non-square sector matrix
    "chain5": lambda: W.random_instance(1, 5, 3, 3, 4201, U=3.0, disorder=0.1,
                                        eps_width=0.3, V=0.4, name="1x5 chain V eps"),
    "ladder2x4": lambda: W.random_instance(2, 4, 3, 5, 4202, U=5.0, disorder=0.1,
                                           name="2x4 ladder U=5"),
}


@pytest.mark.parametrize("key", list(CASES))
def test_sector_vs_oracle(gpu, key):
    w = CASES[key]()
    say(f"[sector] {w.name}")
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    om = make_model(w.nx, w.ny, **w.kwargs())
    nu, nd = m.sector_dims()
    assert nu * nd == osec.dim(om)
    th = torch.tensor(w.theta, dtype=torch.float64, device=gpu)
    # circuit state, element by element
    psi = m.sector_state(th)
    ref = osec.ansatz(om, w.theta, w.layers)
    amp = float(np.max(np.abs(psi.cpu().numpy() - ref)))
    # H on a seeded random sector vector (numpy's generator, fed to both)
    rng = np.random.default_rng(4300)
    x = rng.standard_normal(ref.size) + 1j * rng.standard_normal(ref.size)
    hx = m.sector_apply_h(torch.tensor(x, device=gpu))
    href = osec.ham_apply(om, x)
    herr = float(np.max(np.abs(hx.cpu().numpy() - href)) / max(1.0, np.max(np.abs(href))))
    # energy and gradient against the full-space oracle
    E, g = m.sector_energy_grad(th)
    E_ref, g_ref = oc.energy_grad(om, w.theta, w.layers)
    dE = abs(E.item() - E_ref)
    dg = float(np.max(np.abs(g.cpu().numpy() - g_ref)))
    say(f"[sector] {w.name}: dims {nu}x{nd}, amp {amp:.2e}, H {herr:.2e}, dE {dE:.2e}, "
        f"dg {dg:.2e}")
    assert amp <= AMP_TOL
    assert herr <= AMP_TOL
    assert dE <= e_tol(E_ref)
    assert dg <= GRAD_TOL
    # the same numbers as the full-vector path
    E2, g2 = m.energy_grad(th)
    assert abs(E.item() - E2.item()) <= e_tol(E_ref)
    assert float(np.max(np.abs(g.cpu().numpy() - g2.cpu().numpy()))) <= GRAD_TOL


# Rows long enough for the wider register tiles (2, 4 and 8 elements per
# thread of the 1024-thread row workgroup; the 32-qubit circuit below has 13):
# checked against the sector oracle alone (pinned to the full-space oracle
# in the CPU tests), since the full vectors of 26-30 qubits are beyond the
# full-space oracle's test budget.
TILE_CASES = {
    "chain13 (2 per thread)": lambda: W.random_instance(1, 13, 2, 3, 4310, U=4.0, disorder=0.1,
                                                        eps_width=0.2, V=0.3,
                                                        name="1x13 chain eps V"),
    "ladder2x7 (4 per thread)": lambda: W.random_instance(2, 7, 1, 5, 4311, U=6.0, disorder=0.1,
                                                          name="2x7 ladder U=6"),
    "lattice3x5 (8 per thread)": lambda: W.random_instance(3, 5, 1, 5, 4312, U=3.0,
                                                           disorder=0.1, eps_width=0.3, V=0.4,
                                                           name="3x5 U=3 eps V"),
}


@pytest.mark.parametrize("key", list(TILE_CASES))
def test_sector_register_tiles(gpu, key):
    w = TILE_CASES[key]()
    say(f"[sector tiles] {w.name}")
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    om = make_model(w.nx, w.ny, **w.kwargs())
    th = torch.tensor(w.theta, dtype=torch.float64, device=gpu)
    psi = m.sector_state(th)
    ref = osec.ansatz(om, w.theta, w.layers)
    amp = float(np.max(np.abs(psi.cpu().numpy() - ref)))
    hx = m.sector_apply_h(psi)
    href = osec.ham_apply(om, ref)
    herr = float(np.max(np.abs(hx.cpu().numpy() - href)) / max(1.0, np.max(np.abs(href))))
    E, g = m.sector_energy_grad(th)
    E_ref, g_ref = osec.energy_grad(om, w.theta, w.layers)
    dE = abs(E.item() - E_ref)
    dg = float(np.max(np.abs(g.cpu().numpy() - g_ref)))
    say(f"[sector tiles] {w.name}: amp {amp:.2e}, H {herr:.2e}, dE {dE:.2e}, dg {dg:.2e}")
    assert amp <= AMP_TOL
    assert herr <= AMP_TOL
    assert dE <= e_tol(E_ref)
    assert dg <= GRAD_TOL


def test_sector_general_diagonal_32q(gpu):
    """Rows of 12870 (13 elements per thread) with the general diagonal
    (on-site energies and V): the sector form against the full-vector path
    (itself pinned to the oracle up to 24 qubits with the same diagonal) on a
    4x4 open lattice, two layers: E, every gradient entry, and amplitudes at
    sampled positions."""
    w = W.random_instance(4, 4, 2, 5, 4320, U=6.0, disorder=0.1, eps_width=0.4, V=0.5,
                          name="4x4 open eps V")
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    th = torch.tensor(w.theta, dtype=torch.float64, device=gpu)
    Es, gs = m.sector_energy_grad(th)
    psi_s = m.sector_state(th)
    om = make_model(w.nx, w.ny, **w.kwargs())
    rng = np.random.default_rng(4321)
    pos = np.sort(rng.choice(psi_s.numel(), 256, replace=False))
    idx = osec.indices(om)[pos].astype(np.int64)
    amp_s = psi_s[torch.tensor(pos, device=gpu)].cpu().numpy()
    del psi_s
    m.release_sector_workspaces()
    torch.cuda.empty_cache()
    Ef, gf = m.energy_grad(th)
    psi_f = m.ansatz(th)
    amp_f = psi_f[torch.tensor(idx, device=gpu)].cpu().numpy()
    del psi_f
    dE = abs(Es.item() - Ef.item())
    dg = float(np.max(np.abs(gs.cpu().numpy() - gf.cpu().numpy())))
    amp = float(np.max(np.abs(amp_s - amp_f)))
    say(f"[sector 32q general] dE {dE:.2e} dg {dg:.2e} amp {amp:.2e}")
    assert dE <= e_tol(Ef.item())
    assert dg <= GRAD_TOL
    assert amp <= AMP_TOL


@pytest.mark.parametrize("layers", [0, 1, 2])
def test_sector_short_circuits(gpu, layers):
    w = W.random_instance(2, 3, layers, 5, 4203 + layers, U=4.0, disorder=0.1, eps_width=0.2,
                          V=0.3, name=f"2x3 {layers} layers")
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    om = make_model(w.nx, w.ny, **w.kwargs())
    th = torch.tensor(w.theta, dtype=torch.float64, device=gpu)
    E, g = m.sector_energy_grad(th)
    E_ref, g_ref = oc.energy_grad(om, w.theta, w.layers)
    assert abs(E.item() - E_ref) <= e_tol(E_ref)
    if layers:
        assert float(np.max(np.abs(g.cpu().numpy() - g_ref))) <= GRAD_TOL


def test_sector_errors(gpu):
    m = Hubbard(2, 2, U=4.0)
    with pytest.raises(ValueError):
        m.sector_apply_h(torch.zeros(36, dtype=torch.complex128))   # a host tensor
    a = torch.zeros(36, dtype=torch.complex128, device=gpu)
    ws = torch.empty(1 << 16, dtype=torch.uint8, device=gpu)
    with pytest.raises(abi.HubbardError) as e:
        abi.sector_hamiltonian_apply(m.handle, a.data_ptr(), a.data_ptr(), ws.data_ptr(),
                                     ws.numel(), 0)
    assert e.value.status == abi.HUBBARD_ERR_ARG
    th = torch.zeros(6, dtype=torch.float64, device=gpu)
    with pytest.raises(abi.HubbardError) as e:
        abi.sector_energy_grad(m.handle, th.data_ptr(), 2, th.data_ptr(), th.data_ptr(),
                               ws.data_ptr(), 16, 0)
    assert e.value.status == abi.HUBBARD_ERR_SIZE
    m.set_ansatz("np")
    with pytest.raises(abi.HubbardError) as e:
        m.sector_dims()
    assert e.value.status == abi.HUBBARD_ERR_STATE


def test_sector_32q_benchmark_circuit(gpu):
    """The 4x4 periodic U=8 circuit at the benchmark angles: E, all 80
    gradient entries and the stored amplitudes of the oracle's sector run."""
    gold = json.load(open(GOLDEN))
    w = W.config5()
    assert np.allclose(gold["theta"], w.theta, rtol=0, atol=0)
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    om = make_model(w.nx, w.ny, **w.kwargs())
    nu, nd = m.sector_dims()
    assert nu * nd == gold["sector_dim"]
    th = torch.tensor(w.theta, dtype=torch.float64, device=gpu)
    E, g = m.sector_energy_grad(th)
    dE = abs(E.item() - gold["E"])
    dg = float(np.max(np.abs(g.cpu().numpy() - np.array(gold["grad"]))))
    psi = m.sector_state(th)
    # sector position of a full index: rank of the down pattern times the
    # number of up patterns plus the rank of the up pattern (ranks among the
    # 16-bit patterns with 8 set bits, in increasing order)
    pats = np.array([p for p in range(1 << 16) if bin(p).count("1") == 8], dtype=np.int64)
    idx = np.array(gold["amp_index"], dtype=np.int64)
    pos = np.searchsorted(pats, idx >> 16) * pats.size + np.searchsorted(pats, idx & 0xFFFF)
    assert osec.position(om, int(idx[-1])) == int(pos[-1])   # the start state, by the oracle
    got = psi[torch.tensor(pos, device=gpu)].cpu().numpy()
    want = np.array(gold["amp_re"]) + 1j * np.array(gold["amp_im"])
    amp = float(np.max(np.abs(got - want)))
    norm = float(torch.linalg.vector_norm(psi).item())
    say(f"[sector 32q] dE {dE:.2e} dg {dg:.2e} amp {amp:.2e} |norm-1| {abs(norm - 1):.1e}")
    assert dE <= e_tol(gold["E"])
    assert dg <= GRAD_TOL
    assert amp <= AMP_TOL
    assert abs(norm - 1.0) <= 1e-12


# Degenerate sectors: a single amplitude (one site; every spin up, where
# every hop is Pauli-blocked and the energy is the diagonal alone) and
# one-row / one-column sector matrices (a single electron of one spin),
# where one layout's rows hold one element and its gates no pair at all.
# Graph models with explicit start spins, against the sector and full-space
# oracles; the sector Lanczos against the lowest eigenvalue of the oracle's
# sector H assembled column by column.
DEGENERATE = {
    "one site": (1, [], [0]),
    "ring4 all up": (4, [(0, 1), (1, 2), (2, 3), (0, 3)], [0, 0, 0, 0]),
    "5 sites, one down": (5, [(0, 1), (1, 2), (2, 3), (3, 4), (0, 3)], [0, 0, 0, 1, 0]),
    "6 sites, one up": (6, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (0, 5), (1, 4)],
                        [1, 1, 1, 1, 1, 0]),
}


@pytest.mark.parametrize("key", list(DEGENERATE))
def test_sector_degenerate_sectors(gpu, key):
    from oracle.model import make_graph_model
    n, bonds, spins = DEGENERATE[key]
    rng = np.random.default_rng(77 + n)
    nb = len(bonds)
    kw = dict(t=(1 + 0.2 * rng.standard_normal(nb)) if nb else None, U=3.0,
              V=rng.uniform(-0.5, 0.5, nb) if nb else None, eps=rng.uniform(-0.5, 0.5, n))
    om = make_graph_model(n, bonds, site_spin=spins, **kw)
    m = Hubbard.graph(n, np.asarray(bonds, dtype=np.int32).reshape(-1, 2), site_spin=spins,
                      **kw)
    L = 2
    th_h = rng.uniform(-np.pi / 8, np.pi / 8, L * om.params_per_layer)
    th = torch.tensor(th_h, dtype=torch.float64, device=gpu)
    nu, nd = m.sector_dims()
    dim = osec.dim(om)
    say(f"[sector degenerate] {key}: dims {nu}x{nd}")
    assert nu * nd == dim
    psi = m.sector_state(th)
    ref = osec.ansatz(om, th_h, L)
    amp = float(np.max(np.abs(psi.cpu().numpy() - ref)))
    x = rng.standard_normal(dim) + 1j * rng.standard_normal(dim)
    hx = m.sector_apply_h(torch.tensor(x, device=gpu)).cpu().numpy()
    href = osec.ham_apply(om, x)
    herr = float(np.max(np.abs(hx - href)) / max(1.0, np.max(np.abs(href))))
    E, g = m.sector_energy_grad(th)
    E_ref, g_ref = oc.energy_grad(om, th_h, L)
    dE = abs(E.item() - E_ref)
    dg = float(np.max(np.abs(g.cpu().numpy() - g_ref)))
    Hs = np.stack([osec.ham_apply(om, np.eye(dim, dtype=np.complex128)[:, c])
                   for c in range(dim)], axis=1)
    e0 = float(np.linalg.eigvalsh(0.5 * (Hs + Hs.conj().T))[0])
    lz = m.sector_lanczos()
    say(f"[sector degenerate] {key}: amp {amp:.2e}, H {herr:.2e}, dE {dE:.2e}, dg {dg:.2e}, "
        f"E0 {lz['E0']:.12f} (ED {e0:.12f}, {lz['iters']} steps)")
    assert amp <= AMP_TOL
    assert herr <= AMP_TOL
    assert dE <= e_tol(E_ref)
    assert dg <= GRAD_TOL
    assert abs(lz["E0"] - e0) <= 1e-9 * max(1.0, abs(e0))
    if dim == 1:   # a single amplitude: a phase only, the energy is the diagonal
        assert abs(abs(ref[0]) - 1.0) <= 1e-12
        assert float(np.max(np.abs(g_ref))) <= 1e-12
    E2, g2 = m.energy_grad(th)
    assert abs(E.item() - E2.item()) <= e_tol(E_ref)
    assert float(np.max(np.abs(g.cpu().numpy() - g2.cpu().numpy()))) <= GRAD_TOL
