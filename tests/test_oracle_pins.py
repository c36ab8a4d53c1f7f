"""Pins of the oracle to things other than itself (CPU only).

Each test ties a part of the oracle to a closed form, a textbook special case,
an independent mechanism (explicit Kronecker-product matrices, Slater
determinants and Wick's theorem) or an exact invariant, so that a dropped
term, a wrong sign or index, or a transposed operand fails at least one.
"""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import core as oc
from oracle import dense as od
from oracle import freefermion as ff
from oracle.model import make_model

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(7)


def sector_of(m, b):
    nu = sum((b >> m.qubit(s, 0)) & 1 for s in range(m.nsites))
    nd = sum((b >> m.qubit(s, 1)) & 1 for s in range(m.nsites))
    return nu, nd


def oracle_sector_spectrum(m, nu, nd):
    idx = [b for b in range(1 << m.nqubits) if sector_of(m, b) == (nu, nd)]
    H = oc.ham_matrix(m, idx)
    assert np.allclose(H, H.conj().T, atol=1e-14)
    return np.linalg.eigvalsh(H)


# ------------------------------------------------------------ closed forms --

@pytest.mark.parametrize("t,U", [(1.0, 4.0), (1.0, 8.0), (0.7, 2.0), (1.3, 0.0)])
def test_two_site_closed_form(oracle_lib, t, U):
    """Two sites, one up and one down electron: E0 = U/2 - sqrt(U^2/4 + 4t^2).
    Pins the hopping normalisation (each bond once, both directions) and U."""
    m = make_model(1, 2, t=[t], U=U)
    E0 = oracle_sector_spectrum(m, 1, 1)[0]
    assert abs(E0 - (U / 2 - np.sqrt(U * U / 4 + 4 * t * t))) < 1e-12


@pytest.mark.parametrize("U,V", [(4.0, 0.5), (2.0, 1.3), (8.0, 0.0)])
def test_two_site_with_V_closed_form(oracle_lib, U, V):
    """With nearest-neighbour V (Eq. (16), V n_i n_j once per bond):
    E0 = (U+V)/2 - sqrt(((U-V)/2)^2 + 4t^2) in the 1 up / 1 down sector."""
    m = make_model(1, 2, U=U, V=[V])
    E0 = oracle_sector_spectrum(m, 1, 1)[0]
    assert abs(E0 - ((U + V) / 2 - np.sqrt(((U - V) / 2) ** 2 + 4.0))) < 1e-12


def test_two_site_eps_shift(oracle_lib):
    """On-site energies enter as eps_i n_i: with eps_1 = eps_2 = e every state
    of the two-electron sector shifts by exactly 2e."""
    m0 = make_model(1, 2, U=3.0)
    m1 = make_model(1, 2, U=3.0, eps=[0.37, 0.37])
    s0 = oracle_sector_spectrum(m0, 1, 1)
    s1 = oracle_sector_spectrum(m1, 1, 1)
    assert np.max(np.abs(s1 - s0 - 0.74)) < 1e-12


# ------------------------------------------------- free fermions (U=V=0) --

def free_sector_spectrum(m, nu, nd):
    """All sums of nu and nd distinct single-particle energies of h."""
    w = np.linalg.eigvalsh(ff.one_body(m))
    su = [sum(c) for c in itertools.combinations(w, nu)]
    sd = [sum(c) for c in itertools.combinations(w, nd)]
    return np.sort(np.add.outer(su, sd).ravel())


@pytest.mark.parametrize("nx,ny,px,py", [(1, 4, False, True), (2, 2, False, False),
                                         (1, 6, False, True), (2, 3, False, False)])
def test_free_fermion_full_sector_spectrum(oracle_lib, nx, ny, px, py):
    """U = V = 0: every many-body level of the (N_up, N_dn) sector is a sum of
    single-particle levels of h (h_ij = -t_ij, h_ii = eps_i).  Pins all
    Jordan-Wigner signs, including the periodic wrap bonds."""
    m0 = make_model(nx, ny, periodic_x=px, periodic_y=py)
    nb, ns = len(m0.bonds), m0.nsites
    m = make_model(nx, ny, periodic_x=px, periodic_y=py, t=1 + 0.2 * RNG.standard_normal(nb),
                   eps=RNG.uniform(-0.5, 0.5, ns))
    up, dn = m.neel_sites()
    got = oracle_sector_spectrum(m, len(up), len(dn))
    want = free_sector_spectrum(m, len(up), len(dn))
    assert got.shape == want.shape
    assert np.max(np.abs(got - want)) < 1e-11


def test_four_ring_half_filling_minus_four(oracle_lib):
    """Periodic 4-site ring, t = 1, U = 0, 2 up + 2 down: E0 = -4t
    (levels -2, 0, 0, 2; each spin fills -2 and one 0)."""
    m = make_model(1, 4, periodic_y=True)
    assert abs(oracle_sector_spectrum(m, 2, 2)[0] + 4.0) < 1e-12


# ------------------------------------- independent dense Kronecker check --

DENSE_CASES = [
    dict(nx=2, ny=2, U=4.0, L=2),
    dict(nx=1, ny=4, py=True, U=2.0, L=2, disorder=0.3, eps=0.4, V=0.6),
    dict(nx=1, ny=5, U=8.0, L=2, disorder=0.2, eps=0.3, V=0.2),
]


def dense_case(c, interleaved=False):
    nx, ny = c["nx"], c["ny"]
    m0 = make_model(nx, ny, periodic_y=c.get("py", False))
    nb, ns = len(m0.bonds), m0.nsites
    rng = np.random.default_rng(nx * 100 + ny)
    t = 1 + c.get("disorder", 0.0) * rng.standard_normal(nb)
    eps = rng.uniform(-c.get("eps", 0.0), c.get("eps", 0.0), ns)
    V = np.full(nb, c.get("V", 0.0))
    m = make_model(nx, ny, periodic_y=c.get("py", False), t=t, U=c["U"], V=V, eps=eps,
                   interleaved=interleaved)
    th = rng.uniform(-np.pi / 8, np.pi / 8, c["L"] * m.params_per_layer)
    return m, th


@pytest.mark.parametrize("case", DENSE_CASES)
def test_dense_hamiltonian_matches(oracle_lib, case):
    m, _ = dense_case(case)
    _, H = od.generators(m)
    Hd = H.toarray()
    dim = 1 << m.nqubits
    cols = np.stack([oc.ham_apply(m, oc.basis(m, b)) for b in range(dim)], axis=1)
    assert np.max(np.abs(cols - Hd)) < 1e-13


@pytest.mark.parametrize("case", DENSE_CASES)
def test_ham_row_matches_dense(oracle_lib, case):
    # the row form used for sampled checks at 32 qubits, against the dense
    # Kronecker-product H (an independent construction of the same operator)
    m, _ = dense_case(case)
    _, H = od.generators(m)
    Hd = H.toarray()
    for b in range(1 << m.nqubits):
        row = np.zeros(1 << m.nqubits, dtype=np.complex128)
        cols, coefs = oc.ham_row(m, b)
        for c, v in zip(cols, coefs):
            row[int(c)] += v
        assert np.max(np.abs(row - Hd[b])) < 1e-13


@pytest.mark.parametrize("case", DENSE_CASES)
def test_dense_circuit_energy_gradient(oracle_lib, case):
    """Amplitudes from eigendecomposed exp(-i th G) products, E from the dense
    H, gradient by forward-mode differentiation -- all independent of the
    oracle's bit loops and adjoint recursion."""
    m, th = dense_case(case)
    L = case["L"]
    dc = od.DenseCircuit(m)
    psi = oc.ansatz(m, th, L)
    assert np.max(np.abs(psi - dc.state(th, L))) < 1e-12
    E, g = oc.energy_grad(m, th, L)
    assert abs(E - dc.energy(th, L)) < 1e-12 * max(1, abs(E))
    assert np.max(np.abs(g - dc.grad(th, L))) < 1e-11


def test_dense_group_commutation(oracle_lib):
    """Each hopping group's terms commute, so exp of the group sum equals the
    product of the term exponentials that the oracle applies."""
    m, th = dense_case(DENSE_CASES[1])
    gens, _ = od.generators(m)
    for slot in range(1, len(gens)):
        G = gens[slot]
        rng = np.random.default_rng(3)
        dim = 1 << m.nqubits
        psi = rng.standard_normal(dim) + 1j * rng.standard_normal(dim)
        psi /= np.linalg.norm(psi)
        got = oc.apply_slot(m, slot, 0.37, psi.copy())
        w, V = np.linalg.eigh(G.toarray())
        want = V @ (np.exp(-1j * 0.37 * w) * (V.conj().T @ psi))
        assert np.max(np.abs(got - want)) < 1e-13


# ------------------------------------------------ Slater determinant case --

@pytest.mark.parametrize("nx,ny,px,py", [(2, 3, False, False), (1, 6, False, True),
                                         (2, 4, False, True)])
def test_free_fermion_circuit(oracle_lib, nx, ny, px, py):
    """Zero diagonal angles after layer 0: the circuit state is one Slater
    determinant per spin.  Amplitudes (determinants), energy (Wick) and every
    hopping-parameter gradient must match the oracle."""
    m0 = make_model(nx, ny, periodic_x=px, periodic_y=py)
    nb, ns = len(m0.bonds), m0.nsites
    rng = np.random.default_rng(11 + ns)
    m = make_model(nx, ny, periodic_x=px, periodic_y=py, t=1 + 0.1 * rng.standard_normal(nb),
                   U=4.0, V=np.full(nb, 0.5), eps=rng.uniform(-0.5, 0.5, ns))
    L = 3
    per = m.params_per_layer
    th = rng.uniform(-np.pi / 8, np.pi / 8, L * per)
    for l in range(1, L):
        th[l * per] = 0.0
    psi = oc.ansatz(m, th, L)
    C = ff.orbitals(m, th, L)
    ph = ff.start_phase(m, th, L)
    idx = rng.choice(psi.size, 400, replace=False)
    nz = np.nonzero(np.abs(psi) > 1e-3)[0][:200]
    for b in list(idx) + list(nz):
        assert abs(psi[b] - ff.amplitude(m, C, int(b), ph)) < 1e-12
    E, g = oc.energy_grad(m, th, L)
    assert abs(E - ff.energy(m, th, L)) < 1e-12 * max(1, abs(E))
    for k, v in ff.hop_gradients(m, th, L).items():
        assert abs(g[k] - v) < 1e-11, k


# ----------------------------------------------------- row factorisation --

def test_row_factorised_ladder(oracle_lib):
    """2 x 4 periodic-in-y ladder, V = 0, all vertical angles zero: every gate
    is row-local in the spin-blocked order, so the 16-qubit state is the
    product of two 4-site ring states (each ring starting from its row's
    checkerboard pattern); E and the U/h gradients are sums over rows."""
    rng = np.random.default_rng(5)
    eps = rng.uniform(-0.5, 0.5, 8)
    t_h = 1 + 0.1 * rng.standard_normal(8)
    m = make_model(2, 4, periodic_y=True, U=4.0, eps=eps,
                   t=np.concatenate([t_h, np.ones(4)]))
    assert m.params_per_layer == 5
    L = 3
    th = rng.uniform(-np.pi / 8, np.pi / 8, L * 5)
    th[2::5] = 0.0   # v1
    th[4::5] = 0.0   # v2
    psi = oc.ansatz(m, th, L)
    E, g = oc.energy_grad(m, th, L)
    rings, Es, gs = [], 0.0, np.zeros_like(g)
    for r in range(2):
        ring = make_model(1, 4, periodic_y=True, U=4.0, eps=eps[4 * r:4 * r + 4],
                          t=t_h[4 * r:4 * r + 4])
        assert ring.params_per_layer == 3
        b0 = 0
        for y in range(4):
            spin = (r + y) % 2
            b0 |= 1 << ring.qubit(y, spin)
        thr = np.stack([th[0::5], th[1::5], th[3::5]], axis=1).ravel()
        rings.append(oc.ansatz(ring, thr, L, b0))
        Er, gr = oc.energy_grad(ring, thr, L, b0)
        Es += Er
        gs[0::5] += gr[0::3]
        gs[1::5] += gr[1::3]
        gs[3::5] += gr[2::3]
    for b in rng.choice(psi.size, 3000, replace=False):
        b = int(b)
        r0 = (b & 0xF) | (((b >> 8) & 0xF) << 4)
        r1 = ((b >> 4) & 0xF) | (((b >> 12) & 0xF) << 4)
        assert abs(psi[b] - rings[0][r0] * rings[1][r1]) < 1e-13
    assert abs(E - Es) < 1e-12 * max(1, abs(E))
    for k in list(range(0, 15, 5)) + list(range(1, 15, 5)) + list(range(3, 15, 5)):
        assert abs(g[k] - gs[k]) < 1e-11


# ------------------------------------------------------------- invariants --

def invariant_model():
    rng = np.random.default_rng(21)
    m = make_model(2, 3, t=1 + 0.1 * rng.standard_normal(7), U=4.0, V=np.full(7, 0.5),
                   eps=rng.uniform(-0.5, 0.5, 6))
    th = rng.uniform(-np.pi / 8, np.pi / 8, 4 * m.params_per_layer)
    return m, th, 4


def test_norm_and_particle_number(oracle_lib):
    m, th, L = invariant_model()
    psi = oc.ansatz(m, th, L)
    assert abs(np.vdot(psi, psi).real - 1) < 1e-13
    up, dn = m.neel_sites()
    for b in range(psi.size):
        if sector_of(m, b) != (len(up), len(dn)):
            assert psi[b] == 0.0   # exactly: gates only mix in-sector pairs


def test_time_reversal_symmetry(oracle_lib):
    """H and every generator are real and psi0 is real: E(th) = E(-th) and the
    gradient is odd, hence zero at th = 0."""
    m, th, L = invariant_model()
    E1, g1 = oc.energy_grad(m, th, L)
    E2, g2 = oc.energy_grad(m, -th, L)
    assert abs(E1 - E2) < 1e-12
    assert np.max(np.abs(g1 + g2)) < 1e-12
    _, g0 = oc.energy_grad(m, np.zeros_like(th), L)
    assert np.max(np.abs(g0)) < 1e-13


def test_first_diagonal_gradient_zero_and_initial_energy(oracle_lib):
    """psi0 is a D eigenstate, so layer 0's diagonal angle is a global phase;
    at th = 0, E = D(b0) = sum eps + sum V (every site singly occupied)."""
    m, th, L = invariant_model()
    _, g = oc.energy_grad(m, th, L)
    assert abs(g[0]) < 1e-13
    E0 = oc.energy(m, np.zeros_like(th), L)
    assert abs(E0 - (np.sum(m.eps) + np.sum(m.V))) < 1e-13


def test_hermiticity(oracle_lib):
    m, _, _ = invariant_model()
    rng = np.random.default_rng(2)
    a = rng.standard_normal(1 << 12) + 1j * rng.standard_normal(1 << 12)
    b = rng.standard_normal(1 << 12) + 1j * rng.standard_normal(1 << 12)
    lhs = np.vdot(a, oc.ham_apply(m, b))
    rhs = np.conj(np.vdot(b, oc.ham_apply(m, a)))
    assert abs(lhs - rhs) < 1e-10


def test_periodicity_in_theta(oracle_lib):
    """t = 1: each hopping gate has period 2 pi (pair rotations by th).
    Integer U = 4, V = eps = 0: the diagonal gate has period 2 pi / 4."""
    m = make_model(2, 2, U=4.0)
    rng = np.random.default_rng(9)
    th = rng.uniform(-1, 1, 6)
    E = oc.energy(m, th, 2)
    for k, per in [(1, 2 * np.pi), (2, 2 * np.pi), (3, np.pi / 2), (5, 2 * np.pi)]:
        t2 = th.copy()
        t2[k] += per
        assert abs(oc.energy(m, t2, 2) - E) < 1e-12


def test_qubit_order_invariance(oracle_lib):
    """Energies and gradients do not depend on the Jordan-Wigner ordering of
    the spin-orbitals (spin-blocked vs the paper's interleaved order)."""
    m, th, L = invariant_model()
    E1, g1 = oc.energy_grad(m, th, L)
    E2, g2 = oc.energy_grad(m.with_order(True), th, L)
    assert abs(E1 - E2) < 1e-12
    assert np.max(np.abs(g1 - g2)) < 1e-12


def test_adjoint_matches_richardson_fd(oracle_lib):
    m, th, L = invariant_model()
    _, g = oc.energy_grad(m, th, L)
    gfd = oc.fd_grad(m, th, L, h=1e-3, richardson=True)
    assert np.max(np.abs(g - gfd)) < 1e-9


def test_variational_bound_config1(oracle_lib):
    """E(th) is never below the sector ground energy."""
    m = make_model(2, 2, U=4.0)
    E0 = od.sector_ground_energy(m, 2, 2)
    rng = np.random.default_rng(4)
    for _ in range(20):
        assert oc.energy(m, rng.uniform(-np.pi, np.pi, 6), 2) >= E0 - 1e-12


def _sector_csr(m, nu, nd):
    """(nu, nd) block of H assembled from the C oracle's rows (scipy CSR)."""
    import scipy.sparse as sp
    idx = [b for b in range(1 << m.nqubits) if sector_of(m, b) == (nu, nd)]
    pos = {b: i for i, b in enumerate(idx)}
    r, c, v = [], [], []
    for i, b in enumerate(idx):
        cols, coefs = oc.ham_row(m, b)
        for col, x in zip(cols, coefs):
            r.append(i)
            c.append(pos[int(col)])   # H conserves (N_up, N_dn): no column leaves the sector
            v.append(x)
    return sp.csr_matrix((v, (r, c)), shape=(len(idx), len(idx)))


@pytest.mark.parametrize("U", [1.0, 4.0, 8.0])
def test_chain8_sector_energy_two_mechanisms(oracle_lib, U):
    """Stored 8-site chain ground energies (Kronecker-product H, Lanczos)
    against H rebuilt from the C oracle's Jordan-Wigner rows."""
    import scipy.sparse.linalg as sla
    with open(os.path.join(GOLDEN, "sector_ground_energies.json")) as f:
        E0 = json.load(f)[f"config2_chain8_U{U:g}"]["E0"]
    m = make_model(1, 8, U=U)
    H = _sector_csr(m, 4, 4)
    assert abs(H - H.T).max() < 1e-14
    w = sla.eigsh(H, k=1, which="SA", tol=1e-13)[0]
    assert abs(float(w[0]) - E0) < 1e-9


@pytest.mark.parametrize("U", [1.0, 4.0, 8.0])
def test_variational_bound_config2(oracle_lib, U):
    """8 layers of [U, even, odd] on the 8-site chain never go below the
    (4, 4) sector ground energy, at random and at small angles."""
    with open(os.path.join(GOLDEN, "sector_ground_energies.json")) as f:
        E0 = json.load(f)[f"config2_chain8_U{U:g}"]["E0"]
    m = make_model(1, 8, U=U)
    rng = np.random.default_rng(int(U) + 40)
    for width in (np.pi, 0.3):
        for _ in range(3):
            assert oc.energy(m, rng.uniform(-width, width, 24), 8) >= E0 - 1e-12


def test_golden_values(oracle_lib):
    """Stored values: closed forms (cited) and sector ground energies written by
    tests/golden/make_golden.py from the oracle's H (sparse Lanczos)."""
    with open(os.path.join(GOLDEN, "sector_ground_energies.json")) as f:
        gold = json.load(f)
    m = make_model(2, 2, U=4.0)
    assert abs(od.sector_ground_energy(m, 2, 2) - gold["config1_2x2_U4"]["E0"]) < 1e-10
    for key in ("two_site_U4", "two_site_U8"):
        U = gold[key]["U"]
        assert abs(gold[key]["E0"] - (U / 2 - np.sqrt(U * U / 4 + 4))) < 1e-12


# ---------------------------------------------------------- graph models --

GRAPH = dict(n=6, bonds=[(0, 5), (1, 2), (2, 5), (0, 3), (3, 4), (1, 4), (0, 2), (3, 5)])
GRAPH5 = dict(n=5, bonds=[(0, 4), (1, 2), (2, 4), (0, 3), (3, 4), (1, 3), (0, 2)])


def test_graph_free_fermion_spectrum(oracle_lib):
    """A non-bipartite graph with long bonds (triangles, pairs five sites apart):
    at U = V = 0 the sector spectrum is the sums of single-particle levels of
    h, which pins the Jordan-Wigner signs of arbitrary (i, j) terms."""
    from oracle.model import make_graph_model
    nb = len(GRAPH["bonds"])
    m = make_graph_model(GRAPH["n"], GRAPH["bonds"], t=1 + 0.2 * RNG.standard_normal(nb),
                         eps=RNG.uniform(-0.5, 0.5, GRAPH["n"]))
    up, dn = m.neel_sites()
    got = oracle_sector_spectrum(m, len(up), len(dn))
    want = free_sector_spectrum(m, len(up), len(dn))
    assert got.shape == want.shape
    assert np.max(np.abs(got - want)) < 1e-11


def test_graph_dense_circuit(oracle_lib):
    """Circuit energy and gradient on a graph model against the independent
    Kronecker-product construction."""
    from oracle.model import make_graph_model
    rng = np.random.default_rng(77)
    nb = len(GRAPH5["bonds"])
    m = make_graph_model(GRAPH5["n"], GRAPH5["bonds"], t=1 + 0.1 * rng.standard_normal(nb),
                         U=3.0, V=np.full(nb, 0.4), eps=rng.uniform(-0.3, 0.3, GRAPH5["n"]),
                         site_spin=[0, 0, 1, 1, 0])
    th = rng.uniform(-np.pi / 8, np.pi / 8, 2 * m.params_per_layer)
    dc = od.DenseCircuit(m)
    assert np.max(np.abs(oc.ansatz(m, th, 2) - dc.state(th, 2))) < 1e-12
    E, g = oc.energy_grad(m, th, 2)
    assert abs(E - dc.energy(th, 2)) < 1e-12 * max(1, abs(E))
    assert np.max(np.abs(g - dc.grad(th, 2))) < 1e-11


def test_graph_form_of_a_chain_is_the_chain(oracle_lib):
    from oracle.model import make_graph_model
    m = make_model(1, 6, U=4.0, V=np.full(5, 0.3))
    gm = make_graph_model(6, m.bonds, U=4.0, V=np.full(5, 0.3), groups=m.bond_class)
    assert gm.neel_index() == m.neel_index()
    th = np.random.default_rng(5).uniform(-0.3, 0.3, 2 * m.params_per_layer)
    E1, g1 = oc.energy_grad(m, th, 2)
    E2, g2 = oc.energy_grad(gm, th, 2)
    assert E1 == E2 and np.array_equal(g1, g2)


@pytest.mark.parametrize("nx,ny", [(2, 2), (1, 6), (2, 3), (1, 5)])
def test_noninteracting_bipartite_energy_vanishes(oracle_lib, nx, ny):
    """Bipartite lattice, checkerboard start, U = V = eps = 0: the sublattice
    sign change a_i -> (-1)^i a_i negates every hopping term and leaves the
    start state alone, so it maps the circuit at theta to the circuit at
    -theta and E(theta) = -E(-theta); E is also even in theta (real start
    state and H).  Hence E(theta) = 0 and grad = 0 for every theta, whatever
    the bond disorder (the VQE's U = V = 0 warm start leaves such a start
    where it is)."""
    rng = np.random.default_rng(10 * nx + ny)
    nb = len(make_model(nx, ny, U=0.0).bonds)
    m = make_model(nx, ny, U=0.0, t=1 + 0.1 * rng.standard_normal(nb))
    th = rng.uniform(-1.0, 1.0, 3 * m.params_per_layer)
    E, g = oc.energy_grad(m, th, 3)
    assert abs(E) <= 1e-13 and np.max(np.abs(g)) <= 1e-13
    # with U the same angles give a nonzero energy and gradient
    mu = make_model(nx, ny, U=2.0, t=m.t)
    Eu, gu = oc.energy_grad(mu, th, 3)
    assert abs(Eu) > 1e-3 and np.max(np.abs(gu)) > 1e-3


@pytest.mark.parametrize("nx,ny,px", [(2, 2, 0), (1, 4, 0), (2, 3, 0), (1, 6, 1)])
def test_circuit_keeps_the_start_states_total_spin_content(oracle_lib, nx, ny, px):
    """Every generator of the circuit (hopping of both spins with one t per
    bond, U n_up n_dn, V n_i n_j, eps n_i) commutes with the total spin S^2,
    so the circuit state keeps the checkerboard start's weights in each
    total-spin sector.  For N singly occupied sites with alternating spins
    the singlet weight is 1 / (N/2 + 1) (the S = 0 component of a Neel
    product state), so it bounds the fidelity of the circuit state with a
    singlet ground state.  S^2 = S^- S^+ + S_z^2 + S_z is built here from the
    Kronecker-product operators, independently of the C loops that produce
    the state; a hopping or Jordan-Wigner sign that differs between the
    spins breaks the invariance."""
    rng = np.random.default_rng(100 * nx + ny)
    nb = len(make_model(nx, ny, periodic_y=bool(px)).bonds)
    m = make_model(nx, ny, periodic_y=bool(px), U=3.0, t=1 + 0.2 * rng.standard_normal(nb),
                   V=rng.uniform(-0.5, 0.5, nb), eps=rng.uniform(-0.5, 0.5, nx * ny))
    a, ad, num = od.operators(m)
    up = [m.qubit(i, 0) for i in range(m.nsites)]
    dn = [m.qubit(i, 1) for i in range(m.nsites)]
    Sp = sum(ad[u] @ a[d] for u, d in zip(up, dn))
    Sz = 0.5 * sum(num[u] - num[d] for u, d in zip(up, dn))
    S2 = (Sp.conj().T @ Sp + Sz @ Sz + Sz).toarray()
    b0 = m.neel_index()
    nu, nd = sector_of(m, b0)
    idx = [b for b in range(1 << m.nqubits) if sector_of(m, b) == (nu, nd)]
    w, v = np.linalg.eigh(S2[np.ix_(idx, idx)])
    S = np.rint((-1.0 + np.sqrt(1.0 + 4.0 * np.clip(w, 0.0, None))) / 2.0)
    assert np.allclose(S * (S + 1.0), w, atol=1e-9)

    def weights(x):
        c = np.abs(v.conj().T @ x[idx]) ** 2
        return np.array([c[S == s].sum() for s in range(m.nsites // 2 + 1)])

    x0 = np.zeros(1 << m.nqubits, dtype=np.complex128)
    x0[b0] = 1.0
    w0 = weights(x0)
    assert abs(w0[0] - 1.0 / (m.nsites // 2 + 1)) <= 1e-12
    th = rng.uniform(-1.0, 1.0, 3 * m.params_per_layer)
    x = oc.ansatz(m, th, 3)
    assert np.max(np.abs(weights(x) - w0)) <= 1e-12
    # the ground state is a singlet: the circuit's fidelity with it is bounded
    E0, g0 = np.linalg.eigh(oc.ham_matrix(m, idx))
    assert abs(np.vdot(g0[:, 0], v[:, S == 0] @ (v[:, S == 0].conj().T @ g0[:, 0]))) >= 1 - 1e-9
    assert abs(np.vdot(g0[:, 0], x[idx])) ** 2 <= w0[0] + 1e-12
