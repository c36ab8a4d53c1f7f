"""Pins of the oracle's NP ansatz (Eq. (8), Sec. 2.2.1): the circuit built
from explicit Kronecker-product matrices and matrix exponentials, the
reduction to the Hamiltonian-variational circuit when the parameters are
tied, finite differences, and invariants."""
import numpy as np
import pytest
import scipy.linalg as la

from oracle import core as oc
from oracle import dense as od
from oracle.model import make_model


def rng_theta(seed, n, scale=0.4):
    return np.random.default_rng(seed).uniform(-scale, scale, n)


def dense_np_state(om, theta, layers):
    """exp(i th K_pq) exp(i ph n_p n_q) per term and R_z = exp(-i th Z/2), as
    dense matrices from the Jordan-Wigner operators of oracle/dense.py."""
    a, ad, num = od.operators(om)
    n = om.nqubits
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[om.neel_index()] = 1.0
    eye = np.eye(1 << n)
    for q in range(n):
        Z = eye - 2.0 * num[q].toarray()
        psi = la.expm(-0.5j * theta[q] * Z) @ psi
    terms = oc.np_terms(om)
    k = n
    for _ in range(layers):
        for p, q in terms:
            K = (ad[p] @ a[q] + ad[q] @ a[p]).toarray()
            psi = la.expm(1j * theta[k] * K) @ psi
            psi = la.expm(1j * theta[k + 1] * (num[p] @ num[q]).toarray()) @ psi
            k += 2
    return psi


@pytest.mark.parametrize("shape", [(2, 2), (1, 4)])
def test_np_circuit_equals_dense_matrices(oracle_lib, shape):
    om = make_model(*shape, U=3.0)
    L = 2
    th = rng_theta(1, oc.np_n_params(om, L))
    assert np.max(np.abs(oc.np_ansatz(om, th, L) - dense_np_state(om, th, L))) <= 1e-12


def test_np_with_tied_parameters_is_the_hva_circuit(oracle_lib):
    """With R_z and on-site rotations off, every bond's rotation angle equal
    to its group's HVA angle times t_b, no pair phase, and every on-site
    phase equal to -theta_D U, each NP layer is the HVA layer of Eq. (7)."""
    om = make_model(2, 3, U=4.0, t=1.0 + 0.1 * np.arange(7))
    L = 2
    hva = rng_theta(2, L * om.params_per_layer)
    terms = oc.np_terms(om)
    slots = om.bond_slot()
    per = om.params_per_layer
    th = np.zeros(oc.np_n_params(om, L))
    k = om.nqubits
    for l in range(L):
        for i in range(om.nsites):                       # on-site terms
            th[k + 1] = -hva[l * per] * om.U
            k += 2
        for g in range(1, om.ngroups + 1):
            for b, ((i, j), s) in enumerate(zip(om.bonds, slots)):
                if s == g:
                    for _ in (0, 1):
                        th[k] = hva[l * per + g] * om.t[b]
                        k += 2
    assert k == th.size and len(terms) == om.nsites + 2 * len(om.bonds)
    assert np.max(np.abs(oc.np_ansatz(om, th, L) - oc.ansatz(om, hva, L))) <= 1e-13
    E, _ = oc.np_energy_grad(om, th, L)
    assert abs(E - oc.energy(om, hva, L)) <= 1e-13


def test_np_gradient_and_invariants(oracle_lib):
    om = make_model(2, 2, U=2.0)
    L = 2
    th = rng_theta(3, oc.np_n_params(om, L))
    E, g = oc.np_energy_grad(om, th, L)

    def central(h):
        out = np.zeros(th.size)
        for k in range(th.size):
            e = np.zeros(th.size)
            e[k] = h
            out[k] = (oc.np_energy_grad(om, th + e, L)[0] - oc.np_energy_grad(om, th - e, L)[0]) / (2 * h)
        return out

    fd = (4 * central(5e-5) - central(1e-4)) / 3
    assert np.max(np.abs(fd - g)) <= 1e-9
    # R_z on the basis start state is a global phase: zero gradient
    assert np.max(np.abs(g[:om.nqubits])) <= 1e-14
    E2, g2 = oc.np_energy_grad(om, -th, L)
    assert abs(E - E2) <= 1e-13 and np.max(np.abs(g + g2)) <= 1e-13
    # the on-site rotations move electrons between spins but keep their number
    psi = oc.np_ansatz(om, th, L)
    ntot = np.array([bin(b).count("1") for b in range(psi.size)])
    assert np.all(psi[ntot != 4] == 0.0)
    assert abs(np.vdot(psi, psi).real - 1.0) <= 1e-13
