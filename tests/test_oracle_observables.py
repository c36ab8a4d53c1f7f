"""Pins of the oracle's overlap loss (Eq. (5)/(6)) and spin correlations
(Eq. (17)) against closed forms, finite differences, the Kronecker-product
operators of oracle/dense.py and a sum rule."""
import numpy as np
import pytest

from oracle import core as oc
from oracle import dense as od
from oracle.model import make_model
from paper_2408_00836_amd import workloads as W


def rng_theta(seed, n):
    return np.random.default_rng(seed).uniform(-np.pi / 8, np.pi / 8, n)


CASES = [(2, 2, dict(U=4.0), 2),
         (2, 3, dict(U=3.0, t=1.0 + 0.1 * np.arange(7), V=np.full(7, 0.5),
                     eps=np.linspace(-0.4, 0.4, 6)), 2),
         (1, 6, dict(periodic_y=True, U=8.0), 2)]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_overlap_loss_gradient_is_the_derivative(oracle_lib, case):
    """The adjoint gradient of f = log10(1 - F) equals Richardson-extrapolated
    central differences of f."""
    nx, ny, kw, L = CASES[case]
    om = make_model(nx, ny, **kw)
    th = rng_theta(200 + case, L * om.params_per_layer)
    ref = oc.ansatz(om, rng_theta(300 + case, L * om.params_per_layer), L)
    f, F, g = oc.overlap_grad(om, th, L, ref)
    assert 0.0 < F < 1.0 and abs(f - np.log10(1.0 - F)) <= 1e-15

    def fval(x):
        return oc.overlap_grad(om, x, L, ref)[0]

    def central(h):
        out = np.zeros(th.size)
        for k in range(th.size):
            e = np.zeros(th.size)
            e[k] = h
            out[k] = (fval(th + e) - fval(th - e)) / (2 * h)
        return out

    g1, g2 = central(1e-4), central(5e-5)
    fd = (4 * g2 - g1) / 3
    assert np.max(np.abs(fd - g)) <= 1e-8


def test_overlap_loss_dense_and_basis_reference(oracle_lib):
    """F against the Kronecker-product circuit state, and for a basis-state
    reference F = |psi_b|^2."""
    om = make_model(2, 2, U=4.0)
    L = 2
    th = rng_theta(5, L * om.params_per_layer)
    dense = od.DenseCircuit(om)
    psi_d = dense.state(th, L)
    ref = oc.ansatz(om, rng_theta(6, L * om.params_per_layer), L)
    _, F, _ = oc.overlap_grad(om, th, L, ref)
    assert abs(F - abs(np.vdot(ref, psi_d)) ** 2) <= 1e-13
    b = int(np.argmax(np.abs(psi_d)))
    e_b = np.zeros(psi_d.size, dtype=np.complex128)
    e_b[b] = 1.0
    _, Fb, _ = oc.overlap_grad(om, th, L, e_b)
    assert abs(Fb - abs(psi_d[b]) ** 2) <= 1e-14


def test_spin_correlation_basis_state_and_dense_operators(oracle_lib):
    om = make_model(2, 3, U=4.0)
    L = 2
    # a basis state is a product state: no connected correlation
    C, Sz = oc.spin_correlation(om, oc.basis(om, om.neel_index()))
    up, dn = om.neel_sites()
    assert np.all(C == 0.0)
    assert all(Sz[s] == 0.5 for s in up) and all(Sz[s] == -0.5 for s in dn)
    # a circuit state against S^z_i = (n_i,up - n_i,dn)/2 built from the
    # Kronecker-product number operators
    psi = oc.ansatz(om, rng_theta(11, L * om.params_per_layer), L)
    C, Sz = oc.spin_correlation(om, psi)
    _, _, num = od.operators(om)
    S = [0.5 * (num[om.qubit(i, 0)] - num[om.qubit(i, 1)]) for i in range(om.nsites)]
    for i in range(om.nsites):
        si = np.real(np.vdot(psi, S[i] @ psi))
        assert abs(Sz[i] - si) <= 1e-14
        for j in range(om.nsites):
            sij = np.real(np.vdot(psi, S[i] @ (S[j] @ psi)))
            sj = np.real(np.vdot(psi, S[j] @ psi))
            assert abs(C[i, j] - (sij - si * sj)) <= 1e-14
    # sum rule: S^z_total is fixed in the sector, so every row sums to zero
    assert np.max(np.abs(C.sum(axis=1))) <= 1e-14


@pytest.mark.parametrize("U", [1.0, 4.0, 8.0])
def test_spin_correlation_two_site_closed_form(oracle_lib, U):
    """Two-site ground state with one up and one down electron: by
    Hellmann-Feynman the double occupancy is d = dE0/dU = 1/2 -
    (U/4)/sqrt(U^2/4 + 4t^2), and C_12 = <S^z_1 S^z_2> = -(1 - d)/4."""
    om = make_model(1, 2, U=U)
    _, vec = od.sector_ground_state(om, 1, 1, k=1)
    C, Sz = oc.spin_correlation(om, vec[:, 0])
    d = 0.5 - (U / 4) / np.sqrt(U * U / 4 + 4.0)
    assert abs(C[0, 1] - (-(1 - d) / 4)) <= 1e-13
    assert abs(C[0, 0] - (1 - d) / 4) <= 1e-13 and np.max(np.abs(Sz)) <= 1e-14
