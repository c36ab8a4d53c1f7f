"""Pins of the oracle's particle-number sector form (oracle/sector.py).

The sector form is what the 32-qubit golden values come from, so it is
pinned here against the full-space oracle (itself pinned to closed forms,
free-fermion spectra and dense Kronecker-product matrices in
test_oracle_pins.py), against the free-fermion Slater/Wick case, which
shares no state-vector code, and against the conservation law that
justifies it: the full-space state is exactly zero outside the sector.
"""
import numpy as np
import pytest

from oracle import core, freefermion as ff, sector
from oracle.model import make_model


def rng_theta(seed, n, scale=np.pi / 8):
    return np.random.default_rng(seed).uniform(-scale, scale, n)


CASES = [
    # (nx, ny, kwargs, layers)
    (2, 2, dict(U=4.0), 2),
    (1, 8, dict(U=8.0), 3),
    (2, 4, dict(periodic_y=True, U=3.0), 2),
    (2, 3, dict(U=4.0, t=1.0 + 0.1 * np.random.default_rng(3).standard_normal(7),
                V=np.full(7, 0.5), eps=np.random.default_rng(4).uniform(-0.5, 0.5, 6)), 3),
    (1, 6, dict(periodic_y=True, U=2.0), 3),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_sector_equals_full_space(oracle_lib, case):
    nx, ny, kw, L = CASES[case]
    om = make_model(nx, ny, **kw)
    th = rng_theta(100 + case, L * om.params_per_layer)
    full = core.ansatz(om, th, L)
    sec = sector.ansatz(om, th, L)
    idx = sector.indices(om).astype(np.int64)
    # same arithmetic per pair: identical amplitudes, and nothing outside
    assert np.array_equal(full[idx], sec)
    rest = np.ones(full.size, bool)
    rest[idx] = False
    assert np.all(full[rest] == 0.0)
    assert np.array_equal(core.ham_apply(om, full)[idx], sector.ham_apply(om, sec))
    E, g = core.energy_grad(om, th, L)
    Es, gs = sector.energy_grad(om, th, L)
    assert abs(E - Es) <= 1e-13 * max(1.0, abs(E))
    assert np.max(np.abs(g - gs)) <= 1e-13


def test_sector_positions_and_size(oracle_lib):
    from math import comb
    om = make_model(2, 3, U=1.0)
    idx = sector.indices(om)
    assert idx.size == comb(6, 3) ** 2 == sector.dim(om)
    assert np.all(np.diff(idx.astype(np.int64)) > 0)
    for i in (0, 1, 17, idx.size - 1):
        assert sector.position(om, int(idx[i])) == i
    assert sector.position(om, 0) == -1
    # every listed state has 3 up and 3 down electrons
    for b in idx:
        b = int(b)
        assert bin(b & 0x3F).count("1") == 3 and bin(b >> 6).count("1") == 3


def test_sector_free_fermion_24q(oracle_lib):
    """3x4 lattice (24 qubits): with the diagonal angles after layer 0 set to
    zero the sector state is one Slater determinant per spin; energy (Wick),
    hopping gradients and sampled amplitudes must agree."""
    om = make_model(3, 4, U=4.0)
    L = 2
    per = om.params_per_layer
    th = rng_theta(7, L * per)
    th[per::per] = 0.0
    E, g = sector.energy_grad(om, th, L)
    assert abs(E - ff.energy(om, th, L)) <= 1e-12 * max(1.0, abs(E))
    for k, v in ff.hop_gradients(om, th, L).items():
        assert abs(g[k] - v) <= 1e-10
    psi = sector.ansatz(om, th, L)
    idx = sector.indices(om)
    C = ff.orbitals(om, th, L)
    ph = ff.start_phase(om, th, L)
    pick = np.random.default_rng(8).choice(idx.size, 200, replace=False)
    want = np.array([ff.amplitude(om, C, int(idx[i]), ph) for i in pick])
    assert np.max(np.abs(psi[pick] - want)) <= 1e-12
    assert abs(np.vdot(psi, psi).real - 1.0) <= 1e-12


def test_sector_periodic_4x4_low_filling(oracle_lib):
    """The benchmark's 4x4 torus (wrap bonds with Jordan-Wigner strings
    across whole rows) in the 2-up, 2-down sector of a chosen basis state
    (14400 amplitudes): H against single rows of the full-space H, the
    symmetry E(theta) = E(-theta) with an odd gradient, the first diagonal
    angle's zero gradient, and the norm."""
    om = make_model(4, 4, periodic_x=True, periodic_y=True, U=8.0)
    b0 = (1 << 0) | (1 << 5) | (1 << (16 + 10)) | (1 << (16 + 15))
    L = 2
    th = rng_theta(9, L * om.params_per_layer)
    E1, g1 = sector.energy_grad(om, th, L, b0)
    E2, g2 = sector.energy_grad(om, -th, L, b0)
    assert abs(E1 - E2) <= 1e-12 * max(1.0, abs(E1))
    assert np.max(np.abs(g1 + g2)) <= 1e-12
    assert abs(g1[0]) <= 1e-13
    psi = sector.ansatz(om, th, L, b0)
    assert abs(np.vdot(psi, psi).real - 1.0) <= 1e-12
    phi = sector.ham_apply(om, psi, b0)
    idx = sector.indices(om, b0)
    assert idx.size == 120 ** 2
    pick = np.random.default_rng(10).choice(idx.size, 500, replace=False)
    for i in pick:
        cols, coefs = core.ham_row(om, int(idx[i]))
        pos = np.searchsorted(idx, cols)
        assert np.array_equal(idx[pos], cols)   # H keeps the sector
        assert abs(phi[i] - np.sum(coefs * psi[pos])) <= 1e-13


def test_sector_spin_correlation_equals_full_space(oracle_lib):
    om = make_model(2, 3, U=4.0, V=np.full(7, 0.3))
    th = rng_theta(21, 2 * om.params_per_layer)
    C, Sz = core.spin_correlation(om, core.ansatz(om, th, 2))
    Cs, Szs = sector.spin_correlation(om, sector.ansatz(om, th, 2), chunk=100)
    assert np.max(np.abs(C - Cs)) <= 1e-14 and np.max(np.abs(Sz - Szs)) <= 1e-14
