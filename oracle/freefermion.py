"""Free-fermion (Slater determinant) special case of the circuit.

TEST INFRASTRUCTURE ONLY -- part of the oracle (see oracle/__init__.py).

When every diagonal angle after the first layer is zero, every gate of the
Eq. (7) layer is the exponential of a one-body operator, so the circuit maps
the checkerboard start state to one Slater determinant per spin.  Its
orbitals are C = M_P ... M_1 C0 with M_k = exp(-i th_k h_k), where h_k is the
N_s x N_s hopping matrix of group k ((h_k)_ij = -t_ij on the group's bonds).
The first layer's diagonal gate only multiplies the start state (a D
eigenstate) by the phase exp(-i th D(b0)).

Everything here works with N_s x N_s matrices, so it reaches the 32-qubit
4 x 4 lattice exactly and shares nothing with a state-vector code:
  * amplitude of basis state b (spin-blocked qubit order, JW with
    a_q = Z_{<q} sigma^-_q):  det C[occ_up(b), occ_up(b0)] *
    det C[occ_dn(b), occ_dn(b0)] * exp(-i th_D1 D(b0));
  * energy by Wick's theorem from rho_ij = <a+_i a_j>;
  * hopping-parameter gradients by differentiating C exactly.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as la

from .model import OracleModel


def group_matrices(m: OracleModel):
    """h_g (N_s x N_s) for every hopping slot g = 1..G (index g-1)."""
    ns = m.nsites
    hs = [np.zeros((ns, ns)) for _ in range(m.ngroups)]
    for k, ((i, j), s) in enumerate(zip(m.bonds, m.bond_slot())):
        hs[s - 1][i, j] += -m.t[k]
        hs[s - 1][j, i] += -m.t[k]
    return hs


def one_body(m: OracleModel) -> np.ndarray:
    """Full single-particle matrix: hopping plus eps on the diagonal."""
    h = sum(group_matrices(m)) if m.ngroups else np.zeros((m.nsites, m.nsites))
    return h + np.diag(m.eps)


def _check_gaussian(m: OracleModel, theta, layers: int):
    per = m.params_per_layer
    th = np.asarray(theta, dtype=np.float64)
    for l in range(1, layers):
        if th[l * per] != 0.0:
            raise ValueError("free-fermion case needs zero diagonal angles after layer 0")
    return th


def orbital_factors(m: OracleModel, theta, layers: int):
    """The list of single-particle gates M_k in application order (hop slots)."""
    th = _check_gaussian(m, theta, layers)
    per = m.params_per_layer
    hs = group_matrices(m)
    mats = []
    for k in range(layers * per):
        s = k % per
        if s == 0:
            continue
        mats.append((k, hs[s - 1], la.expm(-1j * th[k] * hs[s - 1])))
    return mats


def orbitals(m: OracleModel, theta, layers: int) -> np.ndarray:
    C = np.eye(m.nsites, dtype=np.complex128)
    for _, _, M in orbital_factors(m, theta, layers):
        C = M @ C
    return C


def start_phase(m: OracleModel, theta, layers: int) -> complex:
    """exp(-i th_D1 D(b0)); in the checkerboard state every site holds one
    electron, so D(b0) = sum_i eps_i + sum_bonds V_b."""
    th = np.asarray(theta, dtype=np.float64)
    d0 = float(np.sum(m.eps) + np.sum(m.V))
    return complex(np.exp(-1j * th[0] * d0)) if layers > 0 else 1.0


def amplitude(m: OracleModel, C: np.ndarray, b: int, phase: complex = 1.0) -> complex:
    """Amplitude of basis index b (spin-blocked qubit order only)."""
    if m.interleaved:
        raise ValueError("determinant formula written for the spin-blocked order")
    up0, dn0 = m.neel_sites()
    ns = m.nsites
    up = [s for s in range(ns) if (b >> s) & 1]
    dn = [s for s in range(ns) if (b >> (s + ns)) & 1]
    if len(up) != len(up0) or len(dn) != len(dn0):
        return 0.0
    du = np.linalg.det(C[np.ix_(up, sorted(up0))]) if up0 else 1.0
    dd = np.linalg.det(C[np.ix_(dn, sorted(dn0))]) if dn0 else 1.0
    return complex(du * dd * phase)


def densities(m: OracleModel, C: np.ndarray):
    """rho^sigma_ij = <a+_i a_j> for both spins."""
    up0, dn0 = m.neel_sites()
    out = []
    for occ in (sorted(up0), sorted(dn0)):
        Co = C[:, occ]
        out.append(np.conj(Co) @ Co.T)
    return out


def wick_energy(m: OracleModel, rho) -> float:
    """<H> of a product of Slater determinants (one per spin)."""
    ru, rd = rho
    h = one_body(m)
    E = np.sum(h * ru) + np.sum(h * rd)
    E += m.U * np.sum(np.diag(ru) * np.diag(rd))
    for k, (i, j) in enumerate(m.bonds):
        nn = 0.0
        for ra in (ru, rd):
            for rb in (ru, rd):
                nn += ra[i, i] * rb[j, j]
        nn -= abs(ru[i, j]) ** 2 + abs(rd[i, j]) ** 2
        E += m.V[k] * nn
    return float(np.real(E))


def energy(m: OracleModel, theta, layers: int) -> float:
    return wick_energy(m, densities(m, orbitals(m, theta, layers)))


def _wick_energy_derivative(m: OracleModel, rho, drho) -> float:
    ru, rd = rho
    du, dd = drho
    h = one_body(m)
    dE = np.sum(h * du) + np.sum(h * dd)
    dE += m.U * np.sum(np.diag(du) * np.diag(rd) + np.diag(ru) * np.diag(dd))
    for k, (i, j) in enumerate(m.bonds):
        dnn = 0.0
        for ra, dra in ((ru, du), (rd, dd)):
            for rb, drb in ((ru, du), (rd, dd)):
                dnn += dra[i, i] * rb[j, j] + ra[i, i] * drb[j, j]
        for r, dr in ((ru, du), (rd, dd)):
            dnn -= 2.0 * np.real(np.conj(r[i, j]) * dr[i, j])
        dE += m.V[k] * dnn
    return float(np.real(dE))


def hop_gradients(m: OracleModel, theta, layers: int) -> dict:
    """{parameter index: dE/dth} for every hopping parameter, exactly."""
    facs = orbital_factors(m, theta, layers)
    up0, dn0 = m.neel_sites()
    C = np.eye(m.nsites, dtype=np.complex128)
    prefixes = []
    for _, _, M in facs:
        prefixes.append(C)
        C = M @ C
    rho = densities(m, C)
    grads = {}
    suffix = np.eye(m.nsites, dtype=np.complex128)
    for idx in range(len(facs) - 1, -1, -1):
        k, h, M = facs[idx]
        dC = suffix @ (-1j * h) @ M @ prefixes[idx]
        drho = []
        for occ in (sorted(up0), sorted(dn0)):
            Co, dCo = C[:, occ], dC[:, occ]
            drho.append(np.conj(dCo) @ Co.T + np.conj(Co) @ dCo.T)
        grads[k] = _wick_energy_derivative(m, rho, drho)
        suffix = suffix @ M
    return grads
