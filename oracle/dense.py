"""Dense / sparse-matrix check of the oracle: second quantisation written out
with Kronecker products (up to ~12 qubits).

TEST INFRASTRUCTURE ONLY -- part of the oracle (see oracle/__init__.py).

This is a second, independent mechanism for the same definitions the C oracle
loops over: the Jordan-Wigner operators a_q = Z x ... x Z x sigma^- x 1 x ... x 1
are built as explicit matrices (qubit q is bit q of the index, so qubit 0 is
the LAST Kronecker factor), H of Eq. (1)/(2)/(15)/(16) and every layer
generator of Eq. (7) are assembled from them by the operator formulas, the
gates exp(-i theta G) come from an eigendecomposition, and gradients come from
forward-mode differentiation of the circuit (no adjoint recursion).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.linalg as la

from .model import OracleModel

_I2 = sp.identity(2, format="csr", dtype=np.complex128)
_Z = sp.csr_matrix(np.diag([1.0, -1.0]).astype(np.complex128))
_SM = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 0.0]], dtype=np.complex128))  # |1> -> |0>


def annihilator(n: int, q: int) -> sp.csr_matrix:
    """a_q on n qubits: Z on qubits below q, sigma^- on q, identity above."""
    op = None
    for r in range(n - 1, -1, -1):          # most significant factor first
        f = _I2 if r > q else (_SM if r == q else _Z)
        op = f if op is None else sp.kron(op, f, format="csr")
    return op


def operators(m: OracleModel):
    n = m.nqubits
    a = [annihilator(n, q) for q in range(n)]
    ad = [x.conj().T.tocsr() for x in a]
    num = [ad[q] @ a[q] for q in range(n)]
    return a, ad, num


def generators(m: OracleModel):
    """[D, H_hop,1, ..., H_hop,G] and the full H as sparse matrices."""
    a, ad, num = operators(m)
    dim = 1 << m.nqubits
    D = sp.csr_matrix((dim, dim), dtype=np.complex128)
    occ = []
    for i in range(m.nsites):
        nu, nd = num[m.qubit(i, 0)], num[m.qubit(i, 1)]
        occ.append(nu + nd)
        D = D + m.U * (nu @ nd) + m.eps[i] * (nu + nd)
    for k, (i, j) in enumerate(m.bonds):
        D = D + m.V[k] * (occ[i] @ occ[j])
    hops = [sp.csr_matrix((dim, dim), dtype=np.complex128) for _ in range(m.ngroups)]
    slots = m.bond_slot()
    for k, (i, j) in enumerate(m.bonds):
        for spin in (0, 1):
            p, q = m.qubit(i, spin), m.qubit(j, spin)
            term = -m.t[k] * (ad[p] @ a[q] + ad[q] @ a[p])
            hops[slots[k] - 1] = hops[slots[k] - 1] + term
    gens = [D] + hops
    H = D
    for h in hops:
        H = H + h
    return gens, H


class DenseCircuit:
    """Eigendecomposed generators for repeated exp(-i theta G) products."""

    def __init__(self, m: OracleModel):
        self.m = m
        gens, H = generators(m)
        self.gens = [g.toarray() for g in gens]
        self.H = H.toarray()
        self.eig = [la.eigh(g) for g in self.gens]

    def gate(self, slot: int, theta: float, psi: np.ndarray) -> np.ndarray:
        w, V = self.eig[slot]
        return V @ (np.exp(-1j * theta * w) * (V.conj().T @ psi))

    def state(self, theta, layers: int, b0=None) -> np.ndarray:
        m = self.m
        psi = np.zeros(1 << m.nqubits, dtype=np.complex128)
        psi[m.neel_index() if b0 is None else b0] = 1.0
        per = m.params_per_layer
        for k in range(layers * per):
            psi = self.gate(k % per, theta[k], psi)
        return psi

    def energy(self, theta, layers: int, b0=None) -> float:
        psi = self.state(theta, layers, b0)
        return float(np.real(np.vdot(psi, self.H @ psi)))

    def grad(self, theta, layers: int, b0=None) -> np.ndarray:
        """Forward mode: dpsi/dth_k = U_P..U_{k+1} (-i G_k) U_k..U_1 psi0 and
        dE/dth_k = 2 Re <psi|H|dpsi/dth_k>."""
        m = self.m
        per = m.params_per_layer
        P = layers * per
        psi0 = np.zeros(1 << m.nqubits, dtype=np.complex128)
        psi0[m.neel_index() if b0 is None else b0] = 1.0
        prefix = [psi0]
        for k in range(P):
            prefix.append(self.gate(k % per, theta[k], prefix[-1]))
        psi = prefix[-1]
        Hpsi = self.H @ psi
        g = np.zeros(P)
        for k in range(P):
            d = -1j * (self.gens[k % per] @ prefix[k + 1])
            for j in range(k + 1, P):
                d = self.gate(j % per, theta[j], d)
            g[k] = 2.0 * np.real(np.vdot(Hpsi, d))
        return g


def sector_states(m: OracleModel, n_up: int, n_dn: int):
    """Basis indices with n_up spin-up and n_dn spin-down electrons."""
    up_q = [m.qubit(s, 0) for s in range(m.nsites)]
    dn_q = [m.qubit(s, 1) for s in range(m.nsites)]
    out = []
    for b in range(1 << m.nqubits):
        if sum((b >> q) & 1 for q in up_q) == n_up and sum((b >> q) & 1 for q in dn_q) == n_dn:
            out.append(b)
    return out


def sector_ground_energy(m: OracleModel, n_up: int, n_dn: int) -> float:
    """Lowest eigenvalue of H in the (n_up, n_dn) sector (dense eigh)."""
    _, H = generators(m)
    idx = sector_states(m, n_up, n_dn)
    block = H[idx][:, idx].toarray()
    return float(la.eigvalsh(block)[0])


def sector_ground_state(m: OracleModel, n_up: int, n_dn: int, k: int = 1):
    """(energies, full-space states) of the k lowest sector eigenpairs, using
    sparse Lanczos (scipy eigsh) for larger sectors."""
    import scipy.sparse.linalg as sla
    _, H = generators(m)
    idx = sector_states(m, n_up, n_dn)
    block = H[idx][:, idx].tocsr()
    if block.shape[0] <= 2000:
        w, v = la.eigh(block.toarray())
        w, v = w[:k], v[:, :k]
    else:
        w, v = sla.eigsh(block, k=k, which="SA", tol=1e-13)
        order = np.argsort(w)
        w, v = w[order], v[:, order]
    full = np.zeros((1 << m.nqubits, k), dtype=np.complex128)
    full[idx, :] = v
    return w, full
