"""Sector form of the oracle: the circuit, H and the adjoint gradient on the
amplitudes of one (N_up, N_dn) particle-number sector only.

TEST INFRASTRUCTURE ONLY -- part of the oracle (see oracle/__init__.py).

Every gate of the Eq. (7) layer and H itself conserve the numbers of spin-up
and spin-down electrons, so the state prepared from the checkerboard start
|b0> (Sec. 2.1) lives in b0's sector; outside it every amplitude is exactly
zero.  Keeping only the sector (C(16,8)^2 = 1.66e8 amplitudes, 2.6 GiB, at
4x4 half filling instead of 2^32, 64 GiB) lets the oracle compute the full
32-qubit energy, gradient and amplitudes at any theta on an ordinary host.
The arithmetic per amplitude pair is that of the full-space oracle, so the
sector amplitudes equal the full-space ones bit for bit (a pinned property).

Spin-blocked qubit order only.  Sector position i holds the full index
sector_indices(m, b0)[i].
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import core
from .model import OracleModel

_ready = False


def _lib():
    global _ready
    L = core.lib()
    if not _ready:
        P = ctypes.POINTER
        vp, cu64, ci = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
        M = P(core._Model)
        L.orc_sector_dim.argtypes = [M, cu64]
        L.orc_sector_dim.restype = ctypes.c_int64
        L.orc_sector_indices.argtypes = [M, cu64, vp]
        L.orc_sector_indices.restype = ci
        L.orc_sector_ansatz.argtypes = [M, vp, ci, cu64, vp]
        L.orc_sector_ansatz.restype = ci
        L.orc_sector_ham_apply.argtypes = [M, cu64, vp, vp]
        L.orc_sector_ham_apply.restype = ci
        L.orc_sector_energy_grad.argtypes = [M, vp, ci, cu64, P(ctypes.c_double), vp]
        L.orc_sector_energy_grad.restype = ci
        _ready = True
    return L


def _b0(m: OracleModel, b0):
    if m.interleaved:
        raise ValueError("the sector form uses the spin-blocked qubit order")
    return m.neel_index() if b0 is None else int(b0)


def dim(m: OracleModel, b0: int | None = None) -> int:
    return int(_lib().orc_sector_dim(ctypes.byref(core._cmodel(m)), _b0(m, b0)))


def indices(m: OracleModel, b0: int | None = None) -> np.ndarray:
    """Full amplitude index of each sector position (uint64)."""
    b0 = _b0(m, b0)
    out = np.zeros(dim(m, b0), dtype=np.uint64)
    if _lib().orc_sector_indices(ctypes.byref(core._cmodel(m)), b0, core._ptr(out)):
        raise MemoryError("sector indices")
    return out


def position(m: OracleModel, b: int) -> int:
    """Sector position of full index b (-1 outside the sector of the start
    state): rank of the down pattern times the up-pattern count plus the
    rank of the up pattern, ranks among patterns of the same popcount."""
    ns = m.nsites
    up, dn = b & ((1 << ns) - 1), b >> ns
    nu, nd = (bin(x).count("1") for x in (m.neel_index() & ((1 << ns) - 1),
                                          m.neel_index() >> ns))
    if bin(up).count("1") != nu or bin(dn).count("1") != nd:
        return -1

    def rank(pat, k):   # patterns below pat with k bits, by brute force
        return sum(1 for v in range(pat) if bin(v).count("1") == k)

    from math import comb
    return rank(dn, nd) * comb(ns, nu) + rank(up, nu)


def ansatz(m: OracleModel, theta, layers: int, b0: int | None = None) -> np.ndarray:
    b0 = _b0(m, b0)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    if th.size != layers * m.params_per_layer:
        raise ValueError("theta must hold layers * params_per_layer values")
    psi = np.zeros(dim(m, b0), dtype=np.complex128)
    if _lib().orc_sector_ansatz(ctypes.byref(core._cmodel(m)), core._ptr(th), layers, b0,
                                core._ptr(psi)):
        raise MemoryError("sector ansatz")
    return psi


def ham_apply(m: OracleModel, psi: np.ndarray, b0: int | None = None) -> np.ndarray:
    b0 = _b0(m, b0)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.zeros_like(psi)
    if _lib().orc_sector_ham_apply(ctypes.byref(core._cmodel(m)), b0, core._ptr(psi),
                                   core._ptr(out)):
        raise MemoryError("sector H")
    return out


def energy_grad(m: OracleModel, theta, layers: int, b0: int | None = None, grad: bool = True):
    """(E, gradient) by the adjoint recursion on the sector (gradient None
    when grad=False)."""
    b0 = _b0(m, b0)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    if th.size != layers * m.params_per_layer:
        raise ValueError("theta must hold layers * params_per_layer values")
    g = np.zeros(th.size) if grad else None
    E = ctypes.c_double()
    if _lib().orc_sector_energy_grad(ctypes.byref(core._cmodel(m)), core._ptr(th), layers, b0,
                                     ctypes.byref(E), core._ptr(g) if grad else None):
        raise MemoryError("sector energy_grad")
    return E.value, g


def spin_correlation(m: OracleModel, psi: np.ndarray, b0: int | None = None, chunk: int = 1 << 22):
    """(C, Sz) of Eq. (17) from a sector vector: C[i, j] = <Sz_i Sz_j> -
    <Sz_i><Sz_j>, Sz_i = (n_i,up - n_i,dn)/2, each expectation summed over the
    sector's amplitudes (|psi_x|^2 times the operator's value at x), in
    chunks."""
    b0 = _b0(m, b0)
    idx = indices(m, b0)
    ns = m.nsites
    ss = np.zeros((ns, ns))
    s1 = np.zeros(ns)
    for a in range(0, idx.size, chunk):
        x = idx[a:a + chunk]
        p = np.abs(psi[a:a + chunk]) ** 2
        sz = np.empty((x.size, ns))
        for i in range(ns):
            up = ((x >> np.uint64(m.qubit(i, 0))) & np.uint64(1)).astype(np.float64)
            dn = ((x >> np.uint64(m.qubit(i, 1))) & np.uint64(1)).astype(np.float64)
            sz[:, i] = 0.5 * (up - dn)
        ss += (sz * p[:, None]).T @ sz
        s1 += p @ sz
    return ss - np.outer(s1, s1), s1
