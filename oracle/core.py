"""ctypes wrapper of the plain C oracle (oracle/hubbard_oracle.c).

TEST INFRASTRUCTURE ONLY -- part of the oracle (see oracle/__init__.py).

The C file is compiled with gcc into oracle/liboracle.so (build() below, also
run by the project's build step).  All vectors are numpy complex128 arrays of
2^n amplitudes; bit q of the index is the occupation of qubit q.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .model import OracleModel

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hubbard_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MAX_SITES = 32
MAX_BONDS = 128


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fcx-fortran-rules", "-fno-fast-math",
               "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Model(ctypes.Structure):
    _fields_ = [
        ("nsites", ctypes.c_int32),
        ("nbonds", ctypes.c_int32),
        ("interleaved", ctypes.c_int32),
        ("ngroups", ctypes.c_int32),
        ("bond_i", ctypes.c_int32 * MAX_BONDS),
        ("bond_j", ctypes.c_int32 * MAX_BONDS),
        ("bond_slot", ctypes.c_int32 * MAX_BONDS),
        ("t", ctypes.c_double * MAX_BONDS),
        ("V", ctypes.c_double * MAX_BONDS),
        ("eps", ctypes.c_double * MAX_SITES),
        ("U", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        cd, cu64, ci = ctypes.c_double, ctypes.c_uint64, ctypes.c_int
        vp = ctypes.c_void_p
        L.orc_init_basis.argtypes = [P(_Model), cu64, vp]
        L.orc_apply_slot.argtypes = [P(_Model), ci, cd, vp]
        L.orc_generator_apply.argtypes = [P(_Model), ci, vp, vp]
        L.orc_ham_apply.argtypes = [P(_Model), vp, vp]
        L.orc_ham_row.argtypes = [P(_Model), cu64, vp, vp]
        L.orc_ham_row.restype = ci
        L.orc_inner.argtypes = [ci, vp, vp, P(cd), P(cd)]
        L.orc_ansatz.argtypes = [P(_Model), vp, ci, cu64, vp]
        L.orc_expectation.argtypes = [P(_Model), vp, vp]
        L.orc_expectation.restype = cd
        L.orc_energy.argtypes = [P(_Model), vp, ci, cu64, P(cd)]
        L.orc_energy.restype = ci
        L.orc_energy_grad.argtypes = [P(_Model), vp, ci, cu64, P(cd), vp]
        L.orc_energy_grad.restype = ci
        L.orc_threads.restype = ci
        L.orc_overlap_grad.argtypes = [P(_Model), vp, ci, cu64, vp, vp, vp]
        L.orc_overlap_grad.restype = ci
        L.orc_spin_correlation.argtypes = [P(_Model), vp, vp, vp]
        L.orc_np_ansatz.argtypes = [P(_Model), ci, vp, vp, vp, ci, cu64, vp]
        L.orc_np_energy_grad.argtypes = [P(_Model), ci, vp, vp, vp, ci, cu64, P(cd), vp]
        L.orc_np_energy_grad.restype = ci
        L.orc_set_threads.argtypes = [ci]
        _lib = L
    return _lib


def _cmodel(m: OracleModel) -> _Model:
    if m.nsites > MAX_SITES or len(m.bonds) > MAX_BONDS:
        raise ValueError("model too large for the oracle")
    c = _Model()
    c.nsites = m.nsites
    c.nbonds = len(m.bonds)
    c.interleaved = 1 if m.interleaved else 0
    c.ngroups = m.ngroups
    slots = m.bond_slot()
    for k, (i, j) in enumerate(m.bonds):
        c.bond_i[k] = i
        c.bond_j[k] = j
        c.bond_slot[k] = slots[k]
        c.t[k] = float(m.t[k])
        c.V[k] = float(m.V[k])
    for s in range(m.nsites):
        c.eps[s] = float(m.eps[s])
    c.U = float(m.U)
    return c


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _vec(m: OracleModel) -> np.ndarray:
    return np.zeros(1 << m.nqubits, dtype=np.complex128)


def threads() -> int:
    return lib().orc_threads()


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def basis(m: OracleModel, b0: int) -> np.ndarray:
    psi = _vec(m)
    lib().orc_init_basis(ctypes.byref(_cmodel(m)), b0, _ptr(psi))
    return psi


def apply_slot(m: OracleModel, slot: int, theta: float, psi: np.ndarray) -> np.ndarray:
    """In place: psi <- exp(-i theta G_slot) psi (slot 0 = diagonal)."""
    lib().orc_apply_slot(ctypes.byref(_cmodel(m)), slot, float(theta), _ptr(psi))
    return psi


def generator_apply(m: OracleModel, slot: int, psi: np.ndarray) -> np.ndarray:
    out = _vec(m)
    lib().orc_generator_apply(ctypes.byref(_cmodel(m)), slot, _ptr(psi), _ptr(out))
    return out


def ham_apply(m: OracleModel, psi: np.ndarray) -> np.ndarray:
    out = _vec(m)
    lib().orc_ham_apply(ctypes.byref(_cmodel(m)), _ptr(np.ascontiguousarray(psi)), _ptr(out))
    return out


def ham_row(m: OracleModel, b: int):
    """Row b of H as (columns, coefficients): (H psi)_b = sum coef * psi[col].
    Works at any size (32 qubits included): it touches only the row."""
    cm = _cmodel(m)
    cap = 1 + 2 * len(m.bonds)
    cols = np.zeros(cap, dtype=np.uint64)
    coefs = np.zeros(cap, dtype=np.float64)
    k = lib().orc_ham_row(ctypes.byref(cm), int(b), _ptr(cols), _ptr(coefs))
    return cols[:k], coefs[:k]


def inner(a: np.ndarray, b: np.ndarray) -> complex:
    n = int(a.size).bit_length() - 1
    re, im = ctypes.c_double(), ctypes.c_double()
    lib().orc_inner(n, _ptr(a), _ptr(b), ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def ansatz(m: OracleModel, theta, layers: int, b0: int | None = None) -> np.ndarray:
    th = np.ascontiguousarray(theta, dtype=np.float64)
    if th.size != layers * m.params_per_layer:
        raise ValueError("theta must hold layers * params_per_layer values")
    psi = _vec(m)
    b0 = m.neel_index() if b0 is None else b0
    lib().orc_ansatz(ctypes.byref(_cmodel(m)), _ptr(th), layers, b0, _ptr(psi))
    return psi


def expectation(m: OracleModel, psi: np.ndarray) -> float:
    scratch = _vec(m)
    return lib().orc_expectation(ctypes.byref(_cmodel(m)), _ptr(np.ascontiguousarray(psi)),
                                 _ptr(scratch))


def energy(m: OracleModel, theta, layers: int, b0: int | None = None) -> float:
    th = np.ascontiguousarray(theta, dtype=np.float64)
    if th.size != layers * m.params_per_layer:
        raise ValueError("theta must hold layers * params_per_layer values")
    E = ctypes.c_double()
    b0 = m.neel_index() if b0 is None else b0
    if lib().orc_energy(ctypes.byref(_cmodel(m)), _ptr(th), layers, b0, ctypes.byref(E)):
        raise MemoryError("oracle energy: allocation failed")
    return E.value


def energy_grad(m: OracleModel, theta, layers: int, b0: int | None = None):
    """(E, grad) by the adjoint recursion."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    if th.size != layers * m.params_per_layer:
        raise ValueError("theta must hold layers * params_per_layer values")
    g = np.zeros(th.size)
    E = ctypes.c_double()
    b0 = m.neel_index() if b0 is None else b0
    if lib().orc_energy_grad(ctypes.byref(_cmodel(m)), _ptr(th), layers, b0,
                             ctypes.byref(E), _ptr(g)):
        raise MemoryError("oracle energy_grad: allocation failed")
    return E.value, g


def fd_grad(m: OracleModel, theta, layers: int, h: float = 1e-5, richardson: bool = False,
            b0: int | None = None) -> np.ndarray:
    """Central finite differences of the oracle energy; with richardson=True
    the (h, h/2) pair is combined to cancel the h^2 term."""
    th = np.asarray(theta, dtype=np.float64)

    def central(step):
        g = np.zeros(th.size)
        for k in range(th.size):
            tp, tm = th.copy(), th.copy()
            tp[k] += step
            tm[k] -= step
            g[k] = (energy(m, tp, layers, b0) - energy(m, tm, layers, b0)) / (2 * step)
        return g

    g1 = central(h)
    if not richardson:
        return g1
    g2 = central(h / 2)
    return (4 * g2 - g1) / 3


def ham_matrix(m: OracleModel, basis_states) -> np.ndarray:
    """Dense block <b'|H|b> over the given basis indices, built by applying the
    oracle's matrix-free H to each basis vector (small systems only)."""
    idx = list(basis_states)
    pos = {b: k for k, b in enumerate(idx)}
    Hm = np.zeros((len(idx), len(idx)), dtype=np.complex128)
    for k, b in enumerate(idx):
        col = ham_apply(m, basis(m, b))
        nz = np.nonzero(col)[0]
        for r in nz:
            if int(r) not in pos:
                raise ValueError("basis set is not closed under H")
            Hm[pos[int(r)], k] = col[r]
    return Hm


def overlap_grad(m: OracleModel, theta, layers: int, ref: np.ndarray, b0: int | None = None):
    """(f, F, df/dtheta): f = log10(1 - F), F = |<ref|psi(theta)>|^2 (Eq. (5)/(6))."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    ref = np.ascontiguousarray(ref, dtype=np.complex128)
    if ref.size != 1 << m.nqubits:
        raise ValueError("ref must hold 2^n amplitudes")
    out = np.zeros(2)
    g = np.zeros(th.size)
    b0 = m.neel_index() if b0 is None else b0
    if lib().orc_overlap_grad(ctypes.byref(_cmodel(m)), _ptr(th), layers, b0, _ptr(ref),
                              _ptr(out), _ptr(g)):
        raise MemoryError("oracle overlap_grad: allocation failed")
    return out[0], out[1], g


def spin_correlation(m: OracleModel, psi: np.ndarray):
    """(C, Sz): C[i, j] = <S^z_i S^z_j> - <S^z_i><S^z_j> (Eq. (17)), Sz[i] = <S^z_i>."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    C = np.zeros((m.nsites, m.nsites))
    Sz = np.zeros(m.nsites)
    lib().orc_spin_correlation(ctypes.byref(_cmodel(m)), _ptr(psi), _ptr(C), _ptr(Sz))
    return C, Sz


def np_terms(m: OracleModel):
    """Qubit pairs of one NP layer in application order (Sec. 2.2.1): the
    two spin qubits of every site, then each hopping group's bonds (group
    order, bond order), spin up then spin down."""
    terms = [(m.qubit(i, 0), m.qubit(i, 1)) for i in range(m.nsites)]
    slots = m.bond_slot()
    for g in range(1, m.ngroups + 1):
        for (i, j), s in zip(m.bonds, slots):
            if s == g:
                for spin in (0, 1):
                    a, b = m.qubit(i, spin), m.qubit(j, spin)
                    terms.append((min(a, b), max(a, b)))
    return terms


def np_n_params(m: OracleModel, layers: int) -> int:
    return m.nqubits + 2 * len(np_terms(m)) * layers


def _np_args(m):
    t = np_terms(m)
    pp = np.ascontiguousarray([a for a, _ in t], dtype=np.int32)
    qq = np.ascontiguousarray([b for _, b in t], dtype=np.int32)
    return len(t), pp, qq


def np_ansatz(m: OracleModel, theta, layers: int, b0: int | None = None) -> np.ndarray:
    """State of the NP circuit (R_z layer included, exact R_z)."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    nt, pp, qq = _np_args(m)
    if th.size != m.nqubits + 2 * nt * layers:
        raise ValueError("theta must hold n_qubits + 2 * terms * layers values")
    psi = _vec(m)
    b0 = m.neel_index() if b0 is None else b0
    lib().orc_np_ansatz(ctypes.byref(_cmodel(m)), nt, _ptr(pp), _ptr(qq), _ptr(th), layers, b0,
                        _ptr(psi))
    return psi


def np_energy_grad(m: OracleModel, theta, layers: int, b0: int | None = None):
    th = np.ascontiguousarray(theta, dtype=np.float64)
    nt, pp, qq = _np_args(m)
    if th.size != m.nqubits + 2 * nt * layers:
        raise ValueError("theta must hold n_qubits + 2 * terms * layers values")
    g = np.zeros(th.size)
    E = ctypes.c_double()
    b0 = m.neel_index() if b0 is None else b0
    if lib().orc_np_energy_grad(ctypes.byref(_cmodel(m)), nt, _ptr(pp), _ptr(qq), _ptr(th),
                                layers, b0, ctypes.byref(E), _ptr(g)):
        raise MemoryError("oracle np_energy_grad: allocation failed")
    return E.value, g
