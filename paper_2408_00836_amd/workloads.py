"""Seeded synthetic workloads (inputs only -- none of the method's arithmetic).

The paper's workloads are lattice definitions, not datasets: open 1D and 2D
Hubbard clusters at half filling with U/t of 2 or 8 (Sec. 3.1, 3.2), hopping
disorder t_ij = t + d N(0,1) and on-site disorder (Sec. 3.3, Eq. (15)), and a
nearest-neighbour V (Eq. (16)).  The configurations below are synthetic
stand-ins with those shapes and distributions; every random number is drawn
here with numpy's PCG64 from a fixed seed and handed identically to the GPU
library and to the oracle.

Draw order inside one seed: t over bonds (canonical order), then eps over
sites, then (batch instances) lattice kind, U, layers, then theta
(layer-major, slot-minor).  Parameters are theta ~ U(-pi/8, pi/8).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

THETA_RANGE = np.pi / 8


def n_bonds(nx: int, ny: int, px: bool, py: bool) -> int:
    """Number of nearest-neighbour bonds (a count, used to size draws)."""
    return nx * (ny - 1 + (1 if py else 0)) + ny * (nx - 1 + (1 if px else 0))


@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    periodic_x: bool
    periodic_y: bool
    U: float
    layers: int
    params_per_layer: int          # as the configuration states it
    theta: np.ndarray
    t: Optional[np.ndarray] = None
    V: Optional[np.ndarray] = None
    eps: Optional[np.ndarray] = None

    @property
    def n_qubits(self) -> int:
        return 2 * self.nx * self.ny

    @property
    def n_params(self) -> int:
        return self.layers * self.params_per_layer

    @property
    def general(self) -> bool:
        """True when the diagonal holds V or eps terms besides U."""
        return any(a is not None and bool(np.any(np.asarray(a) != 0)) for a in (self.V, self.eps))

    def kwargs(self) -> dict:
        """Keyword arguments shared by the GPU model and the oracle model."""
        return dict(periodic_x=self.periodic_x, periodic_y=self.periodic_y, t=self.t,
                    U=self.U, V=self.V, eps=self.eps)


def _theta(rng, layers, per):
    return rng.uniform(-THETA_RANGE, THETA_RANGE, layers * per)


def config1() -> Workload:
    """2x2 open, 8 qubits, t=1, U=4, 2 layers of [U, h, v]."""
    rng = np.random.default_rng(1001)
    return Workload("2x2 open U=4 (8 qubits, 6 params)", 2, 2, False, False, 4.0, 2, 3,
                    _theta(rng, 2, 3))


def config2(U: float = 4.0) -> Workload:
    """Open chain of 8 sites, 16 qubits, 8 layers of [U, even, odd]."""
    rng = np.random.default_rng(1002)
    return Workload(f"1x8 open chain U={U:g} (16 qubits, 24 params)", 1, 8, False, False,
                    float(U), 8, 3, _theta(rng, 8, 3))


def config3() -> Workload:
    """Inhomogeneous 2x6 open ladder, 24 qubits: t = 1 + 0.1 N(0,1),
    eps ~ U(-0.5, 0.5), U = 4, V = 0.5, 12 layers x 5 params."""
    rng = np.random.default_rng(1003)
    nb = n_bonds(2, 6, False, False)
    t = 1.0 + 0.1 * rng.standard_normal(nb)
    eps = rng.uniform(-0.5, 0.5, 12)
    return Workload("2x6 open ladder, disorder, V=0.5 (24 qubits, 60 params)", 2, 6, False,
                    False, 4.0, 12, 5, _theta(rng, 12, 5), t=t, V=np.full(nb, 0.5), eps=eps)


def config5() -> Workload:
    """4x4 periodic, 32 qubits, t=1, U=8, 16 layers x 5 params."""
    rng = np.random.default_rng(1005)
    return Workload("4x4 periodic U=8 (32 qubits, 80 params)", 4, 4, True, True, 8.0, 16, 5,
                    _theta(rng, 16, 5))


# Batch instances: chains of 4..10 sites and 2x2, 2x3, 2x4, 3x3 lattices.
BATCH_KINDS = [(1, 4), (1, 5), (1, 6), (1, 7), (1, 8), (1, 9), (1, 10),
               (2, 2), (2, 3), (2, 4), (3, 3)]
# Parameters per layer the configuration states for each kind: a chain and
# the 2x2 lattice have [U, two hopping groups]; the others [U, h1, v1, h2, v2].
BATCH_PER_LAYER = {(1, L): 3 for L in range(3, 17)}
BATCH_PER_LAYER.update({(2, 2): 3, (2, 3): 5, (2, 4): 5, (3, 3): 5})


def batch_instance(i: int) -> Workload:
    """Instance i of the uneven batch: open boundaries, U ~ U(1,8),
    2..10 layers, disorder as config 3, V = 0.5 on odd instances."""
    rng = np.random.default_rng(20000 + i)
    nx, ny = BATCH_KINDS[int(rng.integers(len(BATCH_KINDS)))]
    U = float(rng.uniform(1.0, 8.0))
    layers = int(rng.integers(2, 11))
    nb = n_bonds(nx, ny, False, False)
    t = 1.0 + 0.1 * rng.standard_normal(nb)
    eps = rng.uniform(-0.5, 0.5, nx * ny)
    per = BATCH_PER_LAYER[(nx, ny)]
    V = np.full(nb, 0.5 if i % 2 else 0.0)
    return Workload(f"batch[{i}] {nx}x{ny}", nx, ny, False, False, U, layers, per,
                    _theta(rng, layers, per), t=t, V=V, eps=eps)


def batch(n: int = 256) -> list:
    return [batch_instance(i) for i in range(n)]


def random_instance(nx: int, ny: int, layers: int, per: int, seed: int, *,
                    periodic_x: bool = False, periodic_y: bool = False, U: float = 4.0,
                    disorder: float = 0.0, eps_width: float = 0.0, V: float = 0.0,
                    name: str = "") -> Workload:
    """A generic seeded instance for parity tests (same draw order)."""
    rng = np.random.default_rng(seed)
    nb = n_bonds(nx, ny, periodic_x, periodic_y)
    t = 1.0 + disorder * rng.standard_normal(nb)
    eps = rng.uniform(-eps_width, eps_width, nx * ny)
    return Workload(name or f"{nx}x{ny} seed {seed}", nx, ny, periodic_x, periodic_y, U, layers,
                    per, _theta(rng, layers, per), t=t, V=np.full(nb, V), eps=eps)


def vqe_starts(n_params: int, n_starts: int = 10, seed: int = 0) -> np.ndarray:
    """Random initial parameters of the VQE runs (Sec. 2.1): independent
    draws from a normal distribution of mean 0 and variance 1e-5, one row
    per start."""
    rng = np.random.default_rng(30000 + seed)
    return rng.normal(0.0, np.sqrt(1e-5), (n_starts, n_params))
