"""MI355X (gfx950) state-vector engine for the Hubbard Hamiltonian-variational
ansatz of Alvertis et al., "Classical Benchmarks for Variational Quantum
Eigensolver Simulations of the Hubbard Model".

The compute path is the HIP library libhubvqe.so (include/hubbard.h); this
package only marshals arguments (abi) and supplies torch device memory and
streams (model).  workloads holds the seeded synthetic inputs.
"""
from . import abi, workloads  # noqa: F401

__all__ = ["abi", "workloads", "model"]


def __getattr__(name):
    if name in ("model", "Hubbard", "EnergyGrad"):
        from . import model as _m
        return _m if name == "model" else getattr(_m, name)
    raise AttributeError(name)
