"""Writes tests/golden/sector_ground_energies.json.

Calls only the oracle (oracle.dense: Kronecker-product H, sparse Lanczos /
dense eigh in the (N_up, N_dn) sector of the checkerboard start state;
oracle.sector: the sector form of the matrix-free H, handed to scipy's
eigsh for the 24-qubit ladder) and the seeded input generator.
Run: python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle import dense as od  # noqa: E402
from oracle import sector as osec  # noqa: E402
from oracle.model import make_model  # noqa: E402
from paper_2408_00836_amd import workloads as W  # noqa: E402


def sector_ground_energy_matfree(m):
    """Lowest eigenvalue of the oracle's sector-form H (real symmetric) by
    scipy's eigsh (ARPACK), deterministic start vector."""
    import scipy.sparse.linalg as sla
    n = osec.dim(m)
    op = sla.LinearOperator((n, n), dtype=np.float64,
                            matvec=lambda x: osec.ham_apply(m, np.ravel(x).astype(np.complex128)).real)
    w = sla.eigsh(op, k=1, which="SA", tol=1e-13, v0=np.ones(n), ncv=40,
                  return_eigenvectors=False)
    return float(w[0])


def main():
    out = {
        "_note": "Sector ground energies (E0) of H in the (N_up, N_dn) sector of the "
                 "checkerboard start state; used as variational lower bounds. "
                 "two_site_*: closed form E0 = U/2 - sqrt(U^2/4 + 4t^2), t = 1, of the "
                 "two-site Hubbard model of Eq. (1) with one up and one down electron.",
    }
    for U in (4.0, 8.0):
        out[f"two_site_U{U:g}"] = dict(U=U, E0=U / 2 - np.sqrt(U * U / 4 + 4.0),
                                       source="closed form, Eq. (1) two sites")
    m = make_model(2, 2, U=4.0)
    out["config1_2x2_U4"] = dict(E0=od.sector_ground_energy(m, 2, 2), sector=[2, 2],
                                 source="oracle.dense eigh")
    for U in (1.0, 4.0, 8.0):
        m = make_model(1, 8, U=U)
        w, _ = od.sector_ground_state(m, 4, 4, k=1)
        out[f"config2_chain8_U{U:g}"] = dict(E0=float(w[0]), sector=[4, 4],
                                             source="oracle.dense Lanczos (eigsh)")
    w = W.config3()
    m = make_model(w.nx, w.ny, **w.kwargs())
    out["config3_ladder_2x6"] = dict(E0=sector_ground_energy_matfree(m), sector=[6, 6],
                                     source="oracle.sector H, scipy eigsh")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sector_ground_energies.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1, sort_keys=True))


if __name__ == "__main__":
    main()
