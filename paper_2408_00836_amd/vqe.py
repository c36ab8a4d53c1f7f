"""The VQE workflow of Sec. 2.1 on the library: for one lattice model, ten
L-BFGS optimisations from random starts N(0, 1e-5), each first run on the
non-interacting model (U = V = 0) and then continued on the interacting one
from the parameters it found; the lowest final energy is the estimate of the
ground-state energy.  The optimisations of one model run in lockstep inside
the library (hubbard_vqe: one batched energy+gradient launch per round);
this module only sequences the two stages and picks the lowest result.

    from paper_2408_00836_amd import vqe, workloads as W
    out = vqe.run(model, layers=8, n_starts=10, seed=0)
    out["E"], out["theta"], out["delta_per_site"]   # with a reference E0
"""
from __future__ import annotations

import numpy as np

from . import workloads as W


def run(model, layers: int, *, n_starts: int = 10, seed: int = 0, warm_start: bool = True,
        opts: dict | None = None, E_ref: float | None = None, sector: bool = False) -> dict:
    """Returns dict(E, theta, best, results, warm_results, delta_per_site):
    the lowest final energy, its parameters (host array), the index of that
    start, every start's result (energy, gradient norm, iterations,
    evaluations, stopping reason) and, with E_ref, (E - E_ref) / N_sites,
    the error per site of Sec. 3.1.  sector: evaluate in the particle-number
    sector form (HVA circuit; the starts run one after another)."""
    P = model.n_params(layers)
    theta0 = W.vqe_starts(P, n_starts, seed)
    warm = None
    if warm_start:
        free = model.noninteracting()
        th, warm = (free.sector_vqe if sector else free.vqe)(theta0, layers, opts)
        theta0 = th.cpu().numpy()
        del free
    th, res = (model.sector_vqe if sector else model.vqe)(theta0, layers, opts)
    th = th.cpu().numpy()
    best = int(np.argmin([r["E"] for r in res]))
    out = dict(E=res[best]["E"], theta=th[best], best=best, results=res, warm_results=warm,
               thetas=th, delta_per_site=None)
    if E_ref is not None:
        n_sites = model.n_qubits // 2
        out["delta_per_site"] = (out["E"] - E_ref) / n_sites
    return out
