"""Write tests/golden/c5_4x4_periodic_U8.json: the oracle's energy, full
adjoint gradient, sampled amplitudes and spin correlations (Eq. (17)) of
the 4x4 periodic, U = 8,
16-layer (80-parameter) 32-qubit circuit at the seeded benchmark angles.

Calls only oracle/ (its particle-number sector form: the state of Eq. (3)
from the checkerboard start stays in the (8 up, 8 down) sector, 1.66e8
amplitudes) and the seeded input generator.  About 10-20 minutes on 8 host
threads and 8 GiB of memory.

    python tests/golden/make_c5_golden.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import core, sector  # noqa: E402
from oracle.model import make_model  # noqa: E402
from paper_2408_00836_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "c5_4x4_periodic_U8.json")


def sample_indices(om, rng, n):
    """Random basis states of the (8 up, 8 down) sector, spin-blocked."""
    out = []
    for _ in range(n):
        up = rng.choice(16, 8, replace=False)
        dn = rng.choice(16, 8, replace=False)
        out.append(int(sum(1 << int(s) for s in up) + sum(1 << (16 + int(s)) for s in dn)))
    return out + [om.neel_index()]


def main():
    w = W.config5()
    om = make_model(w.nx, w.ny, **w.kwargs())
    print(f"{w.name}: sector dimension {sector.dim(om)}, {core.threads()} threads", flush=True)
    t0 = time.time()
    psi = sector.ansatz(om, w.theta, w.layers)
    t1 = time.time()
    print(f"ansatz {t1 - t0:.0f} s", flush=True)
    idx = sample_indices(om, np.random.default_rng(2024), 300)
    pos = np.searchsorted(sector.indices(om), np.array(idx, dtype=np.uint64))
    amps = psi[pos]
    norm = float(np.vdot(psi, psi).real)
    C, Sz = sector.spin_correlation(om, psi)
    del psi
    E, g = sector.energy_grad(om, w.theta, w.layers)
    t2 = time.time()
    print(f"energy_grad {t2 - t1:.0f} s: E = {E!r}", flush=True)
    data = {
        "what": "oracle (sector form) energy, adjoint gradient and sampled amplitudes of "
                "the 4x4 periodic U=8 16-layer HVA circuit at the seeded benchmark angles",
        "workload": w.name,
        "theta": [float(x) for x in w.theta],
        "layers": w.layers,
        "sector_dim": sector.dim(om),
        "E": E,
        "grad": [float(x) for x in g],
        "norm": norm,
        "amp_index": idx,
        "amp_re": [float(a.real) for a in amps],
        "amp_im": [float(a.imag) for a in amps],
        "spin_corr": [[float(v) for v in row] for row in C],
        "sz": [float(v) for v in Sz],
        "oracle_threads": core.threads(),
        "oracle_seconds": {"ansatz": t1 - t0, "energy_grad": t2 - t1},
    }
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
