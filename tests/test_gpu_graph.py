"""Graph-form models (hubbard_create_graph) against the oracle: random graphs
with long-range and non-bipartite bonds, default and custom groups, custom
start spins, general diagonals, single- and multi-tile schedules, and the
sector form's energy and gradient on the same graphs."""
import sys

import numpy as np
import pytest
import torch

from oracle import core as oc
from oracle.model import make_graph_model
from paper_2408_00836_amd.model import Hubbard

pytestmark = pytest.mark.gpu

AMP_TOL = 1e-10
GRAD_TOL = 1e-8


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def random_graph(n, nb, seed):
    rng = np.random.default_rng(seed)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    idx = rng.choice(len(pairs), size=nb, replace=False)
    bonds = []
    for k in idx:
        i, j = pairs[k]
        bonds.append((i, j) if rng.random() < 0.5 else (j, i))   # both orientations
    return bonds, rng


CASES = [
    dict(n=6, nb=9, seed=1, U=4.0, general=False, tiles=None),
    dict(n=7, nb=10, seed=2, U=2.5, general=True, tiles=None),
    dict(n=8, nb=12, seed=3, U=6.0, general=True, tiles=(8, 7, 3)),
    dict(n=8, nb=9, seed=4, U=3.0, general=False, tiles=(6, 6, 2)),
    dict(n=9, nb=14, seed=5, U=1.5, general=True, tiles=(10, 9, 4)),
    # a different V on every bond: many V classes per diagonal op
    dict(n=8, nb=13, seed=6, U=3.5, general=True, tiles=(7, 6, 2), v_each=True),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_graph_parity(gpu, case):
    c = CASES[case]
    bonds, rng = random_graph(c["n"], c["nb"], c["seed"])
    nb = len(bonds)
    kw = dict(t=1 + 0.2 * rng.standard_normal(nb), U=c["U"])
    if c["general"]:
        V = rng.uniform(-0.6, 0.6, nb) if c.get("v_each") else np.full(nb, 0.3)
        kw.update(V=V, eps=rng.uniform(-0.5, 0.5, c["n"]))
    spins = [int(x) for x in rng.integers(0, 2, c["n"])]
    om = make_graph_model(c["n"], bonds, site_spin=spins, **kw)
    m = Hubbard.graph(c["n"], bonds, site_spin=spins, **kw)
    if c["tiles"]:
        m.set_tiles(*c["tiles"])
    assert m.params_per_layer == om.params_per_layer and m.neel_index == om.neel_index()
    L = 3
    th = rng.uniform(-np.pi / 8, np.pi / 8, L * om.params_per_layer)
    say(f"[graph] case {case}: {c['n']} sites, {nb} bonds, {om.ngroups} groups, tiles={c['tiles']}")
    tdev = torch.tensor(th, dtype=torch.float64, device=gpu)
    psi = m.ansatz(tdev)
    torch.cuda.synchronize()
    ref = oc.ansatz(om, th, L)
    assert np.max(np.abs(psi.cpu().numpy() - ref)) <= AMP_TOL
    hp = m.apply_h(psi).cpu().numpy()
    href = oc.ham_apply(om, ref)
    assert np.max(np.abs(hp - href)) <= AMP_TOL * max(1.0, np.max(np.abs(href)))
    E_ref, g_ref = oc.energy_grad(om, th, L)
    E, g = m.energy_grad(tdev)
    assert abs(E.item() - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
    assert np.max(np.abs(g.cpu().numpy() - g_ref)) <= GRAD_TOL
    assert abs(m.energy(tdev).item() - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
    # the sector form on the same graph (the start spins fix N_up, N_dn)
    Es, gs = m.sector_energy_grad(tdev)
    assert abs(Es.item() - E_ref) <= 1e-12 * max(1.0, abs(E_ref))
    assert np.max(np.abs(gs.cpu().numpy() - g_ref)) <= GRAD_TOL
