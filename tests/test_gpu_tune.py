"""Autotuner: every candidate schedule computes the same energy and gradient
(schedule invariance), and the configuration it leaves is oracle-correct."""
import numpy as np
import pytest
import torch

from oracle import core as oc
from oracle.model import make_model
from paper_2408_00836_amd import abi, tune, workloads as W
from paper_2408_00836_amd.model import Hubbard

pytestmark = pytest.mark.gpu


def test_tuner_schedules_agree(gpu, tmp_path):
    w = W.random_instance(2, 6, 3, 5, 81, U=4.0, disorder=0.1, eps_width=0.5, V=0.5)
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    th = torch.tensor(w.theta, dtype=torch.float64, device="cuda")
    ent = tune.autotune(m, th, general=True, reps=1, path=str(tmp_path / "t.json"))
    assert len(ent["table"]) >= 6
    best = abi.hubbard_get_tiles(m.handle)
    assert list(best) == ent["best"]
    om = make_model(w.nx, w.ny, **w.kwargs())
    E_ref, g_ref = oc.energy_grad(om, w.theta, w.layers)
    Es, gs = [], []
    for row in ent["table"]:
        m.set_tiles(row["fwd_k"], row["rev_k"], row["c"])
        E, g = m.energy_grad(th)
        Es.append(E.item())
        gs.append(g.cpu().numpy())
        assert abs(Es[-1] - E_ref) <= 1e-12 * max(1, abs(E_ref)), row
        assert np.max(np.abs(gs[-1] - g_ref)) <= 1e-8, row
    # different schedules sum in different orders: agree to rounding
    assert max(Es) - min(Es) <= 1e-12 * max(1, abs(E_ref))
    assert tune.lookup(m, w.layers, True, str(tmp_path / "t.json"))["best"] == list(best)
