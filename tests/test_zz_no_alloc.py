"""energy_grad_noalloc (scratch in the library's static device array) against
energy_grad (caller workspace), through the C ABI: two calls in a row, the
second on a smaller model, each compared with energy_grad bit for bit (same
kernels, launch configuration and reduction order) and with the oracle."""
import sys

import numpy as np
import pytest
import torch

from oracle import core as oc
from oracle.model import make_model
from paper_2408_00836_amd import abi, workloads as W
from paper_2408_00836_amd.model import Hubbard

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def check(w):
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    th = torch.tensor(w.theta, dtype=torch.float64, device="cuda")
    E_ws, g_ws = m.energy_grad(th)          # uploads the plan
    E_ws, g_ws = E_ws.item(), g_ws.cpu().numpy()
    E = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    g = torch.full((th.numel(),), np.nan, dtype=torch.float64, device="cuda")
    say(f"[noalloc] {w.name}")
    abi.energy_grad_noalloc(m.handle, th.data_ptr(), w.layers, E.data_ptr(), g.data_ptr(),
                            torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    E, g = E.item(), g.cpu().numpy()
    assert E == E_ws and np.array_equal(g, g_ws)
    E_ref, g_ref = oc.energy_grad(make_model(w.nx, w.ny, **w.kwargs()), w.theta, w.layers)
    assert abs(E - E_ref) <= 1e-12 * max(1, abs(E_ref))
    assert np.max(np.abs(g - g_ref)) <= 1e-8
    return m


def test_noalloc_matches_energy_grad_twice(gpu):
    # 16 qubits, then 8: the second call leaves the first's contents behind
    m1 = check(W.config2(4.0))
    m2 = check(W.config1())
    del m1, m2


def test_noalloc_errors(gpu):
    w = W.config1()
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    th = torch.tensor(w.theta, dtype=torch.float64, device="cuda")
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.zeros(th.numel(), dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    with pytest.raises(abi.HubbardError) as ei:   # nothing uploaded yet
        abi.energy_grad_noalloc(m.handle, th.data_ptr(), w.layers, E.data_ptr(), g.data_ptr(), s)
    assert ei.value.status == abi.HUBBARD_ERR_STATE
    big = Hubbard(3, 4, U=4.0)                    # 24 qubits: beyond the scratch
    with pytest.raises(abi.HubbardError) as ei:
        abi.energy_grad_noalloc(big.handle, th.data_ptr(), 1, E.data_ptr(), g.data_ptr(), s)
    assert ei.value.status == abi.HUBBARD_ERR_SIZE
