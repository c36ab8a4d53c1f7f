"""Lifetime of planned batches (energy_grad_batch): a batch is keyed by its
members' identities and tile configurations, never by reused addresses, and
re-tiling, tuning or destroying a member discards it.  Runs the fixed code:
re-tile a member, then destroy and recreate models over the same theta and
workspace buffers, and check every result against the oracle."""
import gc
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


def run(models, wl, theta, ws, E, G):
    offs = np.concatenate([[0], np.cumsum([w.n_params for w in wl])[:-1]]).astype(np.int64)
    th = np.concatenate([w.theta for w in wl])
    theta[: th.size].copy_(torch.tensor(th, dtype=torch.float64))
    abi.energy_grad_batch([m.handle for m in models], theta.data_ptr(), offs,
                          [w.layers for w in wl], E.data_ptr(), G.data_ptr(), ws.data_ptr(),
                          ws.numel(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    e, g = E.cpu().numpy(), G.cpu().numpy()
    for i, w in enumerate(wl):
        om = make_model(w.nx, w.ny, **w.kwargs())
        E_ref, g_ref = oc.energy_grad(om, w.theta, w.layers)
        assert abs(e[i] - E_ref) <= 1e-12 * max(1, abs(E_ref)), (i, e[i], E_ref)
        o = offs[i]
        assert np.max(np.abs(g[o:o + w.n_params] - g_ref)) <= 1e-8, i


def with_U(w, U):
    w2 = W.Workload(w.name, w.nx, w.ny, w.periodic_x, w.periodic_y, U, w.layers,
                    w.params_per_layer, w.theta, w.t, w.V, w.eps)
    return w2


def test_batch_cache_retile_and_recreate(gpu):
    wl = [W.batch_instance(i) for i in range(6)]
    wl = [w for w in wl if w.n_qubits <= 16][:4]
    assert len(wl) >= 2
    theta = torch.zeros(4096, dtype=torch.float64, device="cuda")
    E = torch.zeros(len(wl), dtype=torch.float64, device="cuda")
    G = torch.zeros(4096, dtype=torch.float64, device="cuda")
    models = [Hubbard(w.nx, w.ny, **w.kwargs()) for w in wl]
    need = abi.hubbard_batch_workspace_size([m.handle for m in models], [w.layers for w in wl])
    ws = torch.empty(4 * need, dtype=torch.uint8, device="cuda")
    gc.collect()   # models of earlier tests: their batches go now, not mid-test
    n0 = abi.hubbard_batch_cached()
    say(f"[batch cache] plan a batch of {len(wl)} instances")
    run(models, wl, theta, ws, E, G)
    assert abi.hubbard_batch_cached() == n0 + 1
    run(models, wl, theta, ws, E, G)          # cached plan reused
    assert abi.hubbard_batch_cached() == n0 + 1
    say("[batch cache] re-tile one member")
    models[0].set_tiles(4, 4, 2)
    assert abi.hubbard_batch_cached() == n0
    run(models, wl, theta, ws, E, G)          # planned again with the new tiles
    assert abi.hubbard_batch_cached() == n0 + 1
    say("[batch cache] destroy, recreate other models over the same buffers")
    del models
    gc.collect()
    assert abi.hubbard_batch_cached() == n0
    wl2 = [with_U(w, w.U + 1.75) for w in wl]
    models2 = [Hubbard(w.nx, w.ny, **w.kwargs()) for w in wl2]
    run(models2, wl2, theta, ws, E, G)
    assert abi.hubbard_batch_cached() == n0 + 1
    del models2
    gc.collect()


def test_batch_cache_is_bounded(gpu):
    w = W.config1()
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    theta = torch.tensor(np.tile(w.theta, 40), dtype=torch.float64, device="cuda")
    need = abi.hubbard_batch_workspace_size([m.handle], [w.layers])
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    G = torch.zeros(theta.numel(), dtype=torch.float64, device="cuda")
    E_ref, g_ref = oc.energy_grad(make_model(w.nx, w.ny, **w.kwargs()), w.theta, w.layers)
    s = torch.cuda.current_stream().cuda_stream
    for k in range(20):   # 20 distinct signatures (parameter offsets)
        off = k * w.n_params
        abi.energy_grad_batch([m.handle], theta.data_ptr(), [off], [w.layers], E.data_ptr(),
                              G.data_ptr(), ws.data_ptr(), ws.numel(), s)
        torch.cuda.synchronize()
        assert abi.hubbard_batch_cached() <= 16
        assert abs(E.item() - E_ref) <= 1e-12 * max(1, abs(E_ref))
        assert np.max(np.abs(G[off:off + w.n_params].cpu().numpy() - g_ref)) <= 1e-8
    del m
    gc.collect()
