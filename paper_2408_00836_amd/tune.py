"""Autotuner front end: tile sizes (and with them the fusion schedule) per
lattice, picked by measurement in the library (hubbard_tune) and cached on
disk as JSON.

Cache file: $HUBVQE_TUNE_CACHE, else tune_cache.json next to this module.
Key: lattice shape and boundaries, qubits, whether the diagonal has eps/V
terms, layers used for timing, and the GPU name.  A 32-qubit circuit is
timed with a few layers only (proxy_layers): every layer has the same pass
structure, so the ranking carries over.
"""
from __future__ import annotations

import json
import os

import torch

from . import abi

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def cache_path() -> str:
    return os.environ.get("HUBVQE_TUNE_CACHE", DEFAULT_CACHE)


def _key(model, layers: int, general: bool) -> str:
    name = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
    return (f"{model.nx}x{model.ny}/p{int(model.periodic_x)}{int(model.periodic_y)}/"
            f"q{model.n_qubits}/L{layers}/{'gen' if general else 'u'}/{name}")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(model, layers: int, general: bool, path: str | None = None):
    return _load(path or cache_path()).get(_key(model, layers, general))


def apply_cached(model, layers: int, general: bool, path: str | None = None) -> bool:
    ent = lookup(model, layers, general, path)
    if ent is None:
        return False
    model.set_tiles(*ent["best"])
    return True


def autotune(model, theta: torch.Tensor, *, general: bool, proxy_layers: int | None = None,
             reps: int = 2, path: str | None = None, save: bool = True) -> dict:
    """Time the candidate configurations on this GPU and store the best."""
    per = model.params_per_layer
    L = theta.numel() // per
    Lt = min(L, proxy_layers) if proxy_layers else L
    th = theta[: Lt * per].contiguous()
    # psi, lambda and room for the partial rows of the smallest-tile candidate
    need = abi.hubbard_workspace_size(model.handle, Lt, abi.HUBBARD_OP_ENERGY_GRAD) + (32 << 20)
    ws = next((w for w in model._ws.values() if w.numel() >= need and w.device == theta.device),
              None)
    if ws is None:
        model._ws.clear()
        torch.cuda.empty_cache()
        ws = torch.empty(need, dtype=torch.uint8, device=theta.device)
        model._ws[(Lt, abi.HUBBARD_OP_ENERGY_GRAD, str(theta.device))] = ws
    table = abi.hubbard_tune(model.handle, Lt, th.data_ptr(), ws.data_ptr(), ws.numel(),
                             torch.cuda.current_stream().cuda_stream, reps)
    best = abi.hubbard_get_tiles(model.handle)
    model.set_tiles(*best)   # the tuner leaves the winner set; drop cached sizes
    ent = {"best": list(best), "timed_layers": Lt,
           "table": [dict(fwd_k=a, rev_k=b, c=c, ms=ms) for a, b, c, ms in table]}
    if save:
        p = path or cache_path()
        data = _load(p)
        data[_key(model, L, general)] = ent
        tmp = p + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    return ent
