"""Autotuner front end.  The library times the candidates on the GPU; this
module keeps the winners in a JSON cache and applies them on the product
path:

  * tile sizes (and with them the fusion schedule) per lattice:
    hubbard_tune times energy_grad for every candidate (forward k, reverse k,
    c); `Hubbard` applies the cached winner when it is built;
  * batch planning parameters per batch composition: the members' tiles
    (the library defaults, or each lattice's cached winner -- tuned for one
    instance at a time, which need not suit a batch, where the widest pass
    of a launch sets its workgroup size), work items per instance pass and
    stream lanes: autotune_batch times one batched evaluation per
    candidate; `Batch` applies the cached winner before its first call.

Cache file: $HUBVQE_TUNE_CACHE, else tune_cache.json next to this module.
Model key: lattice shape and boundaries, qubits, the diagonal's kind (U only,
or with eps/V terms, derived from the model) and the GPU name.  The layer
count is not part of the key: every layer has the same pass structure, so a
ranking timed on a few layers (the count is stored with the entry) carries
over to deeper circuits.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import torch

from . import abi

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
BATCH_ITEMS = (16, 32, 64)
BATCH_LANES = (1, 2, 3, 4)
BATCH_TILES = ("default", "lattice")
DEFAULT_TILES = (12, 12, 4)   # the library's compiled-in configuration


def cache_path() -> str:
    return os.environ.get("HUBVQE_TUNE_CACHE", DEFAULT_CACHE)


def gpu_name() -> str:
    return torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"


def model_key(model) -> str:
    kind = "gen" if model.general else "u"
    ans = "" if model.ansatz_kind == "hva" else f"/{model.ansatz_kind}"
    return (f"{model.nx}x{model.ny}/p{int(model.periodic_x)}{int(model.periodic_y)}/"
            f"q{model.n_qubits}/{kind}{ans}/{gpu_name()}")


def batch_key(models, layers) -> str:
    sig = ";".join(f"{m.nx}x{m.ny}/q{m.n_qubits}/{'gen' if m.general else 'u'}/L{L}"
                   for m, L in zip(models, layers))
    return f"batch/{len(models)}/{hashlib.sha256(sig.encode()).hexdigest()[:16]}/{gpu_name()}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, key, ent):
    data = _load(path)
    data[key] = ent
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(model, path: str | None = None):
    return _load(path or cache_path()).get(model_key(model))


def apply_cached(model, path: str | None = None):
    """Set the cached best tiles on the model; returns them, or None when the
    cache has no entry for this lattice and GPU (the library defaults stay)."""
    ent = lookup(model, path)
    if ent is None:
        return None
    model.set_tiles(*ent["best"])
    return tuple(ent["best"])


def autotune(model, theta: torch.Tensor, *, proxy_layers: int | None = None, reps: int = 2,
             path: str | None = None, save: bool = True) -> dict:
    """Time the candidate tile configurations on this GPU, leave the best on
    the model and store it."""
    per = model.params_per_layer
    lead = model.n_params(0)
    L = (theta.numel() - lead) // per
    Lt = min(L, proxy_layers) if proxy_layers else L
    th = theta[: lead + Lt * per].contiguous()
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
    model.tiles_source = "autotuned"
    ent = {"best": list(best), "timed_layers": Lt,
           "table": [dict(fwd_k=a, rev_k=b, c=c, ms=ms) for a, b, c, ms in table]}
    if save:
        _store(path or cache_path(), model_key(model), ent)
    return ent


def lookup_batch(models, layers, path: str | None = None):
    return _load(path or cache_path()).get(batch_key(models, layers))


def apply_member_tiles(models, policy: str, path: str | None = None) -> None:
    """Batch members on the library defaults or on their lattices' cached
    winners (members without an entry keep the defaults)."""
    for m in models:
        if policy == "lattice" and apply_cached(m, path) is not None:
            m.tiles_source = "tune cache"
        elif tuple(m.tiles()) != DEFAULT_TILES:
            m.set_tiles(*DEFAULT_TILES)
            m.tiles_source = "library default"


def autotune_batch(batch, theta: torch.Tensor, *, reps: int = 3, path: str | None = None,
                   save: bool = True) -> dict:
    """Time one batched evaluation per (work items, lanes) candidate (each a
    plan of its own) and store the fastest for this batch composition; the
    batch is left on it."""
    table = []
    for tiles in BATCH_TILES:
        apply_member_tiles(batch.models, tiles, path)
        for items in BATCH_ITEMS:
            for lanes in BATCH_LANES:
                batch.set_config(items, lanes, tiles)
                batch.energy_grad(theta)          # plans this configuration
                torch.cuda.synchronize()
                best = None
                for _ in range(reps):
                    t0 = time.perf_counter()
                    batch.energy_grad(theta)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                    best = dt if best is None else min(best, dt)
                table.append(dict(tiles=tiles, items=items, lanes=lanes, ms=best * 1e3))
    win = min(table, key=lambda r: r["ms"])
    apply_member_tiles(batch.models, win["tiles"], path)
    batch.set_config(win["items"], win["lanes"], win["tiles"])
    batch.config_source = "autotuned"
    ent = {"best": [win["items"], win["lanes"], win["tiles"]], "table": table}
    if save:
        _store(path or cache_path(), batch_key(batch.models, batch.layers), ent)
    return ent
