"""PyTorch-facing wrapper of the gfx950 library: device memory and streams
come from torch, every step of the path runs in the library's kernels.

    m = Hubbard(nx=2, ny=2, U=4.0)
    E = m.energy(theta)                 # theta: float64 CUDA/HIP tensor
    E, g = m.energy_grad(theta)
    E = EnergyGrad.apply(theta, m)      # differentiable, adjoint backward
"""
from __future__ import annotations

import sys

import numpy as np
import torch

from . import abi


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _require_gpu(t: torch.Tensor, name: str, dtype=None):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (the library has no CPU path)")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Hubbard:
    """One Hubbard model instance (Eq. (1)/(2)/(15)/(16)) and its HVA circuit."""

    def __init__(self, nx: int, ny: int, *, periodic_x: bool = False, periodic_y: bool = False,
                 t=None, U: float = 0.0, V=None, eps=None, groups=None, ansatz: str = "hva",
                 tuned: bool = True, _handle=None):
        """ansatz: "hva" (the Hamiltonian-variational layer of Eq. (7)) or "np"
        (the number-preserving ansatz of Eq. (8), see hubbard_set_ansatz).
        tuned: apply the autotuner's cached tile configuration for this
        lattice, ansatz and GPU when the cache has one (else the library
        defaults)."""
        self.handle = (_handle if _handle is not None else
                       abi.hubbard_create(nx, ny, periodic_x, periodic_y, t, U, V, eps, groups))
        if ansatz not in ("hva", "np"):
            raise ValueError("ansatz must be 'hva' or 'np'")
        self.ansatz_kind = ansatz
        if ansatz == "np":
            abi.hubbard_set_ansatz(self.handle, abi.HUBBARD_ANSATZ_NP)
        self._ctor = dict(nx=nx, ny=ny, periodic_x=periodic_x, periodic_y=periodic_y, t=t, U=U,
                          V=V, eps=eps, groups=groups, ansatz=ansatz)
        self.nx, self.ny = nx, ny
        self.periodic_x, self.periodic_y = bool(periodic_x), bool(periodic_y)
        # the diagonal has eps or V terms besides U (selects the general kernels)
        self.general = any(a is not None and bool(np.any(np.asarray(a, dtype=np.float64) != 0))
                           for a in (V, eps))
        q = abi.hubbard_query(self.handle)
        self.n_qubits = q["n_qubits"]
        self.n_bonds = q["n_bonds"]
        self.n_groups = q["n_groups"]
        self.params_per_layer = q["params_per_layer"]
        self.neel_index = q["neel_index"]
        self._ws = {}
        self._ws_bytes = {}   # (layers, op) -> bytes, per tile configuration
        self.tiles_gen = 0    # counts tile changes (workspace sizes depend on tiles)
        self.tiles_source = "library default"
        if tuned:
            from . import tune
            if tune.apply_cached(self) is not None:
                self.tiles_source = "tune cache"

    @classmethod
    def graph(cls, n_sites: int, bonds, *, t=None, U: float = 0.0, V=None, eps=None,
              groups=None, site_spin=None) -> "Hubbard":
        """The model on an arbitrary graph of sites (see hubbard_create_graph)."""
        h = abi.hubbard_create_graph(n_sites, bonds, t, U, V, eps, groups, site_spin)
        m = cls(1, n_sites, V=V, eps=eps, tuned=False, _handle=h)
        m._ctor = dict(graph=True, n_sites=n_sites, bonds=bonds, t=t, U=U, V=V, eps=eps,
                       groups=groups, site_spin=site_spin)
        return m

    def set_ansatz(self, ansatz: str) -> None:
        """Switch between "hva" and "np" (drops plans and cached workspaces)."""
        if ansatz not in ("hva", "np"):
            raise ValueError("ansatz must be 'hva' or 'np'")
        abi.hubbard_set_ansatz(self.handle, abi.HUBBARD_ANSATZ_NP if ansatz == "np"
                               else abi.HUBBARD_ANSATZ_HVA)
        self.ansatz_kind = ansatz
        self.params_per_layer = abi.hubbard_query(self.handle)["params_per_layer"]
        self._ctor["ansatz"] = ansatz
        self._ws.clear()
        self._ws_bytes.clear()

    def noninteracting(self) -> "Hubbard":
        """The same lattice, hoppings and on-site energies with U = V = 0 (the
        non-interacting model whose optimum starts the interacting VQE,
        Sec. 2.1)."""
        a = dict(self._ctor, U=0.0, V=None)
        if a.pop("graph", False):
            m = Hubbard.graph(**a)
            m.set_ansatz(self.ansatz_kind)
            return m
        return Hubbard(**a)

    def __del__(self):
        h = getattr(self, "handle", None)
        # at interpreter exit the process releases the device tables itself,
        # and module globals this path needs may already be gone
        if h and not sys.is_finalizing():
            try:
                torch.cuda.synchronize()
            except Exception:
                pass
            abi.hubbard_destroy(h)
            self.handle = None

    @property
    def dim(self) -> int:
        return 1 << self.n_qubits

    def n_params(self, layers: int) -> int:
        """Parameters of a circuit of `layers` layers (NP: the R_z angles first)."""
        return abi.hubbard_param_count(self.handle, layers)

    def bonds(self):
        return abi.hubbard_bonds(self.handle)

    def set_tiles(self, fwd_k: int, rev_k: int, c: int) -> None:
        abi.hubbard_set_tiles(self.handle, fwd_k, rev_k, c)
        self._ws.clear()
        self._ws_bytes.clear()
        self.tiles_gen += 1
        self.tiles_source = "set by caller"

    def tiles(self):
        """(forward k, reverse k, c) currently configured."""
        return abi.hubbard_get_tiles(self.handle)

    def workspace(self, layers: int, op: int, device=None) -> torch.Tensor:
        """Device workspace of at least hubbard_workspace_size bytes; an existing
        larger buffer of this model is reused (psi sits at its start)."""
        key = (layers, op)
        nbytes = self._ws_bytes.get(key)
        if nbytes is None:
            nbytes = self._ws_bytes[key] = abi.hubbard_workspace_size(self.handle, layers, op)
        dev = torch.device(device or "cuda")
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        for key, ws in self._ws.items():
            if ws.numel() >= nbytes and ws.device == dev and (key[1] == op or
                                                              op == abi.HUBBARD_OP_ENERGY):
                return ws
        # none fits: release this device's smaller ones first (at 32 qubits
        # two gradient workspaces do not fit in HBM together)
        for key in [k for k, w in self._ws.items() if w.device == dev]:
            del self._ws[key]
        torch.cuda.empty_cache()
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self._ws[(layers, op, str(dev))] = ws
        return ws

    def _layers(self, theta: torch.Tensor) -> int:
        _require_gpu(theta, "theta", torch.float64)
        lead = self.n_params(0)
        if theta.numel() < lead or (theta.numel() - lead) % self.params_per_layer:
            raise ValueError("theta must hold n_params(layers) values")
        return (theta.numel() - lead) // self.params_per_layer

    def new_state(self, device="cuda") -> torch.Tensor:
        psi = torch.empty(self.dim, dtype=torch.complex128, device=device)
        abi.hubbard_init_neel(self.handle, psi.data_ptr(), _stream())
        return psi

    def ansatz(self, theta: torch.Tensor, psi: torch.Tensor | None = None) -> torch.Tensor:
        L = self._layers(theta)
        if psi is None:
            psi = self.new_state(theta.device)
        _require_gpu(psi, "psi", torch.complex128)
        abi.ansatz_apply(self.handle, theta.data_ptr(), L, psi.data_ptr(), _stream())
        return psi

    def apply_h(self, psi: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        _require_gpu(psi, "psi", torch.complex128)
        if out is None:
            out = torch.empty_like(psi)
        abi.hamiltonian_apply(self.handle, psi.data_ptr(), out.data_ptr(), _stream())
        return out

    def energy(self, theta: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        L = self._layers(theta)
        ws = self.workspace(L, abi.HUBBARD_OP_ENERGY, theta.device)
        E = out if out is not None else torch.empty(1, dtype=torch.float64, device=theta.device)
        abi.energy(self.handle, theta.data_ptr(), L, E.data_ptr(), ws.data_ptr(), ws.numel(),
                   _stream())
        return E

    def energy_grad(self, theta: torch.Tensor, E: torch.Tensor | None = None,
                    grad: torch.Tensor | None = None):
        L = self._layers(theta)
        ws = self.workspace(L, abi.HUBBARD_OP_ENERGY_GRAD, theta.device)
        if E is None:
            E = torch.empty(1, dtype=torch.float64, device=theta.device)
        if grad is None:
            grad = torch.empty(theta.numel(), dtype=torch.float64, device=theta.device)
        abi.energy_grad(self.handle, theta.data_ptr(), L, E.data_ptr(), grad.data_ptr(),
                        ws.data_ptr(), ws.numel(), _stream())
        return E, grad

    def overlap(self, a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
        """<a|b> over all amplitudes (a complex128 scalar tensor on the device)."""
        for t, nm in ((a, "a"), (b, "b")):
            _require_gpu(t, nm, torch.complex128)
            if t.numel() != self.dim:
                raise ValueError(f"{nm} must hold 2^n amplitudes")
        nb = abi.hubbard_vector_workspace_size(self.handle, abi.HUBBARD_OP_OVERLAP)
        ws = torch.empty(nb, dtype=torch.uint8, device=a.device)
        out = torch.empty(2, dtype=torch.float64, device=a.device)
        abi.hubbard_overlap(self.handle, a.data_ptr(), b.data_ptr(), out.data_ptr(),
                            ws.data_ptr(), ws.numel(), _stream())
        return torch.complex(out[0], out[1])

    def overlap_grad(self, theta: torch.Tensor, ref: torch.Tensor):
        """Overlap loss of Eq. (5)/(6): (f, F, df/dtheta) with F = |<ref|psi(theta)>|^2
        and f = log10(1 - F), the gradient by the adjoint sweep."""
        L = self._layers(theta)
        _require_gpu(ref, "ref", torch.complex128)
        if ref.numel() != self.dim:
            raise ValueError("ref must hold 2^n amplitudes")
        nb = abi.hubbard_workspace_size(self.handle, L, abi.HUBBARD_OP_OVERLAP_GRAD)
        ws = torch.empty(nb, dtype=torch.uint8, device=theta.device)
        out = torch.empty(2, dtype=torch.float64, device=theta.device)
        grad = torch.empty(theta.numel(), dtype=torch.float64, device=theta.device)
        abi.overlap_grad(self.handle, theta.data_ptr(), L, ref.data_ptr(), out.data_ptr(),
                         grad.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
        return out[0], out[1], grad

    def spin_correlation(self, psi: torch.Tensor):
        """Eq. (17): (C, Sz) with C[i, j] = <Sz_i Sz_j> - <Sz_i><Sz_j>, Sz[i] = <Sz_i>."""
        _require_gpu(psi, "psi", torch.complex128)
        if psi.numel() != self.dim:
            raise ValueError("psi must hold 2^n amplitudes")
        ns = self.n_qubits // 2
        nb = abi.hubbard_vector_workspace_size(self.handle, abi.HUBBARD_OP_SPIN_CORR)
        ws = torch.empty(nb, dtype=torch.uint8, device=psi.device)
        C = torch.empty((ns, ns), dtype=torch.float64, device=psi.device)
        Sz = torch.empty(ns, dtype=torch.float64, device=psi.device)
        abi.hubbard_spin_correlation(self.handle, psi.data_ptr(), C.data_ptr(), Sz.data_ptr(),
                                     ws.data_ptr(), ws.numel(), _stream())
        return C, Sz

    def lanczos(self, start: torch.Tensor | None = None, *, max_iter: int = 400,
                tol: float = 1e-10, want_state: bool = False, seed: int = 7):
        """Ground state of H in the particle-number sector of `start` (default:
        the checkerboard state after two ansatz layers at angles drawn from
        `seed`, a generic vector of the start state's sector).  Returns
        dict(E0, iters, residual, state)."""
        if start is None:
            th = np.random.default_rng(seed).uniform(-np.pi / 8, np.pi / 8, self.n_params(2))
            start = self.ansatz(torch.tensor(th, dtype=torch.float64, device="cuda"))
        _require_gpu(start, "start", torch.complex128)
        if start.numel() != self.dim:
            raise ValueError("start must hold 2^n amplitudes")
        nb = abi.hubbard_vector_workspace_size(self.handle, abi.HUBBARD_OP_LANCZOS)
        ws = torch.empty(nb, dtype=torch.uint8, device=start.device)
        gs = torch.empty_like(start) if want_state else None
        E0, it, res = abi.hubbard_lanczos(self.handle, start.data_ptr(), max_iter, tol,
                                          gs.data_ptr() if gs is not None else None,
                                          ws.data_ptr(), ws.numel(), _stream())
        return dict(E0=E0, iters=it, residual=res, state=gs)

    def vqe(self, theta0, layers: int, opts: dict | None = None):
        """L-BFGS minimisation of E(theta) (hubbard_vqe) from each row of
        theta0 (n_starts x P); several starts run in lockstep, one batched
        evaluation per round.  Returns (final thetas on the device, results)."""
        th = torch.as_tensor(np.asarray(theta0, dtype=np.float64), device="cuda")
        th = th.reshape(-1, self.n_params(layers)).contiguous()
        n = th.shape[0]
        nb = abi.hubbard_vqe_workspace_size(self.handle, layers, n)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        res = abi.hubbard_vqe(self.handle, layers, n, th.data_ptr(), ws.data_ptr(), ws.numel(),
                              _stream(), opts)
        return th, res

    def sector_vqe(self, theta0, layers: int, opts: dict | None = None):
        """vqe() with every energy+gradient evaluation in the sector form (the
        same optimiser and stopping rules, driven from here; the starts run
        one after another).  Returns (final thetas on the device, results)."""
        th0 = np.asarray(theta0, dtype=np.float64).reshape(-1, self.n_params(layers))
        out = torch.empty(th0.shape, dtype=torch.float64, device="cuda")
        E = torch.empty(1, dtype=torch.float64, device="cuda")
        g = torch.empty(th0.shape[1], dtype=torch.float64, device="cuda")
        results = []
        for i, x0 in enumerate(th0):
            opt = abi.Lbfgs(x0, opts)
            x = opt.start
            while True:
                th = torch.as_tensor(x, device="cuda")
                self.sector_energy_grad(th, E, g)
                state, x = opt.tell(E.item(), g.cpu().numpy())
                if state != 0:
                    break
            out[i] = torch.as_tensor(x, device="cuda")
            results.append(opt.result())
        return out, results

    # ---- particle-number sector form (HVA only; see hubbard_sector_dim) ----
    def sector_dims(self):
        """(C(Ns, N_up), C(Ns, N_dn)): a sector vector holds their product,
        element r_dn * C(Ns, N_up) + r_up."""
        return abi.hubbard_sector_dim(self.handle)

    def _sector_ws(self, layers: int, op: int, device) -> torch.Tensor:
        nb = abi.hubbard_sector_workspace_size(self.handle, layers, op)
        cache = self.__dict__.setdefault("_sector_ws_cache", {})
        key = (op, str(device))
        ws = cache.get(key)
        if ws is None or ws.numel() < nb:
            cache.pop(key, None)
            torch.cuda.empty_cache()
            ws = cache[key] = torch.empty(nb, dtype=torch.uint8, device=device)
        return ws

    def release_sector_workspaces(self) -> None:
        """Drop the cached sector workspaces (device memory back to torch)."""
        self.__dict__.pop("_sector_ws_cache", None)

    def sector_state(self, theta: torch.Tensor | None = None) -> torch.Tensor:
        """psi(theta) as a sector vector (|b0> when theta is None)."""
        nu, nd = self.sector_dims()
        dev = theta.device if theta is not None else torch.device("cuda")
        psi = torch.empty(nu * nd, dtype=torch.complex128, device=dev)
        abi.hubbard_sector_init_neel(self.handle, psi.data_ptr(), _stream())
        if theta is not None:
            L = self._layers(theta)
            ws = self._sector_ws(L, abi.HUBBARD_SECTOR_ANSATZ, dev)
            abi.sector_ansatz_apply(self.handle, theta.data_ptr(), L, psi.data_ptr(),
                                    ws.data_ptr(), ws.numel(), _stream())
        return psi

    def sector_apply_h(self, psi: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        _require_gpu(psi, "psi", torch.complex128)
        if out is None:
            out = torch.empty_like(psi)
        ws = self._sector_ws(0, abi.HUBBARD_SECTOR_HAMILTONIAN, psi.device)
        abi.sector_hamiltonian_apply(self.handle, psi.data_ptr(), out.data_ptr(), ws.data_ptr(),
                                     ws.numel(), _stream())
        return out

    def sector_energy_grad(self, theta: torch.Tensor, E: torch.Tensor | None = None,
                           grad: torch.Tensor | None = None):
        """energy_grad in the sector form (same results, 1/26 of the bytes at 4x4)."""
        L = self._layers(theta)
        ws = self._sector_ws(L, abi.HUBBARD_SECTOR_ENERGY_GRAD, theta.device)
        if E is None:
            E = torch.empty(1, dtype=torch.float64, device=theta.device)
        if grad is None:
            grad = torch.empty(theta.numel(), dtype=torch.float64, device=theta.device)
        abi.sector_energy_grad(self.handle, theta.data_ptr(), L, E.data_ptr(), grad.data_ptr(),
                               ws.data_ptr(), ws.numel(), _stream())
        return E, grad

    def sector_lanczos(self, start: torch.Tensor | None = None, *, max_iter: int = 400,
                       tol: float = 1e-10, want_state: bool = False, seed: int = 7):
        """lanczos() on sector vectors: the ground state of H in the start
        state's sector (default start: the checkerboard state after two
        ansatz layers at angles drawn from `seed`).  Returns dict(E0, iters,
        residual, state) with `state` a sector vector."""
        if start is None:
            th = np.random.default_rng(seed).uniform(-np.pi / 8, np.pi / 8, self.n_params(2))
            start = self.sector_state(torch.tensor(th, dtype=torch.float64, device="cuda"))
        _require_gpu(start, "start", torch.complex128)
        nu, nd = self.sector_dims()
        if start.numel() != nu * nd:
            raise ValueError("start must hold C(Ns, N_up) * C(Ns, N_dn) amplitudes")
        ws = self._sector_ws(0, abi.HUBBARD_SECTOR_LANCZOS, start.device)
        gs = torch.empty_like(start) if want_state else None
        E0, it, res = abi.hubbard_sector_lanczos(self.handle, start.data_ptr(), max_iter, tol,
                                                 gs.data_ptr() if gs is not None else None,
                                                 ws.data_ptr(), ws.numel(), _stream())
        return dict(E0=E0, iters=it, residual=res, state=gs)

    def workspace_views(self, layers: int):
        """Two plain vector buffers carved out of the energy_grad workspace
        (scratch for ansatz/apply_h at the benchmark size; energy_grad stores
        its own psi and lambda there in a layout of its own)."""
        ws = self.workspace(layers, abi.HUBBARD_OP_ENERGY_GRAD, "cuda")
        vb = ((self.dim * 16 + 255) // 256) * 256
        psi = ws[: self.dim * 16].view(torch.complex128)
        lam = ws[vb: vb + self.dim * 16].view(torch.complex128)
        return psi, lam


class EnergyGrad(torch.autograd.Function):
    """E(theta) whose backward is the adjoint gradient computed by the forward
    call's single reverse sweep (Sec. 2.1)."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, model: Hubbard):
        E, g = model.energy_grad(theta.detach().contiguous())
        ctx.save_for_backward(g)
        return E.reshape(())

    @staticmethod
    def backward(ctx, gE):
        (g,) = ctx.saved_tensors
        return gE * g, None


class Batch:
    """Many independent instances evaluated (energy + adjoint gradient) by one
    fixed launch sequence: the instances in lanes by schedule length, each
    lane one launch per schedule position on a stream of its own (forked
    from and joined to the current stream), then one reduction.  Parameters
    of instance i live at
    theta[offsets[i] : offsets[i] + n_params[i]] of one device vector; the
    gradient uses the same layout.

        b = Batch(models, layers)
        E, g = b.energy_grad(theta)        # eager
        b.capture(theta)                   # optional: hipGraph of the launch
        E, g = b.replay()                  # reads theta in place
    """

    def __init__(self, models, layers, device="cuda", tuned: bool = True):
        """tuned: plan with the autotuner's cached (work items, lanes,
        member tiles) for this batch composition and GPU when the cache has
        them -- the members' tiles are then set as the entry says -- else
        with the library's defaults and the members as they are."""
        self.models = list(models)
        self.layers = [int(L) for L in layers]
        self.n_params = [m.n_params(L) for m, L in zip(self.models, self.layers)]
        self.offsets = np.concatenate([[0], np.cumsum(self.n_params)[:-1]]).astype(np.int64)
        self.total = int(sum(self.n_params))
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        hs = [m.handle for m in self.models]
        self.ws = None          # sized for the configuration on the first launch
        self._ws_need = {}      # (config, member tile generations) -> workspace bytes
        self.E = torch.empty(len(self.models), dtype=torch.float64, device=dev)
        self.grad = torch.empty(max(self.total, 1), dtype=torch.float64, device=dev)
        self.theta = torch.zeros(max(self.total, 1), dtype=torch.float64, device=dev)
        self.graph = None
        self.config = abi.hubbard_batch_get_config()
        self.member_tiles = "as built"
        self.config_source = "library default"
        if tuned:
            from . import tune
            ent = tune.lookup_batch(self.models, self.layers)
            if ent is not None:
                items, lanes, tiles = ent["best"]
                tune.apply_member_tiles(self.models, tiles)
                self.config = (int(items), int(lanes))
                self.member_tiles = tiles
                self.config_source = "tune cache"

    def set_config(self, items: int, lanes: int, member_tiles: str | None = None) -> None:
        """Work items per instance pass and stream lanes for this batch's plan
        (a new plan on the next call; a captured graph must be re-captured)."""
        self.config = (int(items), int(lanes))
        if member_tiles is not None:
            self.member_tiles = member_tiles
        self.config_source = "set by caller"
        self.graph = None

    def workspace(self) -> torch.Tensor:
        """Device workspace sized for the current configuration (the partial
        sums grow with the work items); sets that configuration in the
        library, which plans and keys a batch with the values current at its
        first call."""
        abi.hubbard_batch_set_config(*self.config)
        key = (self.config, tuple(m.tiles_gen for m in self.models))
        need = self._ws_need.get(key)
        if need is None:
            need = self._ws_need[key] = abi.hubbard_batch_workspace_size(
                [m.handle for m in self.models], self.layers)
        if self.ws is None or self.ws.numel() < need:
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self.ws

    def _launch(self):
        self.workspace()
        abi.energy_grad_batch([m.handle for m in self.models], self.theta.data_ptr(),
                              self.offsets, self.layers, self.E.data_ptr(),
                              self.grad.data_ptr(), self.ws.data_ptr(), self.ws.numel(),
                              _stream())

    def energy_grad(self, theta: torch.Tensor):
        _require_gpu(theta, "theta", torch.float64)
        if theta.numel() != self.total:
            raise ValueError("theta must hold every instance's parameters")
        self.theta[: self.total].copy_(theta)
        self._launch()
        return self.E, self.grad[: self.total]

    def capture(self, theta: torch.Tensor):
        """Record the batch launch in a graph (after one eager call, which
        plans and uploads the batch tables)."""
        self.energy_grad(theta)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            g.capture_begin()
            self._launch()
            g.capture_end()
        torch.cuda.current_stream().wait_stream(s)
        self.graph = g
        return g

    def replay(self, theta: torch.Tensor | None = None):
        if self.graph is None:
            raise RuntimeError("capture() first")
        if theta is not None:
            self.theta[: self.total].copy_(theta)
        self.graph.replay()
        return self.E, self.grad[: self.total]
