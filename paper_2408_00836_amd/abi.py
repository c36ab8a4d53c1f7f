"""ctypes binding of include/hubbard.h (argument marshalling only).

Every function here has the name of the C entry point it calls and takes
plain integers for device pointers and streams.  All computation happens in
the gfx950 library libhubvqe.so; if it is missing, loading fails loudly --
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhubvqe.so")

HUBBARD_OK = 0
HUBBARD_ERR_ARG = 1
HUBBARD_ERR_SIZE = 2
HUBBARD_ERR_DEVICE = 3
HUBBARD_ERR_NOMEM = 4
HUBBARD_ERR_STATE = 5
HUBBARD_OP_ENERGY = 0
HUBBARD_OP_ENERGY_GRAD = 1
HUBBARD_OP_OVERLAP = 2
HUBBARD_OP_LANCZOS = 3
HUBBARD_OP_OVERLAP_GRAD = 4
HUBBARD_OP_SPIN_CORR = 5
HUBBARD_ANSATZ_HVA = 0
HUBBARD_ANSATZ_NP = 1
HUBBARD_SECTOR_ANSATZ = 0
HUBBARD_SECTOR_ENERGY_GRAD = 1
HUBBARD_SECTOR_HAMILTONIAN = 2
HUBBARD_SECTOR_LANCZOS = 3

# Every symbol the headers in include/ declare.
EXPORTED = [
    "hubbard_create", "hubbard_create_graph", "hubbard_destroy", "hubbard_query", "hubbard_bonds",
    "hubbard_last_error", "hubbard_workspace_size", "hubbard_init_neel",
    "ansatz_apply", "hamiltonian_apply", "energy", "energy_grad",
    "hubbard_plan_dump", "hubbard_set_tiles", "hubbard_set_timing", "hubbard_phase_ms",
    "hubbard_kernel_ms",
    "hubbard_batch_workspace_size", "energy_grad_batch", "hubbard_get_tiles", "hubbard_tune",
    "hubbard_batch_cached", "hubbard_batch_set_config", "hubbard_batch_get_config",
    "energy_grad_noalloc", "hubbard_vector_workspace_size", "hubbard_overlap", "hubbard_lanczos",
    "hubbard_tridiag_lowest", "hubbard_vqe_workspace_size", "hubbard_vqe", "hubbard_lbfgs_create",
    "hubbard_lbfgs_tell", "hubbard_lbfgs_result", "hubbard_lbfgs_destroy", "overlap_grad",
    "hubbard_spin_correlation", "hubbard_set_ansatz", "hubbard_param_count",
    "hubbard_sector_dim", "hubbard_sector_workspace_size", "hubbard_sector_init_neel",
    "sector_ansatz_apply", "sector_hamiltonian_apply", "sector_energy_grad",
    "hubbard_sector_lanczos",
]


class hubbard_vqe_opts(ctypes.Structure):
    _fields_ = [("max_steps", ctypes.c_int32), ("history", ctypes.c_int32),
                ("e_tol", ctypes.c_double), ("g_tol", ctypes.c_double)]


class hubbard_vqe_result(ctypes.Structure):
    _fields_ = [("E", ctypes.c_double), ("grad_norm", ctypes.c_double),
                ("steps", ctypes.c_int32), ("evals", ctypes.c_int32),
                ("reason", ctypes.c_int32), ("pad", ctypes.c_int32)]


VQE_REASONS = {0: "running", 1: "energy tolerance", 2: "gradient tolerance", 3: "max steps",
               4: "line search", 5: "not finite"}


class HubbardError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hubbard status {status}: {msg}")
        self.status = status


class hubbard_desc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("periodic_x", ctypes.c_int32), ("periodic_y", ctypes.c_int32),
        ("t_bond", ctypes.POINTER(ctypes.c_double)),
        ("U", ctypes.c_double),
        ("V_bond", ctypes.POINTER(ctypes.c_double)),
        ("eps_site", ctypes.POINTER(ctypes.c_double)),
        ("bond_group", ctypes.POINTER(ctypes.c_int32)),
    ]


class hubbard_graph_desc(ctypes.Structure):
    _fields_ = [
        ("n_sites", ctypes.c_int32), ("n_bonds", ctypes.c_int32),
        ("bond_i", ctypes.POINTER(ctypes.c_int32)), ("bond_j", ctypes.POINTER(ctypes.c_int32)),
        ("t_bond", ctypes.POINTER(ctypes.c_double)),
        ("U", ctypes.c_double),
        ("V_bond", ctypes.POINTER(ctypes.c_double)),
        ("eps_site", ctypes.POINTER(ctypes.c_double)),
        ("bond_group", ctypes.POINTER(ctypes.c_int32)),
        ("site_spin", ctypes.POINTER(ctypes.c_int32)),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is not built; run `python -m paper_2408_00836_amd.build` "
                "(hipcc, gfx950). There is no CPU fallback.")
        L = ctypes.CDLL(LIB_PATH)
        vp, st, i32, i64, u64 = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int32,
                                 ctypes.c_int64, ctypes.c_uint64)
        P = ctypes.POINTER
        sig = {
            "hubbard_create": ([P(hubbard_desc), P(vp)], st),
            "hubbard_create_graph": ([P(hubbard_graph_desc), P(vp)], st),
            "hubbard_destroy": ([vp], None),
            "hubbard_query": ([vp, P(i32), P(i32), P(i32), P(i32), P(u64)], st),
            "hubbard_bonds": ([vp, P(i32), P(i32), P(i32)], st),
            "hubbard_last_error": ([], ctypes.c_char_p),
            "hubbard_workspace_size": ([vp, i32, i32, P(ctypes.c_size_t)], st),
            "hubbard_init_neel": ([vp, vp, vp], st),
            "ansatz_apply": ([vp, vp, i32, vp, vp], st),
            "hamiltonian_apply": ([vp, vp, vp, vp], st),
            "energy": ([vp, vp, i32, vp, vp, ctypes.c_size_t, vp], st),
            "energy_grad": ([vp, vp, i32, vp, vp, vp, ctypes.c_size_t, vp], st),
            "hubbard_plan_dump": ([vp, i32, i32, P(i32), i64, P(i64)], st),
            "hubbard_set_tiles": ([vp, i32, i32, i32], st),
            "hubbard_set_timing": ([vp, i32], st),
            "hubbard_get_tiles": ([vp, P(i32)], st),
            "hubbard_tune": ([vp, i32, vp, vp, ctypes.c_size_t, vp, i32, P(i32), i32, P(i32),
                              P(ctypes.c_float)], st),
            "hubbard_batch_workspace_size": ([P(vp), i32, P(i32), P(ctypes.c_size_t)], st),
            "energy_grad_batch": ([P(vp), i32, vp, P(i64), P(i32), vp, vp, vp, ctypes.c_size_t,
                                   vp], st),
            "hubbard_phase_ms": ([vp, P(ctypes.c_float), P(ctypes.c_float),
                                  P(ctypes.c_float)], st),
            "hubbard_kernel_ms": ([vp, i32, P(ctypes.c_float), P(i32)], st),
            "hubbard_batch_cached": ([P(i32)], st),
            "hubbard_batch_set_config": ([i32, i32], st),
            "hubbard_batch_get_config": ([P(i32), P(i32)], st),
            "energy_grad_noalloc": ([vp, vp, i32, vp, vp, vp], st),
            "hubbard_vector_workspace_size": ([vp, i32, P(ctypes.c_size_t)], st),
            "hubbard_overlap": ([vp, vp, vp, vp, vp, ctypes.c_size_t, vp], st),
            "hubbard_lanczos": ([vp, vp, i32, ctypes.c_double, P(ctypes.c_double), P(i32),
                                 P(ctypes.c_double), vp, vp, ctypes.c_size_t, vp], st),
            "hubbard_tridiag_lowest": ([P(ctypes.c_double), P(ctypes.c_double), i32,
                                        P(ctypes.c_double), P(ctypes.c_double)], st),
            "hubbard_vqe_workspace_size": ([vp, i32, i32, P(ctypes.c_size_t)], st),
            "hubbard_vqe": ([vp, i32, i32, vp, P(hubbard_vqe_opts), P(hubbard_vqe_result), vp,
                             ctypes.c_size_t, vp], st),
            "hubbard_lbfgs_create": ([P(ctypes.c_double), i32, P(hubbard_vqe_opts), P(vp)], st),
            "hubbard_lbfgs_tell": ([vp, ctypes.c_double, P(ctypes.c_double), P(i32),
                                    P(ctypes.c_double)], st),
            "hubbard_lbfgs_result": ([vp, P(hubbard_vqe_result)], st),
            "hubbard_lbfgs_destroy": ([vp], None),
            "overlap_grad": ([vp, vp, i32, vp, vp, vp, vp, ctypes.c_size_t, vp], st),
            "hubbard_spin_correlation": ([vp, vp, vp, vp, vp, ctypes.c_size_t, vp], st),
            "hubbard_set_ansatz": ([vp, i32], st),
            "hubbard_param_count": ([vp, i32, P(i64)], st),
            "hubbard_sector_dim": ([vp, P(i64), P(i64)], st),
            "hubbard_sector_workspace_size": ([vp, i32, i32, P(ctypes.c_size_t)], st),
            "hubbard_sector_init_neel": ([vp, vp, vp], st),
            "sector_ansatz_apply": ([vp, vp, i32, vp, vp, ctypes.c_size_t, vp], st),
            "sector_hamiltonian_apply": ([vp, vp, vp, vp, ctypes.c_size_t, vp], st),
            "sector_energy_grad": ([vp, vp, i32, vp, vp, vp, ctypes.c_size_t, vp], st),
            "hubbard_sector_lanczos": ([vp, vp, i32, ctypes.c_double, P(ctypes.c_double),
                                        P(i32), P(ctypes.c_double), vp, vp, ctypes.c_size_t,
                                        vp], st),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != HUBBARD_OK:
        msg = lib().hubbard_last_error()
        raise HubbardError(status, msg.decode() if msg else "")


def _dptr(arr):
    if arr is None:
        return None
    a = np.ascontiguousarray(arr, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def hubbard_create(nx: int, ny: int, periodic_x: bool = False, periodic_y: bool = False,
                   t_bond=None, U: float = 0.0, V_bond=None, eps_site=None,
                   bond_group=None) -> int:
    """Returns the opaque handle (an int)."""
    keep = []
    d = hubbard_desc()
    d.nx, d.ny = int(nx), int(ny)
    d.periodic_x, d.periodic_y = int(bool(periodic_x)), int(bool(periodic_y))
    d.U = float(U)
    for field, arr in (("t_bond", t_bond), ("V_bond", V_bond), ("eps_site", eps_site)):
        if arr is not None:
            a, p = _dptr(arr)
            keep.append(a)
            setattr(d, field, p)
    if bond_group is not None:
        g = np.ascontiguousarray(bond_group, dtype=np.int32)
        keep.append(g)
        d.bond_group = g.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    h = ctypes.c_void_p()
    _check(lib().hubbard_create(ctypes.byref(d), ctypes.byref(h)))
    return h.value


def hubbard_create_graph(n_sites: int, bonds, t_bond=None, U: float = 0.0, V_bond=None,
                         eps_site=None, bond_group=None, site_spin=None) -> int:
    """Model on an arbitrary graph: `bonds` is a sequence of (i, j) site pairs.
    Returns the opaque handle (an int)."""
    keep = []
    d = hubbard_graph_desc()
    b = np.asarray(list(bonds), dtype=np.int32).reshape(-1, 2)
    d.n_sites, d.n_bonds = int(n_sites), int(b.shape[0])
    bi, bj = np.ascontiguousarray(b[:, 0]), np.ascontiguousarray(b[:, 1])
    keep += [bi, bj]
    d.bond_i = bi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.bond_j = bj.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.U = float(U)
    for field, arr in (("t_bond", t_bond), ("V_bond", V_bond), ("eps_site", eps_site)):
        if arr is not None:
            a, p = _dptr(arr)
            keep.append(a)
            setattr(d, field, p)
    for field, arr in (("bond_group", bond_group), ("site_spin", site_spin)):
        if arr is not None:
            g = np.ascontiguousarray(arr, dtype=np.int32)
            keep.append(g)
            setattr(d, field, g.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    h = ctypes.c_void_p()
    _check(lib().hubbard_create_graph(ctypes.byref(d), ctypes.byref(h)))
    return h.value


def hubbard_destroy(h: int) -> None:
    lib().hubbard_destroy(h)


def hubbard_query(h: int) -> dict:
    nq, nb, ng, ppl = (ctypes.c_int32() for _ in range(4))
    neel = ctypes.c_uint64()
    _check(lib().hubbard_query(h, ctypes.byref(nq), ctypes.byref(nb), ctypes.byref(ng),
                               ctypes.byref(ppl), ctypes.byref(neel)))
    return dict(n_qubits=nq.value, n_bonds=nb.value, n_groups=ng.value,
                params_per_layer=ppl.value, neel_index=neel.value)


def hubbard_bonds(h: int):
    nb = hubbard_query(h)["n_bonds"]
    bi, bj, g = (np.zeros(max(nb, 1), dtype=np.int32) for _ in range(3))
    P = ctypes.POINTER(ctypes.c_int32)
    _check(lib().hubbard_bonds(h, bi.ctypes.data_as(P), bj.ctypes.data_as(P), g.ctypes.data_as(P)))
    return bi[:nb], bj[:nb], g[:nb]


def hubbard_workspace_size(h: int, n_layers: int, op: int) -> int:
    b = ctypes.c_size_t()
    _check(lib().hubbard_workspace_size(h, int(n_layers), int(op), ctypes.byref(b)))
    return b.value


def hubbard_init_neel(h: int, psi_dev: int, stream: int = 0) -> None:
    _check(lib().hubbard_init_neel(h, psi_dev, stream))


def ansatz_apply(h: int, theta_dev: int, n_layers: int, psi_dev: int, stream: int = 0) -> None:
    _check(lib().ansatz_apply(h, theta_dev, int(n_layers), psi_dev, stream))


def hamiltonian_apply(h: int, psi_dev: int, out_dev: int, stream: int = 0) -> None:
    _check(lib().hamiltonian_apply(h, psi_dev, out_dev, stream))


def energy(h: int, theta_dev: int, n_layers: int, E_dev: int, ws_dev: int, ws_bytes: int,
           stream: int = 0) -> None:
    _check(lib().energy(h, theta_dev, int(n_layers), E_dev, ws_dev, int(ws_bytes), stream))


def energy_grad(h: int, theta_dev: int, n_layers: int, E_dev: int, grad_dev: int, ws_dev: int,
                ws_bytes: int, stream: int = 0) -> None:
    _check(lib().energy_grad(h, theta_dev, int(n_layers), E_dev, grad_dev, ws_dev,
                             int(ws_bytes), stream))


def hubbard_set_tiles(h: int, fwd_k: int, rev_k: int, c: int) -> None:
    _check(lib().hubbard_set_tiles(h, int(fwd_k), int(rev_k), int(c)))


def hubbard_plan_dump(h: int, n_layers: int, which: int):
    """Parsed schedule: list of passes {tile, flags, ops: [(kind, param, p, q,
    umask, emask, vbonds)]}."""
    n = ctypes.c_int64()
    _check(lib().hubbard_plan_dump(h, int(n_layers), int(which), None, 0, ctypes.byref(n)))
    buf = np.zeros(n.value, dtype=np.int32)
    _check(lib().hubbard_plan_dump(h, int(n_layers), int(which),
                                   buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   n.value, ctypes.byref(n)))
    it = iter(buf.tolist())
    passes = []
    for _ in range(next(it)):
        k = next(it)
        tile = [next(it) for _ in range(k)]
        flags = next(it)
        ops = []
        for _ in range(next(it)):
            kind, param, p, q, um, em, nv = (next(it) for _ in range(7))
            vb = [next(it) for _ in range(nv)]
            ops.append((kind, param, p, q, um & 0xffffffff, em & 0xffffffff, vb))
        passes.append(dict(tile=tile, flags=flags, ops=ops))
    return passes


def hubbard_set_timing(h: int, enable: bool) -> None:
    _check(lib().hubbard_set_timing(h, int(bool(enable))))


def hubbard_phase_ms(h: int):
    """(forward, H-or-expectation, reverse) milliseconds of the last call."""
    a, b, c = ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
    _check(lib().hubbard_phase_ms(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


KERNEL_MODES = {"forward": 0, "reverse": 1, "hamiltonian": 2, "expectation": 3}


def hubbard_kernel_ms(h: int, mode: int):
    """(summed milliseconds, launches) of one pass-kernel mode in the last call."""
    ms, n = ctypes.c_float(), ctypes.c_int32()
    _check(lib().hubbard_kernel_ms(h, int(mode), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def _handles(hs):
    arr = (ctypes.c_void_p * len(hs))(*hs)
    return arr


def hubbard_batch_workspace_size(hs, n_layers) -> int:
    lay = np.ascontiguousarray(n_layers, dtype=np.int32)
    b = ctypes.c_size_t()
    _check(lib().hubbard_batch_workspace_size(_handles(hs), len(hs),
                                              lay.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                              ctypes.byref(b)))
    return b.value


def energy_grad_batch(hs, theta_dev: int, theta_off, n_layers, E_dev: int, grad_dev: int,
                      ws_dev: int, ws_bytes: int, stream: int = 0) -> None:
    off = np.ascontiguousarray(theta_off, dtype=np.int64)
    lay = np.ascontiguousarray(n_layers, dtype=np.int32)
    _check(lib().energy_grad_batch(_handles(hs), len(hs), theta_dev,
                                   off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   lay.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   E_dev, grad_dev, ws_dev, int(ws_bytes), stream))


def hubbard_get_tiles(h: int):
    cfg = (ctypes.c_int32 * 3)()
    _check(lib().hubbard_get_tiles(h, cfg))
    return tuple(cfg)


def hubbard_tune(h: int, n_layers: int, theta_dev: int, ws_dev: int, ws_bytes: int,
                 stream: int = 0, reps: int = 2):
    """Returns [(fwd_k, rev_k, c, ms), ...]; the best is left configured."""
    cap = 64
    table = (ctypes.c_int32 * (3 * cap))()
    ms = (ctypes.c_float * cap)()
    n = ctypes.c_int32()
    _check(lib().hubbard_tune(h, int(n_layers), theta_dev, ws_dev, int(ws_bytes), stream,
                              int(reps), table, cap, ctypes.byref(n), ms))
    return [(table[3 * i], table[3 * i + 1], table[3 * i + 2], ms[i]) for i in range(n.value)]


def hubbard_batch_set_config(items: int, lanes: int) -> None:
    _check(lib().hubbard_batch_set_config(int(items), int(lanes)))


def hubbard_batch_get_config():
    """(work items per instance pass, stream lanes) used for newly planned batches."""
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().hubbard_batch_get_config(ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def hubbard_batch_cached() -> int:
    n = ctypes.c_int32()
    _check(lib().hubbard_batch_cached(ctypes.byref(n)))
    return n.value


def energy_grad_noalloc(h: int, theta_dev: int, n_layers: int, E_dev: int, grad_dev: int,
                        stream: int = 0) -> None:
    _check(lib().energy_grad_noalloc(h, theta_dev, int(n_layers), E_dev, grad_dev, stream))


def hubbard_vector_workspace_size(h: int, op: int) -> int:
    n = ctypes.c_size_t()
    _check(lib().hubbard_vector_workspace_size(h, int(op), ctypes.byref(n)))
    return n.value


def hubbard_overlap(h: int, a_dev: int, b_dev: int, out_dev: int, ws_dev: int, ws_bytes: int,
                    stream: int = 0) -> None:
    _check(lib().hubbard_overlap(h, a_dev, b_dev, out_dev, ws_dev, int(ws_bytes), stream))


def hubbard_lanczos(h: int, start_dev: int, max_iter: int, tol: float, gs_dev, ws_dev: int,
                    ws_bytes: int, stream: int = 0):
    """(E0, iterations, Ritz residual); the unit ground state goes to gs_dev
    unless it is None."""
    E0, it, res = ctypes.c_double(), ctypes.c_int32(), ctypes.c_double()
    _check(lib().hubbard_lanczos(h, start_dev, int(max_iter), float(tol), ctypes.byref(E0),
                                 ctypes.byref(it), ctypes.byref(res), gs_dev, ws_dev,
                                 int(ws_bytes), stream))
    return E0.value, it.value, res.value


def hubbard_tridiag_lowest(a, b):
    """Lowest eigenpair of the symmetric tridiagonal matrix (diag a, off-diag b)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    vec = np.zeros(a.size)
    lam = ctypes.c_double()
    P = ctypes.POINTER(ctypes.c_double)
    _check(lib().hubbard_tridiag_lowest(a.ctypes.data_as(P), b.ctypes.data_as(P) if b.size else None,
                                        a.size, ctypes.byref(lam), vec.ctypes.data_as(P)))
    return lam.value, vec


def _opts(opts):
    if opts is None:
        return None
    o = hubbard_vqe_opts()
    o.max_steps = int(opts.get("max_steps", 1000))
    o.history = int(opts.get("history", 10))
    o.e_tol = float(opts.get("e_tol", 1e-7))
    o.g_tol = float(opts.get("g_tol", 1e-6))
    return o


def _result(r):
    return dict(E=r.E, grad_norm=r.grad_norm, steps=r.steps, evals=r.evals, reason=r.reason,
                why=VQE_REASONS.get(r.reason, "?"))


def hubbard_vqe_workspace_size(h: int, n_layers: int, n_starts: int) -> int:
    n = ctypes.c_size_t()
    _check(lib().hubbard_vqe_workspace_size(h, int(n_layers), int(n_starts), ctypes.byref(n)))
    return n.value


def hubbard_vqe(h: int, n_layers: int, n_starts: int, theta_dev: int, ws_dev: int, ws_bytes: int,
                stream: int = 0, opts: dict | None = None):
    """Runs the optimisations in place on theta_dev; returns one result dict per start."""
    res = (hubbard_vqe_result * int(n_starts))()
    o = _opts(opts)
    _check(lib().hubbard_vqe(h, int(n_layers), int(n_starts), theta_dev,
                             ctypes.byref(o) if o is not None else None, res, ws_dev,
                             int(ws_bytes), stream))
    return [_result(r) for r in res]


class Lbfgs:
    """The library's optimiser driven from Python (reverse communication):
    x = opt.start; loop: f, g = F(x); state, x = opt.tell(f, g)."""

    def __init__(self, x0, opts: dict | None = None):
        x0 = np.ascontiguousarray(x0, dtype=np.float64)
        self.n = x0.size
        self.start = x0.copy()
        self._h = ctypes.c_void_p()
        o = _opts(opts)
        _check(lib().hubbard_lbfgs_create(x0.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          self.n, ctypes.byref(o) if o is not None else None,
                                          ctypes.byref(self._h)))

    def tell(self, f: float, g):
        g = np.ascontiguousarray(g, dtype=np.float64)
        x = np.zeros(self.n)
        st = ctypes.c_int32()
        P = ctypes.POINTER(ctypes.c_double)
        _check(lib().hubbard_lbfgs_tell(self._h, float(f), g.ctypes.data_as(P), ctypes.byref(st),
                                        x.ctypes.data_as(P)))
        return st.value, x

    def result(self):
        r = hubbard_vqe_result()
        _check(lib().hubbard_lbfgs_result(self._h, ctypes.byref(r)))
        return _result(r)

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().hubbard_lbfgs_destroy(self._h)
            self._h = ctypes.c_void_p()


def overlap_grad(h: int, theta_dev: int, n_layers: int, ref_dev: int, out_dev: int,
                 grad_dev: int, ws_dev: int, ws_bytes: int, stream: int = 0) -> None:
    _check(lib().overlap_grad(h, theta_dev, int(n_layers), ref_dev, out_dev, grad_dev, ws_dev,
                              int(ws_bytes), stream))


def hubbard_spin_correlation(h: int, psi_dev: int, C_dev: int, Sz_dev: int, ws_dev: int,
                             ws_bytes: int, stream: int = 0) -> None:
    _check(lib().hubbard_spin_correlation(h, psi_dev, C_dev, Sz_dev, ws_dev, int(ws_bytes),
                                          stream))


def hubbard_set_ansatz(h: int, ansatz: int) -> None:
    _check(lib().hubbard_set_ansatz(h, int(ansatz)))


def hubbard_param_count(h: int, n_layers: int) -> int:
    n = ctypes.c_int64()
    _check(lib().hubbard_param_count(h, int(n_layers), ctypes.byref(n)))
    return n.value


def hubbard_sector_dim(h: int):
    """(C(Ns, N_up), C(Ns, N_dn)) of the handle's start state."""
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().hubbard_sector_dim(h, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def hubbard_sector_workspace_size(h: int, n_layers: int, op: int) -> int:
    n = ctypes.c_size_t()
    _check(lib().hubbard_sector_workspace_size(h, int(n_layers), int(op), ctypes.byref(n)))
    return n.value


def hubbard_sector_init_neel(h: int, psi_dev: int, stream: int = 0) -> None:
    _check(lib().hubbard_sector_init_neel(h, psi_dev, stream))


def sector_ansatz_apply(h: int, theta_dev: int, n_layers: int, psi_dev: int, ws_dev: int,
                        ws_bytes: int, stream: int = 0) -> None:
    _check(lib().sector_ansatz_apply(h, theta_dev, int(n_layers), psi_dev, ws_dev, int(ws_bytes),
                                     stream))


def sector_hamiltonian_apply(h: int, psi_dev: int, out_dev: int, ws_dev: int, ws_bytes: int,
                             stream: int = 0) -> None:
    _check(lib().sector_hamiltonian_apply(h, psi_dev, out_dev, ws_dev, int(ws_bytes), stream))


def sector_energy_grad(h: int, theta_dev: int, n_layers: int, E_dev: int, grad_dev: int,
                       ws_dev: int, ws_bytes: int, stream: int = 0) -> None:
    _check(lib().sector_energy_grad(h, theta_dev, int(n_layers), E_dev, grad_dev, ws_dev,
                                    int(ws_bytes), stream))


def hubbard_sector_lanczos(h: int, start_dev: int, max_iter: int, tol: float, gs_dev,
                           ws_dev: int, ws_bytes: int, stream: int = 0):
    """(E0, iterations, Ritz residual) on sector vectors; the unit ground
    state goes to gs_dev unless it is None."""
    E0, it, res = ctypes.c_double(), ctypes.c_int32(), ctypes.c_double()
    _check(lib().hubbard_sector_lanczos(h, start_dev, int(max_iter), float(tol),
                                        ctypes.byref(E0), ctypes.byref(it), ctypes.byref(res),
                                        gs_dev, ws_dev, int(ws_bytes), stream))
    return E0.value, it.value, res.value
