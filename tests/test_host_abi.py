"""Host-side tests of the C ABI (no GPU calls): the library loads and exports
every declared symbol, argument validation, and the invariants of the pass
schedule (every circuit operation applied exactly once, in an order that
keeps every non-commuting pair in circuit order, inside its tile)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.model import make_model
from paper_2408_00836_amd import abi, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            for m in re.finditer(r"^\s*(?:const\s+)?[\w\s\*]+?\b(\w+)\s*\(", src, flags=re.M):
                if m.group(1) not in ("if", "for", "while", "sizeof"):
                    names.add(m.group(1))
    return names


def test_library_exports_declared_symbols():
    L = abi.lib()
    decl = declared_functions()
    assert {"hubbard_create", "ansatz_apply", "hamiltonian_apply", "energy",
            "energy_grad"} <= decl
    for name in decl:
        assert hasattr(L, name), name
    assert set(abi.EXPORTED) >= decl


@pytest.mark.parametrize("args,msg", [
    (dict(nx=0, ny=2), "nx and ny"),
    (dict(nx=5, ny=4), "16 sites"),
    (dict(nx=1, ny=2, periodic_y=True), "periodic_y"),
    (dict(nx=1, ny=3, periodic_y=True), "not a matching"),
    (dict(nx=1, ny=4, U=float("nan")), "finite"),
    (dict(nx=1, ny=3, t_bond=[1.0, float("inf")]), "finite"),
    (dict(nx=1, ny=3, bond_group=[0, 0]), "not a matching"),
    (dict(nx=1, ny=3, bond_group=[0, -1]), ">= 0"),
])
def test_create_rejects_invalid(args, msg):
    with pytest.raises(abi.HubbardError) as e:
        abi.hubbard_create(**args)
    assert e.value.status == abi.HUBBARD_ERR_ARG
    assert msg in str(e.value)


def test_null_arguments_are_errors():
    L = abi.lib()
    assert L.hubbard_create(None, None) == abi.HUBBARD_ERR_ARG
    assert L.ansatz_apply(None, None, 1, None, None) == abi.HUBBARD_ERR_ARG
    assert L.energy(None, None, 1, None, None, 0, None) == abi.HUBBARD_ERR_ARG
    h = abi.hubbard_create(2, 2, U=4.0)
    try:
        with pytest.raises(abi.HubbardError) as e:
            abi.hubbard_workspace_size(h, 2, 7)
        assert e.value.status == abi.HUBBARD_ERR_ARG
        # aliasing is rejected before anything touches the device
        st = L.hamiltonian_apply(h, ctypes.c_void_p(4096), ctypes.c_void_p(4096 + 16), None)
        assert st == abi.HUBBARD_ERR_ARG
    finally:
        abi.hubbard_destroy(h)


LATTICES = [(1, 2, 0, 0), (1, 5, 0, 0), (1, 8, 0, 0), (1, 4, 0, 1), (1, 6, 0, 1), (2, 2, 0, 0),
            (2, 3, 0, 0), (2, 4, 0, 0), (2, 6, 0, 0), (3, 3, 0, 0), (3, 2, 0, 0), (6, 2, 0, 0),
            (4, 4, 1, 1), (4, 4, 0, 0), (2, 4, 0, 1), (4, 2, 1, 0), (1, 1, 0, 0), (4, 3, 1, 0)]


@pytest.mark.parametrize("nx,ny,px,py", LATTICES)
def test_bonds_groups_neel_agree_with_oracle(nx, ny, px, py):
    """The library and the oracle enumerate bonds, groups and the start state
    independently; they must agree."""
    om = make_model(nx, ny, periodic_x=bool(px), periodic_y=bool(py))
    h = abi.hubbard_create(nx, ny, px, py, U=1.0)
    try:
        q = abi.hubbard_query(h)
        bi, bj, g = abi.hubbard_bonds(h)
        assert q["n_qubits"] == om.nqubits
        assert q["n_bonds"] == len(om.bonds)
        assert list(zip(bi.tolist(), bj.tolist())) == [tuple(b) for b in om.bonds]
        assert [s - 1 for s in om.bond_slot()] == g.tolist()
        assert q["params_per_layer"] == om.params_per_layer
        assert q["neel_index"] == om.neel_index()
    finally:
        abi.hubbard_destroy(h)


def test_stated_parameter_counts():
    """Per-layer parameter counts the configurations state match the model."""
    for w in [workloads.config1(), workloads.config2(), workloads.config3(), workloads.config5()]:
        om = make_model(w.nx, w.ny, periodic_x=w.periodic_x, periodic_y=w.periodic_y)
        assert om.params_per_layer == w.params_per_layer, w.name
    for (nx, ny), per in workloads.BATCH_PER_LAYER.items():
        if nx * ny <= 16:
            assert make_model(nx, ny).params_per_layer == per


# ------------------------------------------------------ schedule checks --

def circuit_elements(om, layers):
    """Elementary ops (key, kind, qubits, payload) in circuit order; key =
    (layer, slot) orders non-commuting pairs."""
    per = om.params_per_layer
    slots = om.bond_slot()
    out = []
    for l in range(layers):
        for i in range(om.nsites):
            out.append(((l, 0), "site", frozenset({om.qubit(i, 0), om.qubit(i, 1)}), i))
        for b, (i, j) in enumerate(om.bonds):
            if om.V[b] != 0:
                out.append(((l, 0), "vbond",
                            frozenset({om.qubit(i, 0), om.qubit(i, 1), om.qubit(j, 0),
                                       om.qubit(j, 1)}), b))
        for s in range(1, per):
            for b, (i, j) in enumerate(om.bonds):
                if slots[b] == s:
                    for sp in (0, 1):
                        p, q = sorted((om.qubit(i, sp), om.qubit(j, sp)))
                        out.append(((l, s), "hop", frozenset({p, q}), (p, q)))
    return out


def schedule_elements(om, passes, layers):
    """Expand the dumped schedule into elementary ops with their keys."""
    per = om.params_per_layer
    seq = []
    for pi, P in enumerate(passes):
        tile = set(P["tile"])
        for kind, param, p, q, um, em, vb in P["ops"]:
            l, s = divmod(param, per)
            if kind == 1:
                assert p in tile and q in tile
                seq.append(((l, s), "hop", frozenset({p, q}), (p, q), pi))
            else:
                sites = [i for i in range(om.nsites) if (um >> om.qubit(i, 0)) & 1 or
                         (em >> om.qubit(i, 0)) & 1]
                for i in sites:
                    seq.append(((l, 0), "site", frozenset({om.qubit(i, 0), om.qubit(i, 1)}),
                                i, pi))
                for b in vb:
                    i, j = om.bonds[b]
                    seq.append(((l, 0), "vbond",
                                frozenset({om.qubit(i, 0), om.qubit(i, 1), om.qubit(j, 0),
                                           om.qubit(j, 1)}), b, pi))
    return seq


def check_order(seq):
    for a in range(len(seq)):
        for b in range(a + 1, len(seq)):
            ka, kb = seq[a], seq[b]
            if ka[1] != "hop" and kb[1] != "hop":
                continue
            if ka[2] & kb[2]:
                assert ka[0] < kb[0], (ka, kb)


SCHED_CASES = [(2, 2, 0, 0, 2, 0.0), (1, 8, 0, 0, 3, 0.0), (2, 6, 0, 0, 3, 0.5),
               (3, 3, 0, 0, 2, 0.5), (4, 4, 1, 1, 3, 0.0), (2, 4, 0, 1, 2, 0.3)]


@pytest.mark.parametrize("nx,ny,px,py,L,V", SCHED_CASES)
@pytest.mark.parametrize("tiles", [None, (6, 6, 2), (8, 7, 3)])
def test_forward_and_reverse_schedules(nx, ny, px, py, L, V, tiles):
    om0 = make_model(nx, ny, periodic_x=bool(px), periodic_y=bool(py))
    nb = len(om0.bonds)
    rng = np.random.default_rng(1)
    eps = rng.uniform(-0.5, 0.5, nx * ny)
    om = make_model(nx, ny, periodic_x=bool(px), periodic_y=bool(py), U=4.0,
                    V=np.full(nb, V), eps=eps)
    h = abi.hubbard_create(nx, ny, px, py, U=4.0, V_bond=np.full(nb, V), eps_site=eps)
    try:
        if tiles:
            abi.hubbard_set_tiles(h, *tiles)
        want = circuit_elements(om, L)
        fwd = abi.hubbard_plan_dump(h, L, 0)
        seq = schedule_elements(om, fwd, L)
        key = lambda e: (e[0], e[1], sorted(e[2]), str(e[3]))
        assert sorted(map(key, seq)) == sorted(map(key, want))
        check_order(seq)
        rev = abi.hubbard_plan_dump(h, L, 2)
        rseq = schedule_elements(om, rev, L)
        assert sorted(map(key, rseq)) == sorted(map(key, want))
        check_order(rseq[::-1])   # read backwards it is a forward order
        for P in fwd + rev:
            assert len(P["tile"]) <= (tiles[0] if tiles else 13)
            assert P["tile"] == sorted(P["tile"])
    finally:
        abi.hubbard_destroy(h)


@pytest.mark.parametrize("nx,ny,px,py,L,V", SCHED_CASES)
def test_hamiltonian_schedule_covers_every_term_once(nx, ny, px, py, L, V):
    om = make_model(nx, ny, periodic_x=bool(px), periodic_y=bool(py))
    nb = len(om.bonds)
    h = abi.hubbard_create(nx, ny, px, py, U=4.0, V_bond=np.full(nb, V))
    try:
        for which in (1, 3):
            ps = abi.hubbard_plan_dump(h, L, which)
            terms, diags = [], 0
            for pi, P in enumerate(ps):
                for kind, param, p, q, um, em, vb in P["ops"]:
                    assert param == -1
                    if kind == 1:
                        assert p in P["tile"] and q in P["tile"]
                        terms.append((p, q))
                    else:
                        diags += 1
                        assert pi == 0
                        assert sorted(vb) == [b for b in range(nb) if V != 0]
            want = sorted(tuple(sorted((om.qubit(i, s), om.qubit(j, s))))
                          for (i, j) in om.bonds for s in (0, 1))
            assert sorted(terms) == want
            assert diags == 1
    finally:
        abi.hubbard_destroy(h)


def test_workspace_sizes():
    for w in [workloads.config1(), workloads.config3(), workloads.config5()]:
        h = abi.hubbard_create(w.nx, w.ny, w.periodic_x, w.periodic_y, w.t, w.U, w.V, w.eps)
        try:
            vec = (1 << w.n_qubits) * 16
            e = abi.hubbard_workspace_size(h, w.layers, abi.HUBBARD_OP_ENERGY)
            g = abi.hubbard_workspace_size(h, w.layers, abi.HUBBARD_OP_ENERGY_GRAD)
            assert vec <= e < vec + (64 << 20)
            assert 2 * vec <= g < 2 * vec + (64 << 20)
        finally:
            abi.hubbard_destroy(h)


def test_batch_workspace_size():
    ws = workloads.batch(12)
    hs = [abi.hubbard_create(w.nx, w.ny, w.periodic_x, w.periodic_y, w.t, w.U, w.V, w.eps)
          for w in ws]
    try:
        layers = [w.layers for w in ws]
        vecs = sum(2 * (((1 << w.n_qubits) * 16 + 255) // 256 * 256) for w in ws)
        b = abi.hubbard_batch_workspace_size(hs, layers)
        # psi and lambda of every instance, then the partial sums: at most one
        # row per parameter and reverse pass, each of at most 64 items
        assert vecs < b <= vecs + 256 + 8 * 64 * sum(
            w.n_params * 64 + 1 for w in ws)
        assert b == abi.hubbard_batch_workspace_size(hs, layers)   # deterministic
        more = abi.hubbard_batch_workspace_size(hs, [L + 2 for L in layers])
        assert more > b   # more layers, more reduction rows
        with pytest.raises(abi.HubbardError):
            abi.hubbard_batch_workspace_size(hs, [-1] + layers[1:])
    finally:
        for h in hs:
            abi.hubbard_destroy(h)


def test_create_graph_matches_lattice_form():
    from oracle.model import make_model as om_make
    m = om_make(4, 4, periodic_x=True, periodic_y=True)
    spins = [((s // 4) + (s % 4)) % 2 for s in range(16)]
    h1 = abi.hubbard_create(4, 4, True, True, None, 8.0)
    h2 = abi.hubbard_create_graph(16, m.bonds, None, 8.0, bond_group=m.bond_class,
                                  site_spin=spins)
    try:
        assert abi.hubbard_query(h1) == abi.hubbard_query(h2)
        for which in (0, 1, 2):
            assert abi.hubbard_plan_dump(h1, 3, which) == abi.hubbard_plan_dump(h2, 3, which)
    finally:
        abi.hubbard_destroy(h1)
        abi.hubbard_destroy(h2)


def test_create_graph_defaults_agree_with_oracle():
    from oracle.model import make_graph_model
    bonds = [(0, 5), (1, 2), (2, 5), (0, 3), (3, 4), (1, 4), (0, 2)]
    om = make_graph_model(6, bonds, U=2.0)
    h = abi.hubbard_create_graph(6, bonds, None, 2.0)
    try:
        q = abi.hubbard_query(h)
        assert q["neel_index"] == om.neel_index()
        assert q["params_per_layer"] == om.params_per_layer
        bi, bj, grp = abi.hubbard_bonds(h)
        assert list(zip(bi, bj)) == bonds
        assert [g + 1 for g in grp] == om.bond_slot()   # hubbard_bonds slots are 0-based
    finally:
        abi.hubbard_destroy(h)


@pytest.mark.parametrize("n,bonds,kw,msg", [
    (0, [], {}, "n_sites"),
    (17, [], {}, "n_sites"),
    (3, [(0, 3)], {}, "bad site"),
    (3, [(1, 1)], {}, "bad site"),
    (3, [(0, 1), (1, 0)], {}, "twice"),
    (3, [(0, 1), (1, 2)], {"bond_group": [0, 0]}, "matching"),
    (3, [(0, 1)], {"site_spin": [0, 2, 1]}, "site_spin"),
    (3, [(0, 1)], {"t_bond": [float("nan")]}, "finite"),
])
def test_create_graph_rejects_invalid(n, bonds, kw, msg):
    with pytest.raises(abi.HubbardError, match=msg):
        abi.hubbard_create_graph(n, bonds, **kw)


def test_tiles_too_small_for_a_hop_are_rejected():
    """A tile with fewer than two bits beyond its contiguous low bits cannot
    hold a hopping term on two higher qubits: rejected up front instead of
    planned."""
    h = abi.hubbard_create(2, 3, False, False, None, 4.0, None, None, None)
    try:
        with pytest.raises(abi.HubbardError) as e:
            abi.hubbard_set_tiles(h, 3, 3, 2)
        assert e.value.status == abi.HUBBARD_ERR_ARG
        abi.hubbard_set_tiles(h, 4, 4, 2)              # two free bits: fine
        assert len(abi.hubbard_plan_dump(h, 2, 0)) > 1
        h1 = abi.hubbard_create(1, 1, False, False, None, 4.0, None, None, None)
        abi.hubbard_set_tiles(h1, 2, 2, 2)             # the tile holds every qubit
        abi.hubbard_destroy(h1)
    finally:
        abi.hubbard_destroy(h)


@pytest.mark.parametrize("seed", range(6))
def test_tridiag_lowest_matches_lapack(seed):
    """The Lanczos driver's projected problem (host code): lowest eigenpair of
    a symmetric tridiagonal matrix against LAPACK (scipy's
    eigh_tridiagonal), including clustered and 1x1 cases."""
    import scipy.linalg as sla
    rng = np.random.default_rng(seed)
    m = [1, 2, 5, 40, 150, 300][seed]
    a = rng.normal(size=m) * (10.0 if seed % 2 else 1.0)
    b = rng.normal(size=m - 1)
    if seed == 4:
        b[::7] = 1e-13   # nearly decoupled blocks: clustered eigenvalues
    lam, vec = abi.hubbard_tridiag_lowest(a, b)
    w, V = sla.eigh_tridiagonal(a, b)
    assert abs(lam - w[0]) <= 1e-13 * max(1.0, abs(w[0]))
    if m > 1 and w[1] - w[0] > 1e-8:
        ref = V[:, 0] * np.sign(V[np.argmax(np.abs(V[:, 0])), 0])
        assert np.max(np.abs(vec - ref)) <= 1e-9
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    assert np.linalg.norm(T @ vec - lam * vec) <= 1e-10 * max(1.0, abs(lam))
