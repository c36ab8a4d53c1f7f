"""Oracle-side model description: lattice, bonds, hopping groups, Neel start.

TEST INFRASTRUCTURE ONLY -- part of the oracle.  Only the tests, the smoke
check and the CPU-baseline leg of the benchmark may import this package.  It
shares nothing with the GPU library and never imports it.

Conventions (readings of the paper, written out here from scratch):

* Sites of an Nx x Ny lattice are numbered row-major, s = x*Ny + y (the 0-based
  form of the site index of Sec. 2.2.1).
* Bonds are the unordered nearest-neighbour pairs of Eq. (1), each once, in the
  canonical order: every horizontal bond (x,y)-(x,y+1) by start site
  row-major (with the periodic wrap (x,Ny-1)-(x,0) right after the row's last
  ordinary bond), then every vertical bond (x,y)-(x+1,y) by start site
  row-major (the wrap (Nx-1,y)-(0,y) last).
* Hopping groups follow Eq. (7): the horizontal bonds split into h1/h2 and the
  vertical ones into v1/v2 so that each group holds mutually commuting terms.
  Horizontal bonds go by the parity of their start column y, vertical bonds by
  the parity of their start row x.  A direction of length 2 whose transverse
  length is at least 3 (a 2 x L ladder) splits by the transverse parity
  instead, so every group is a matching.  Groups are applied in the order
  h1, v1, h2, v2 after the diagonal, empty ones skipped.
* The start state is the checkerboard product state of Sec. 2.1: site (x,y)
  holds one spin-up electron if x+y is even and one spin-down otherwise.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

H1, V1, H2, V2 = 0, 1, 2, 3
CLASS_ORDER = (H1, V1, H2, V2)


@dataclasses.dataclass
class OracleModel:
    nx: int
    ny: int
    periodic_x: bool
    periodic_y: bool
    bonds: list          # list of (i, j) site pairs, canonical order
    bond_class: list     # raw group class per bond (H1, V1, H2, V2) or user id
    t: np.ndarray        # hopping per bond
    V: np.ndarray        # nearest-neighbour interaction per bond
    eps: np.ndarray      # on-site energy per site
    U: float
    interleaved: bool = False
    site_spin: Optional[list] = None   # graph models: start spin per site (0 up, 1 down)

    @property
    def nsites(self) -> int:
        return self.nx * self.ny

    @property
    def nqubits(self) -> int:
        return 2 * self.nsites

    @property
    def group_ids(self) -> list:
        """Distinct group ids in application order (empty ones never appear)."""
        return sorted(set(self.bond_class))

    @property
    def ngroups(self) -> int:
        return len(self.group_ids)

    @property
    def params_per_layer(self) -> int:
        return 1 + self.ngroups

    def bond_slot(self) -> list:
        """Parameter slot (1..G) of each bond."""
        ids = self.group_ids
        return [1 + ids.index(c) for c in self.bond_class]

    def qubit(self, site: int, spin: int) -> int:
        if self.interleaved:
            return 2 * site + spin
        return site + self.nsites * spin

    def neel_sites(self):
        """(up_sites, down_sites) of the checkerboard start state (graph
        models: of their stated start spins)."""
        up, dn = [], []
        if self.site_spin is not None:
            for s, sp in enumerate(self.site_spin):
                (dn if sp else up).append(s)
            return up, dn
        for x in range(self.nx):
            for y in range(self.ny):
                (up if (x + y) % 2 == 0 else dn).append(x * self.ny + y)
        return up, dn

    def neel_index(self) -> int:
        up, dn = self.neel_sites()
        b = 0
        for s in up:
            b |= 1 << self.qubit(s, 0)
        for s in dn:
            b |= 1 << self.qubit(s, 1)
        return b

    def with_order(self, interleaved: bool) -> "OracleModel":
        return dataclasses.replace(self, interleaved=interleaved)


def enumerate_bonds(nx: int, ny: int, periodic_x: bool, periodic_y: bool):
    """Canonical bond list and default group class of each bond."""
    if nx < 1 or ny < 1:
        raise ValueError("lattice must have at least one site")
    for length, per, name in ((ny, periodic_y, "y"), (nx, periodic_x, "x")):
        if per and length < 3:
            raise ValueError(f"periodic {name} needs length >= 3")
    bonds, cls = [], []
    h_by_x = ny == 2 and nx >= 3          # 2-long rows of a tall ladder
    v_by_y = nx == 2 and ny >= 3          # 2-long columns of a wide ladder
    for x in range(nx):
        for y in range(ny):
            if y + 1 < ny:
                nb = (x, y + 1)
            elif periodic_y:
                nb = (x, 0)
            else:
                continue
            bonds.append((x * ny + y, nb[0] * ny + nb[1]))
            par = (x if h_by_x else y) % 2
            cls.append(H1 if par == 0 else H2)
    for x in range(nx):
        for y in range(ny):
            if x + 1 < nx:
                nb = (x + 1, y)
            elif periodic_x:
                nb = (0, y)
            else:
                continue
            bonds.append((x * ny + y, nb[0] * ny + nb[1]))
            par = (y if v_by_y else x) % 2
            cls.append(V1 if par == 0 else V2)
    return bonds, cls


def check_matchings(bonds, cls):
    """Every group must be a matching (no site in two of its bonds)."""
    seen = {}
    for (i, j), c in zip(bonds, cls):
        used = seen.setdefault(c, set())
        if i in used or j in used:
            raise ValueError(f"group {c} is not a matching (site {i} or {j} repeated)")
        used.add(i)
        used.add(j)


def make_model(nx: int, ny: int, *, periodic_x: bool = False, periodic_y: bool = False,
               t: Optional[Sequence[float]] = None, U: float = 0.0,
               V: Optional[Sequence[float]] = None, eps: Optional[Sequence[float]] = None,
               groups: Optional[Sequence[int]] = None, interleaved: bool = False) -> OracleModel:
    bonds, cls = enumerate_bonds(nx, ny, periodic_x, periodic_y)
    if groups is not None:
        if len(groups) != len(bonds):
            raise ValueError("one group id per bond")
        cls = [int(g) for g in groups]
    check_matchings(bonds, cls)
    nb, ns = len(bonds), nx * ny
    t_arr = np.ones(nb) if t is None else np.asarray(t, dtype=np.float64).copy()
    V_arr = np.zeros(nb) if V is None else np.asarray(V, dtype=np.float64).copy()
    e_arr = np.zeros(ns) if eps is None else np.asarray(eps, dtype=np.float64).copy()
    if t_arr.shape != (nb,) or V_arr.shape != (nb,) or e_arr.shape != (ns,):
        raise ValueError("t and V need one value per bond, eps one per site")
    return OracleModel(nx, ny, bool(periodic_x), bool(periodic_y), bonds, cls,
                       t_arr, V_arr, e_arr, float(U), bool(interleaved))


def greedy_matchings(bonds):
    """Default groups of a graph: in bond order, each bond joins the lowest
    group in which neither of its sites is used yet (so every group is a
    matching)."""
    used, out = [], []
    for i, j in bonds:
        g = 0
        while g < len(used) and (i in used[g] or j in used[g]):
            g += 1
        if g == len(used):
            used.append(set())
        used[g] |= {i, j}
        out.append(g)
    return out


def make_graph_model(n_sites: int, bonds, *, t: Optional[Sequence[float]] = None,
                     U: float = 0.0, V: Optional[Sequence[float]] = None,
                     eps: Optional[Sequence[float]] = None,
                     groups: Optional[Sequence[int]] = None,
                     site_spin: Optional[Sequence[int]] = None,
                     interleaved: bool = False) -> OracleModel:
    """Hubbard model of Eq. (2)/(15)/(16) on an arbitrary graph: the sites
    0..n_sites-1, one hopping term and one V term per listed bond (unordered,
    each once).  Start state: one electron per site with spin site_spin[s]
    (default: up on even sites, down on odd ones)."""
    if n_sites < 1:
        raise ValueError("at least one site")
    bonds = [(int(i), int(j)) for i, j in bonds]
    seen = set()
    for i, j in bonds:
        if not (0 <= i < n_sites and 0 <= j < n_sites) or i == j:
            raise ValueError(f"bad bond ({i}, {j})")
        key = (min(i, j), max(i, j))
        if key in seen:
            raise ValueError(f"bond ({i}, {j}) listed twice")
        seen.add(key)
    cls = greedy_matchings(bonds) if groups is None else [int(g) for g in groups]
    if len(cls) != len(bonds):
        raise ValueError("one group id per bond")
    check_matchings(bonds, cls)
    spins = [s % 2 for s in range(n_sites)] if site_spin is None else [int(x) for x in site_spin]
    if len(spins) != n_sites or any(x not in (0, 1) for x in spins):
        raise ValueError("site_spin needs one 0/1 entry per site")
    nb = len(bonds)
    t_arr = np.ones(nb) if t is None else np.asarray(t, dtype=np.float64).copy()
    V_arr = np.zeros(nb) if V is None else np.asarray(V, dtype=np.float64).copy()
    e_arr = np.zeros(n_sites) if eps is None else np.asarray(eps, dtype=np.float64).copy()
    if t_arr.shape != (nb,) or V_arr.shape != (nb,) or e_arr.shape != (n_sites,):
        raise ValueError("t and V need one value per bond, eps one per site")
    return OracleModel(1, n_sites, False, False, bonds, cls, t_arr, V_arr, e_arr, float(U),
                       bool(interleaved), spins)
