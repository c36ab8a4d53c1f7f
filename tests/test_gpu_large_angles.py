"""Large angles on the general diagonal (U, V and eps terms) and hopping
periodicity, through the C ABI against the oracle.

The general diagonal's phase exp(-i th D(b)) is evaluated on the GPU from a
256-entry table of unit phases after a two-part Cody-Waite reduction of
th D(b); the reduction is exact while th D(b) stays below 2^17 table steps
(|th D| < 3216.99).  The oracle calls libm's sin/cos directly.  The cases
below push th D into the thousands and compare energies, gradients and
amplitudes with the oracle, and check that a hopping parameter is 2 pi
periodic at t = 1 (each pair rotation is (cos th, i s sin th)).

Bars as elsewhere: amplitudes max-abs <= 1e-10, |dE| <= 1e-12 max(1, |E|),
gradient max-abs <= 1e-8.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import core as oc
from oracle.model import make_model
from paper_2408_00836_amd import workloads as W
from paper_2408_00836_amd.model import Hubbard

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def e_tol(E):
    return 1e-12 * max(1.0, abs(E))


def ladder(seed, layers=4, disorder=0.0):
    # 2x4 open ladder, 16 qubits, U = 4, V = 0.5, eps ~ U(-0.5, 0.5): the
    # general-diagonal kernels; t = 1 unless disorder is given
    return W.random_instance(2, 4, layers, 5, seed, U=4.0, disorder=disorder, eps_width=0.5,
                             V=0.5, name=f"2x4 ladder V=0.5 eps seed {seed}")


def max_diag(om):
    """Largest |D(b)| over the basis (D = U n_up n_dn + V n n + eps n)."""
    b = np.arange(1 << om.nqubits, dtype=np.int64)
    up = [(b >> om.qubit(i, 0)) & 1 for i in range(om.nsites)]
    dn = [(b >> om.qubit(i, 1)) & 1 for i in range(om.nsites)]
    n = [u + d for u, d in zip(up, dn)]
    D = om.U * sum(u * d for u, d in zip(up, dn)).astype(np.float64)
    D = D + sum(om.eps[i] * n[i] for i in range(om.nsites))
    D = D + sum(V * n[i] * n[j] for (i, j), V in zip(om.bonds, om.V))
    return float(np.max(np.abs(D)))


@pytest.mark.parametrize("scale", [12.0, 40.0])
def test_large_diagonal_angles_vs_oracle(gpu, scale):
    w = ladder(4101, disorder=0.1)
    per = w.params_per_layer
    th = w.theta.copy()
    # every diagonal angle of the circuit scaled up: th_D in the tens to hundreds
    th[0::per] = scale * np.sign(th[0::per]) * (1.0 + np.abs(th[0::per]))
    om = make_model(w.nx, w.ny, **w.kwargs())
    x_max = float(np.max(np.abs(th[0::per]))) * max_diag(om)
    say(f"[large-angle] {w.name}: max |th D| = {x_max:.1f} (exact reduction below 3216.99)")
    assert x_max < 3216.0
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    assert m.general
    tdev = torch.tensor(th, dtype=torch.float64, device=gpu)
    psi = m.ansatz(tdev)
    E, g = m.energy_grad(tdev)
    torch.cuda.synchronize()
    ref = oc.ansatz(om, th, w.layers)
    E_ref, g_ref = oc.energy_grad(om, th, w.layers)
    amp_err = float(np.max(np.abs(psi.cpu().numpy() - ref)))
    dE = abs(E.item() - E_ref)
    dg = float(np.max(np.abs(g.cpu().numpy() - g_ref)))
    say(f"[large-angle] scale {scale}: amp {amp_err:.2e}, dE {dE:.2e}, dg {dg:.2e}")
    assert amp_err <= 1e-10
    assert dE <= e_tol(E_ref)
    assert dg <= 1e-8


def test_hop_parameters_are_2pi_periodic(gpu):
    w = ladder(4102)          # t = 1 on every bond
    per = w.params_per_layer
    m = Hubbard(w.nx, w.ny, **w.kwargs())
    th0 = torch.tensor(w.theta, dtype=torch.float64, device=gpu)
    E0, g0 = m.energy_grad(th0)
    E0 = E0.item()
    g0 = g0.cpu().numpy()
    for k in (1, 2, per + 3, 3 * per + 4):
        th = w.theta.copy()
        th[k] += 2.0 * np.pi * (1 if k % 2 else -3)
        E, g = m.energy_grad(torch.tensor(th, dtype=torch.float64, device=gpu))
        dE = abs(E.item() - E0)
        dg = float(np.max(np.abs(g.cpu().numpy() - g0)))
        say(f"[periodic] param {k}: dE {dE:.2e}, dg {dg:.2e}")
        assert dE <= e_tol(E0)
        assert dg <= 1e-8
