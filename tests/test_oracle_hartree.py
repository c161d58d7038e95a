"""Pins of the oracle's multipole Hartree potential (oracle/hartree.py) against closed forms of
Gaussian charge distributions; CPU only."""
import math

import numpy as np
import pytest
from scipy.special import erf

import synth
from oracle.hartree import hartree


def _grid(centres, n_radial=75, angular="lobatto302"):
    def f(r):
        e = np.exp(-r * r)
        return e, -0.5 * (4 * r * r - 6) * e
    na = len(centres)
    return synth.custom_instance(np.asarray(centres, dtype=np.float64), list(range(na)),
                                 [[0]] * na, [f] * na, n_log=200, n_radial=n_radial,
                                 angular=angular)


def _gauss(pts, centre, alpha, charge):
    r2 = ((pts - centre) ** 2).sum(1)
    return charge * (alpha / math.pi) ** 1.5 * np.exp(-alpha * r2)


def _gauss_potential(pts, centre, alpha, charge):
    r = np.linalg.norm(pts - centre, axis=1)
    return charge * erf(math.sqrt(alpha) * r) / r


def test_single_gaussian_closed_form():
    """n = (a/pi)^(3/2) e^{-a r^2}: v_H = erf(sqrt(a) r)/r, E_H = sqrt(a / (2 pi)), and the
    error falls as the fourth power of the radial spacing (cubic splines in theta)."""
    a = 1.7
    errs = {}
    for K in (75, 150):
        inst = _grid([[0.2, -0.1, 0.3]], n_radial=K, angular="gl110")
        shell, KK, rm = synth.radial_shells(inst)
        n = _gauss(inst.pt_xyz, inst.atom_xyz[0], a, 1.0)
        ref = _gauss_potential(inst.pt_xyz, inst.atom_xyz[0], a, 1.0)
        for l_max in (0, 4):
            h = hartree(inst, n, shell, KK, rm, l_max)
            errs[K, l_max] = np.max(np.abs(h["v"] - ref))
            if K == 75:
                assert errs[K, l_max] < 5e-6
                assert abs(h["E_H"] - math.sqrt(a / (2 * math.pi))) < 2e-6
                # total charge from the monopole moment: q_00 sqrt(4 pi) = N
                assert abs(h["q"][0, 0] * math.sqrt(4 * math.pi) - 1.0) < 1e-5
    assert errs[150, 0] < errs[75, 0] / 10           # ~16 for fourth order
    assert abs(errs[75, 4] - errs[75, 0]) < 1e-9       # a spherical density has no l > 0 part


def test_two_centre_expansion_converges():
    """Two Gaussian charges on two atoms: exact v_H is the sum of erf potentials; the partitioned
    multipole expansion converges to it as l_max grows."""
    A = np.array([0.0, 0.0, 0.0])
    B = np.array([0.0, 0.4, 1.3])
    inst = _grid([A, B])
    shell, K, rm = synth.radial_shells(inst)
    n = _gauss(inst.pt_xyz, A, 1.2, 1.0) + _gauss(inst.pt_xyz, B, 0.8, 2.0)
    ref = _gauss_potential(inst.pt_xyz, A, 1.2, 1.0) + _gauss_potential(inst.pt_xyz, B, 0.8, 2.0)
    errs = []
    for l_max in (0, 2, 4, 6, 8):
        h = hartree(inst, n, shell, K, rm, l_max)
        errs.append(np.max(np.abs(h["v"] - ref)) / np.max(np.abs(ref)))
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs
    assert errs[-2] < 2e-3 and errs[-1] < 1e-3, errs
    # the energy converges faster (variational in the charge distribution)
    g = 1.2 * 0.8 / 2.0
    E_ref = 0.5 * (math.sqrt(2 * 1.2 / math.pi) + 4.0 * math.sqrt(2 * 0.8 / math.pi)) \
        + 2.0 * erf(math.sqrt(g) * np.linalg.norm(A - B)) / np.linalg.norm(A - B)
    h = hartree(inst, n, shell, K, rm, 8)
    assert abs(h["E_H"] - E_ref) < 1e-4 * E_ref


def test_off_centre_charge_needs_higher_multipoles():
    """A Gaussian off its atom's centre has dipole and higher moments: l_max = 0 misses them."""
    inst = _grid([[0.0, 0.0, 0.0]])
    shell, K, rm = synth.radial_shells(inst)
    c = np.array([0.0, 0.0, 0.25])
    n = _gauss(inst.pt_xyz, c, 2.0, 1.0)
    ref = _gauss_potential(inst.pt_xyz, c, 2.0, 1.0)
    e0 = np.max(np.abs(hartree(inst, n, shell, K, rm, 0)["v"] - ref))
    e6 = np.max(np.abs(hartree(inst, n, shell, K, rm, 6)["v"] - ref))
    assert e6 < 1e-2 * e0
    # the dipole moment along z: q_10 = sqrt(3/(4 pi)) * 0.25
    h = hartree(inst, n, shell, K, rm, 1)
    assert abs(h["q"][0, 2] - math.sqrt(3 / (4 * math.pi)) * 0.25) < 1e-5      # spline order, as above


def test_exterior_form_beyond_the_support():
    """Two atoms 9 bohr apart, a Gaussian charge on the first atom's points.  Its points end
    at a finite radius (the partition weights vanish beyond it), its edge node lies there, and
    at the second atom's outer points, beyond that edge, the potential is the exterior form of
    the first atom's moments: for a spherical charge Q/r, the erf potential of the Gaussian to
    the quadrature accuracy of Q."""
    from oracle.hartree import edge_nodes, radial_nodes
    A = np.array([0.0, 0.0, 0.0])
    B = np.array([0.0, 0.0, 9.0])
    inst = _grid([A, B])
    shell, K, rm = synth.radial_shells(inst)
    ke = edge_nodes(inst, shell, K)
    _, r, _ = radial_nodes(K, rm)
    own_a = np.asarray(inst.pt_atom) == 0
    ra = np.linalg.norm(inst.pt_xyz - A, axis=1)
    R_a = r[ke[0]]
    assert ke[0] > 0 and ra[own_a].max() < R_a             # the support ends inside the grid
    far = ra >= R_a
    assert far.sum() > 100                                  # points beyond it (atom B's far side)
    alpha = 2.0
    # the Gaussian on the first atom's points only (the second atom's share, ~1e-7 of the
    # charge, is dropped), so the second atom's piece is exactly zero
    n = _gauss(inst.pt_xyz, A, alpha, 1.0) * own_a
    h = hartree(inst, n, shell, K, rm, 0)
    ref = _gauss_potential(inst.pt_xyz, A, alpha, 1.0)
    Q = h["q"][0, 0] * math.sqrt(4 * math.pi)
    assert abs(Q - 1.0) < 1e-5
    # beyond the support: exactly Q / r (the second atom carries no charge)
    assert np.max(np.abs(h["v"][far] * ra[far] - Q)) < 1e-12
    assert np.max(np.abs(h["v"][far] - ref[far])) < 1e-5 / R_a
