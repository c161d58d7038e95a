"""Pins of the oracle's moving-grid energy gradient (oracle/forces.py).

* The energy it differentiates equals the plain quadrature on the generator's grid (whose
  partition weights and nuclear potential come from separate code): the torch re-statement
  of the partition and of the potential is checked by value.
* Translation invariance: moving every atom (and so every grid) by the same vector leaves E
  unchanged, so the gradients sum to zero.
* Finite differences: E on grids rebuilt from scratch at displaced atoms (the generator's own
  construction), Richardson-extrapolated central differences, against the gradient along one
  random direction per atom.  Bar: 1e-6 absolute (Ha/bohr) plus 1e-6 relative."""
import numpy as np
import pytest

import synth
from oracle import GridOracle
from oracle.forces import moving_grid_gradient


def _systems():
    c1 = synth.make_instance("c1")
    mol = synth.make_molecule_set(n_mol=1, seed=3, n_min=5, n_max=5)[0]
    return [c1, mol]


@pytest.fixture(scope="module", params=[0, 1], ids=["triatomic", "grown5"])
def system(request):
    inst = _systems()[request.param]
    o = GridOracle(inst)
    E, G = moving_grid_gradient(o, inst.P)
    return inst, o, E, G


def test_energy_matches_plain_quadrature(system):
    inst, o, E, G = system
    E_plain = o.energy(inst.P, inst.v)
    assert abs(E - E_plain) <= 1e-12 * max(1.0, abs(E_plain)), (E, E_plain)


def test_translation_invariance(system):
    inst, o, E, G = system
    tot = G.sum(axis=0)
    assert np.max(np.abs(tot)) <= 1e-10 * max(1.0, np.max(np.abs(G))), (tot, np.max(np.abs(G)))
    assert np.max(np.abs(G)) > 1e-3          # the gradient is not trivially zero


def test_finite_differences_on_rebuilt_grids(system):
    inst, o, E, G = system
    rng = np.random.default_rng(11)
    h = 1e-3

    def energy(xyz):
        r = synth.regrid(inst, xyz)
        return GridOracle(r).energy(inst.P, r.v)

    for a in range(inst.n_atoms):
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        e = np.zeros_like(inst.atom_xyz)
        e[a] = u
        d1 = (energy(inst.atom_xyz + h * e) - energy(inst.atom_xyz - h * e)) / (2 * h)
        d2 = (energy(inst.atom_xyz + 2 * h * e) - energy(inst.atom_xyz - 2 * h * e)) / (4 * h)
        fd = (4 * d1 - d2) / 3
        an = float(G[a] @ u)
        assert abs(an - fd) <= 1e-6 + 1e-6 * abs(an), (a, an, fd)
