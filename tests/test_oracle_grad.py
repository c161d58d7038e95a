"""The oracle's derivatives against central finite differences of its own energy.

E = sum_p w v n + sum_p w sum_ij P_ij phi_i tphi_j.  Basis centres move (grid, weights and v
stay), h = 1e-4 bohr; E is linear in P and v, so finite differences there are exact."""
import numpy as np
import pytest

import synth
from oracle import GridOracle


def _fd_R(inst, atoms, h=1e-4):
    out = np.zeros((len(atoms), 3))
    for k, a in enumerate(atoms):
        for c in range(3):
            Xp = inst.atom_xyz.copy()
            Xp[a, c] += h
            Xm = inst.atom_xyz.copy()
            Xm[a, c] -= h
            Ep = GridOracle(inst.moved(Xp)).energy(inst.P, inst.v)
            Em = GridOracle(inst.moved(Xm)).energy(inst.P, inst.v)
            out[k, c] = (Ep - Em) / (2 * h)
    return out


def test_c1_position_gradient_vs_fd(c1, c1_oracle):
    g = c1_oracle.gradient(c1.P, c1.v)
    fd = _fd_R(c1, [0, 1, 2])
    assert np.max(np.abs(g["dE_dR"] - fd)) < 1e-6
    # the analytic basis-gradient formula agrees with automatic differentiation
    gc = c1_oracle.gradient_closed_form(c1.P, c1.v)
    assert np.max(np.abs(gc - g["dE_dR"])) < 1e-10 * np.max(np.abs(gc))


def test_small_cluster_position_gradient_vs_fd():
    inst = synth.make_instance("c2", n_atoms=5, box=5.0, seed=2)
    o = GridOracle(inst)
    atoms = [1, 3]
    g = o.gradient(inst.P, inst.v, atoms=atoms)
    fd = _fd_R(inst, atoms)
    assert np.max(np.abs(g["dE_dR"][atoms] - fd)) < 1e-6
    gc = o.gradient_closed_form(inst.P, inst.v)
    assert np.max(np.abs(gc[atoms] - g["dE_dR"][atoms])) < 1e-10 * np.max(np.abs(gc))
    # restricting to a subset of atoms gives the same rows as the full gradient
    gfull = o.gradient(inst.P, inst.v)["dE_dR"]
    assert np.max(np.abs(gfull[atoms] - g["dE_dR"][atoms])) < 1e-11 * np.max(np.abs(gfull))
    # and so does the closed form restricted to them (points near them, their columns only)
    gr = o.gradient_closed_form(inst.P, inst.v, atoms=atoms)
    assert np.max(np.abs(gr[atoms] - gfull[atoms])) < 1e-10 * np.max(np.abs(gfull))
    assert np.all(gr[[0, 2, 4]] == 0.0)


def test_density_matrix_and_potential_gradients_exact(c1, c1_oracle):
    g = c1_oracle.gradient(c1.P, c1.v)
    E0 = g["E"]
    rng = np.random.default_rng(0)
    for (i, j) in [(0, 0), (3, 17), (17, 3), (22, 5)]:
        P = c1.P.copy()
        P[i, j] += 1e-3                          # independent-entry convention
        E1 = c1_oracle.energy(P, c1.v)
        assert abs((E1 - E0) / 1e-3 - g["dE_dP"][i, j]) < 1e-9 * max(1, abs(g["dE_dP"][i, j]))
    for p in rng.choice(c1.n_points, 5, replace=False):
        v = c1.v.copy()
        v[p] += 0.5
        E1 = c1_oracle.energy(c1.P, v)
        assert abs((E1 - E0) / 0.5 - g["dE_dv"][p]) < 1e-10 * max(1e-3, abs(g["dE_dv"][p]))
