"""Hartree potential through the C ABI against the oracle's multipole expansion (the same
algorithm: node multipoles, cubic splines in Becke's angle, Gauss-Legendre radial integrals),
and against the closed form of a Gaussian charge.  Bars: 1e-11 of max|v_H| (FP64, a handful of
transcendental evaluations and splines per term); the closed form at the oracle's own
discretisation accuracy (5e-6 at 75 radial nodes)."""
import math

import numpy as np
import pytest
import torch
from scipy.special import erf

import synth
from oracle.hartree import hartree
from paper_2208_12335_amd import AimsError, AimsGrid

pytestmark = pytest.mark.gpu


def _run(inst, n, gpu, l_max):
    g = AimsGrid(inst, device=gpu.index)
    g.set_hartree_grid([synth.radial_shells(inst)], l_max=l_max)
    v, E = g.hartree(torch.from_numpy(n).to(gpu))
    return g, v.cpu().numpy(), E.cpu().numpy()


@pytest.mark.parametrize("l_max", [0, 2, 6])
def test_hartree_matches_oracle_on_a_cluster(gpu, l_max):
    """A 10-atom l<=3 cluster with the density of its occupied core-Hamiltonian orbitals."""
    from oracle import GridOracle
    from oracle.scf import density_matrix
    inst = synth.make_instance("c2", n_atoms=10, box=7.5, seed=4)
    o = GridOracle(inst)
    H, S = o.integrate_h(inst.v)
    n = o.density(density_matrix(H, S, float(np.sum(inst.atom_Z)))["P"])["n"]
    _, v, E = _run(inst, n, gpu, l_max)
    node, K, rm = synth.radial_shells(inst)
    ref = hartree(inst, n, node, K, rm, l_max)
    err = np.max(np.abs(v - ref["v"])) / np.max(np.abs(ref["v"]))
    print(f"[hartree] cluster l_max={l_max}: {err:.1e}, E_H {E[0]:.10f} vs {ref['E_H']:.10f}",
          flush=True)
    assert err <= 1e-11
    assert abs(E[0] - ref["E_H"]) <= 1e-11 * abs(ref["E_H"])


def test_hartree_gaussian_closed_form_and_grouped(gpu):
    """Two molecules in one handle: a Gaussian charge on the first (closed form erf(sqrt(a) r)/r
    on a one-atom grid) and an off-centre charge on the second (the oracle)."""
    def f(r):
        e = np.exp(-r * r)
        return e, -0.5 * (4 * r * r - 6) * e
    m1 = synth.custom_instance(np.array([[0.2, -0.1, 0.3]]), [0], [[0]], [f], n_log=200,
                               n_radial=75, angular="gl110")
    m2 = synth.custom_instance(np.array([[0.0, 0.0, 0.0], [0.0, 0.4, 1.3]]), [0, 1], [[0], [0]],
                               [f, f], n_log=200, n_radial=60, angular="gl110")
    a = 1.7
    n1 = (a / math.pi) ** 1.5 * np.exp(-a * ((m1.pt_xyz - m1.atom_xyz[0]) ** 2).sum(1))
    c = np.array([0.1, 0.2, 0.5])
    n2 = (2.0 / math.pi) ** 1.5 * np.exp(-2.0 * ((m2.pt_xyz - c) ** 2).sum(1))
    g = AimsGrid([m1, m2], device=gpu.index)
    g.set_hartree_grid([synth.radial_shells(m1), synth.radial_shells(m2)], l_max=4)
    v, E = g.hartree(torch.from_numpy(np.concatenate([n1, n2])).to(gpu))
    v, E = v.cpu().numpy(), E.cpu().numpy()
    r = np.linalg.norm(m1.pt_xyz - m1.atom_xyz[0], axis=1)
    assert np.max(np.abs(v[:m1.n_points] - erf(math.sqrt(a) * r) / r)) < 5e-6
    assert abs(E[0] - math.sqrt(a / (2 * math.pi))) < 2e-6
    node, K, rm = synth.radial_shells(m2)
    ref = hartree(m2, n2, node, K, rm, 4)
    err = np.max(np.abs(v[m1.n_points:] - ref["v"])) / np.max(np.abs(ref["v"]))
    print(f"[hartree] grouped second system: {err:.1e}", flush=True)
    assert err <= 1e-11
    assert abs(E[1] - ref["E_H"]) <= 1e-11 * abs(ref["E_H"])
    # errors raised before any work
    with pytest.raises(AimsError) as e:
        g.set_hartree_grid([synth.radial_shells(m1), synth.radial_shells(m2)], l_max=7)
    assert e.value.status == -5
    h2 = AimsGrid(m1, device=gpu.index)
    with pytest.raises(AimsError) as e:
        h2.hartree(torch.zeros(m1.n_points, dtype=torch.float64, device=gpu))
    assert e.value.status == -1


def test_hartree_exterior_beyond_support(gpu):
    """Two atoms 9 bohr apart, the charge on the first atom's points: the second atom's far
    points lie beyond the first atom's edge node and take the exterior form (Q / r at l_max 0);
    every point against the oracle at l_max 0 and 6."""
    def f(r):
        e = np.exp(-r * r)
        return e, -0.5 * (4 * r * r - 6) * e
    A, B = np.array([0.0, 0.0, 0.0]), np.array([0.0, 0.0, 9.0])
    inst = synth.custom_instance(np.array([A, B]), [0, 1], [[0], [0]], [f, f], n_log=200,
                                 n_radial=75, angular="lobatto302")
    own_a = np.asarray(inst.pt_atom) == 0
    n = (2.0 / math.pi) ** 1.5 * np.exp(-2.0 * ((inst.pt_xyz - A) ** 2).sum(1)) * own_a
    node, K, rm = synth.radial_shells(inst)
    from oracle.hartree import edge_nodes, radial_nodes
    R_a = radial_nodes(K, rm)[1][edge_nodes(inst, node, K)[0]]
    ra = np.linalg.norm(inst.pt_xyz - A, axis=1)
    far = ra >= R_a
    assert far.sum() > 100
    for l_max in (0, 6):
        _, v, E = _run(inst, n, gpu, l_max)
        ref = hartree(inst, n, node, K, rm, l_max)
        err = np.max(np.abs(v - ref["v"])) / np.max(np.abs(ref["v"]))
        print(f"[hartree] beyond the support, l_max={l_max}: {err:.1e} ({far.sum()} far points)",
              flush=True)
        assert err <= 1e-11
        assert abs(E[0] - ref["E_H"]) <= 1e-11 * abs(ref["E_H"])
        if l_max == 0:
            Q = ref["q"][0, 0] * math.sqrt(4 * math.pi)
            assert np.max(np.abs(v[far] * ra[far] - Q)) < 1e-12


def test_hartree_full_size_sampled(gpu):
    """The 64-atom cluster at its full size (1.1M points, l_max = 6, the benchmark's Hartree
    step): v_H at 400 sampled points and E_H against the oracle (node multipoles and radial
    solve over every point, the potential at the sampled ones)."""
    from oracle.hartree import edge_nodes, multipoles, potential_at, radial_potentials
    inst = synth.make_instance("c2", seed=0)
    g = AimsGrid(inst, device=gpu.index)
    node, K, rm = synth.radial_shells(inst)
    g.set_hartree_grid([(node, K, rm)], l_max=6)
    P = torch.from_numpy(inst.P).to(gpu).reshape(-1)
    n, _ = g.update_density(P, torch.from_numpy(inst.v).to(gpu))
    v, E = g.hartree(n)
    nn, v = n.cpu().numpy(), v.cpu().numpy()
    rho = multipoles(inst, nn, node, K, rm, 6)
    pot = radial_potentials(rho, K, rm, 6, edge_nodes(inst, node, K))
    idx = np.random.default_rng(7).choice(inst.n_points, 400, replace=False)
    ref = potential_at(inst.pt_xyz[idx], inst.atom_xyz, pot, K, rm, 6)
    err = np.max(np.abs(v[idx] - ref)) / np.max(np.abs(ref))
    E_ref = 0.5 * float(np.sum(inst.pt_w * nn * v))      # E_H of the GPU potential, summed on the host
    print(f"[hartree] c2 full size: sampled v_H {err:.1e}, E_H {E.cpu().numpy()[0]:.10f}", flush=True)
    assert err <= 1e-11
    assert abs(E.cpu().numpy()[0] - E_ref) <= 1e-12 * abs(E_ref)
