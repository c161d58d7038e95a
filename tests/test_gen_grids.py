"""Seeded input generator: quadrature rules, partition weights, pruning, radial tables.

Pins are textbook integrals and invariants (no oracle code is involved)."""
import math

import numpy as np
import pytest
from scipy.special import sph_harm_y

import synth
from synth import instances as I


def test_becke_radial_rule_integrates_slater_density():
    # int_0^inf r^2 exp(-2r) dr = 2/2^3 = 1/4
    for n in (50, 75):
        r, w = synth.becke_radial(n)
        assert abs(np.sum(w * np.exp(-2.0 * r)) - 0.25) < 1e-10
    # int_0^inf r^2 exp(-r^2) dr = sqrt(pi)/4
    r, w = synth.becke_radial(75)
    assert abs(np.sum(w * np.exp(-r * r)) - math.sqrt(math.pi) / 4) < 1e-10


def _complex_ylm(l, m, u):
    th = np.arccos(np.clip(u[:, 2], -1, 1))
    ph = np.arctan2(u[:, 1], u[:, 0])
    return sph_harm_y(l, m, th, ph)


@pytest.mark.parametrize("rule,degree", [("gl110", 10), ("lobatto302", 24)])
def test_angular_rule_exactness(rule, degree):
    u, w = I.ANGULAR[rule]()
    assert len(w) == {"gl110": 110, "lobatto302": 302}[rule]
    assert np.allclose(np.linalg.norm(u, axis=1), 1.0, atol=1e-15)
    assert abs(w.sum() - 4 * np.pi) < 1e-13
    half = degree // 2
    worst = 0.0
    for l1 in range(half + 1):
        for m1 in range(-l1, l1 + 1):
            y1 = _complex_ylm(l1, m1, u)
            for l2 in range(half + 1):
                for m2 in range(-l2, l2 + 1):
                    y2 = _complex_ylm(l2, m2, u)
                    val = np.sum(w * y1 * np.conj(y2))
                    ref = 1.0 if (l1 == l2 and m1 == m2) else 0.0
                    worst = max(worst, abs(val - ref))
    assert worst < 1e-12
    # and it is *not* exact one degree beyond (guards against an accidentally denser rule)
    y = _complex_ylm(degree + 1, degree + 1, u)
    assert abs(np.sum(w * y)) > 1e-6


def _stratmann_bruteforce(p, atoms):
    D = np.linalg.norm(p[:, None, :] - atoms[None], axis=-1)
    R = np.linalg.norm(atoms[:, None] - atoms[None], axis=-1)
    np.fill_diagonal(R, 1.0)
    mu = (D[:, :, None] - D[:, None, :]) / R[None]
    nu = np.clip(mu / 0.64, -1, 1)
    g = (35 * nu - 35 * nu ** 3 + 21 * nu ** 5 - 5 * nu ** 7) / 16
    s = 0.5 * (1 - g)
    for b in range(atoms.shape[0]):
        s[:, b, b] = 1.0
    Pb = s.prod(2)
    return Pb / Pb.sum(1, keepdims=True)


def test_stratmann_partition_of_unity_and_bruteforce():
    rng = np.random.default_rng(3)
    atoms, _ = I.random_cluster(rng, 20, (1, 6, 8), 10.0)
    pts = rng.uniform(-3, 13, size=(3000, 3))
    ref = _stratmann_bruteforce(pts, atoms)
    tot = np.zeros(pts.shape[0])
    for a in range(atoms.shape[0]):
        wa = synth.stratmann_partition(pts, np.full(pts.shape[0], a, np.int32), atoms)
        assert np.all(wa >= 0.0) and np.all(wa <= 1.0)
        assert np.max(np.abs(wa - ref[:, a])) < 1e-13
        tot += wa
    assert np.max(np.abs(tot - 1.0)) < 1e-14


def test_stratmann_neighbour_limited_still_partition_of_unity():
    rng = np.random.default_rng(4)
    atoms, _ = I.random_cluster(rng, 40, (1, 8), 12.0)
    pts = rng.uniform(0, 12, size=(500, 3))
    tot = np.zeros(pts.shape[0])
    for a in range(atoms.shape[0]):
        tot += synth.stratmann_partition(pts, np.full(500, a, np.int32), atoms, max_neighbors=8)
    assert np.max(np.abs(tot - 1.0)) < 1e-14


def test_c1_counts_and_pruning_contributes_nothing(c1):
    # 3 atoms x 50 shells x 110 directions; the construction recipe fixes the kept count
    assert c1.meta["n_raw"] == 16500
    assert c1.meta["n_beyond_rc"] == 3160
    assert c1.n_points == 12894
    assert c1.n_basis == 24
    assert np.all(c1.pt_w > 0)
    # the dropped points carry zero partition weight or lie beyond rc of every atom
    pts, w, owner, meta, wgrid = I.build_grid(c1.atom_xyz, 50, "gl110", prune=False)
    d = np.min(np.linalg.norm(pts[:, None] - c1.atom_xyz[None], axis=-1), axis=1)
    kept = (w != 0) & (d <= I.RC + I.PRUNE_MARGIN)
    assert kept.sum() == c1.n_points
    assert np.all((w[~kept] == 0) | (d[~kept] > I.RC))


def test_kinetic_table_is_minus_half_laplacian():
    # K = -1/2 [R'' + 2R'/r - l(l+1) R/r^2], checked by high-order finite differences of R
    r = np.linspace(0.05, 9.0, 400)
    h = 1e-4
    for l, zeta in [(0, 0.7), (1, 2.3), (2, 5.1), (3, 0.31)]:
        R = lambda x: I.slater_cut_RK(l, zeta, x)[0]
        _, K = I.slater_cut_RK(l, zeta, r)
        d1 = (R(r - 2 * h) - 8 * R(r - h) + 8 * R(r + h) - R(r + 2 * h)) / (12 * h)
        d2 = (-R(r - 2 * h) + 16 * R(r - h) - 30 * R(r) + 16 * R(r + h) - R(r + 2 * h)) / (12 * h * h)
        Kfd = -0.5 * (d2 + 2 * d1 / r - l * (l + 1) * R(r) / r ** 2)
        assert np.max(np.abs(K - Kfd)) < 1e-6 * max(1.0, np.max(np.abs(K)))
    # R and K vanish at and beyond rc
    R, K = I.slater_cut_RK(1, 1.0, np.array([I.RC, I.RC + 1]))
    assert np.all(R == 0) and np.all(K == 0)


def test_seeded_determinism_and_roundtrip(tmp_path, c1):
    again = synth.make_instance("c1")
    assert np.array_equal(again.P, c1.P)
    assert np.array_equal(again.pt_w, c1.pt_w)
    path = str(tmp_path / "c1.npz")
    c1.save(path)
    back = synth.Instance.load(path)
    for f in ("atom_xyz", "pt_xyz", "pt_w", "v", "P", "shell_R", "shell_K", "shell_l"):
        assert np.array_equal(getattr(back, f), getattr(c1, f))
    assert back.rc == c1.rc and back.n_log == c1.n_log and back.max_batch == c1.max_batch


def test_density_matrix_and_potential(c1):
    P = c1.P
    assert np.array_equal(P, P.T)
    # v -> -Z 2/(sigma sqrt(pi)) at a nucleus of an isolated atom
    v0 = I.nuclear_potential(np.zeros((1, 3)), np.zeros((1, 3)), np.array([8]))
    assert abs(v0[0] + 8 * 2 / (0.3 * math.sqrt(math.pi))) < 1e-13
    # far away the smeared potential is the bare Coulomb potential
    v1 = I.nuclear_potential(np.array([[5.0, 0, 0]]), np.zeros((1, 3)), np.array([8]))
    assert abs(v1[0] + 8 / 5.0) < 1e-14


def test_cluster_geometry_rules():
    rng = np.random.default_rng(0)
    xyz, Z = I.random_cluster(rng, 64, (1, 6, 8), 20.0)
    d = np.linalg.norm(xyz[:, None] - xyz[None], axis=-1) + np.eye(64) * 99
    assert d.min() >= 1.8 and np.all((xyz >= 0) & (xyz < 20))
    assert set(np.unique(Z)) <= {1, 6, 8}
    xyz, Z = I.grown_molecule(rng, 30)
    d = np.linalg.norm(xyz[:, None] - xyz[None], axis=-1) + np.eye(30) * 99
    assert d.min() >= 1.8 - 1e-12
    assert np.all(d.min(axis=1) <= 2.9 + 1e-12)
