"""Pins of the oracle's density-matrix step (oracle/scf.py) against closed forms, the
variational principle and invariants of the generalised eigenproblem; CPU only."""
import math

import numpy as np
import pytest

import synth
from oracle import GridOracle
from oracle.scf import density_matrix, occupations, symmetric_part


def _two_level(a, b, c, s):
    """Lowest root and S-normalised vector of [[a,b],[b,c]] x = lam [[1,s],[s,1]] x from the
    quadratic (1 - s^2) lam^2 - (a + c - 2 b s) lam + (a c - b^2) = 0."""
    A = 1.0 - s * s
    B = -(a + c - 2.0 * b * s)
    C = a * c - b * b
    lam = (-B - math.sqrt(B * B - 4.0 * A * C)) / (2.0 * A)
    v = np.array([-(b - lam * s), a - lam])
    v /= math.sqrt(v[0] ** 2 + v[1] ** 2 + 2.0 * s * v[0] * v[1])
    return lam, v


@pytest.mark.parametrize("a,b,c,s", [(-1.0, -0.4, 0.3, 0.25), (0.2, 0.7, -0.5, -0.6)])
def test_two_level_closed_form(a, b, c, s):
    lam, v = _two_level(a, b, c, s)
    S = np.array([[1.0, s], [s, 1.0]])
    for d in (0.0, 0.37):                     # an antisymmetric part of H must not matter
        H = np.array([[a, b + d], [b - d, c]])
        r = density_matrix(H, S, 2.0)
        assert abs(r["eps"][0] - lam) < 1e-14
        assert np.allclose(r["P"], 2.0 * np.outer(v, v), atol=1e-13, rtol=0)
        assert np.allclose(r["f"], [2.0, 0.0])


def _slater_s(zeta):
    # R = e^{-zeta r}, K = -1/2 (R'' + 2 R'/r) = -1/2 (zeta^2 - 2 zeta / r) e^{-zeta r}
    return lambda r: (np.exp(-zeta * r), -0.5 * (zeta * zeta - 2.0 * zeta / r) * np.exp(-zeta * r))


def _slater_rs(zeta):
    # R = r e^{-zeta r}, K = -1/2 (zeta^2 r - 4 zeta + 2 / r) e^{-zeta r}
    return lambda r: (r * np.exp(-zeta * r),
                      -0.5 * (zeta * zeta * r - 4.0 * zeta + 2.0 / r) * np.exp(-zeta * r))


def hydrogen_multi_s(n_log=1000, n_radial=75):
    """Hydrogen atom, v = -1/r, in four s functions whose span holds the exact 1s state e^{-r}."""
    shells = [_slater_s(1.0), _slater_s(1.8), _slater_s(0.8), _slater_rs(1.3)]
    return synth.custom_instance(np.zeros((1, 3)), [0], [[0, 0, 0, 0]], shells, n_log=n_log,
                                 rc=40.0, n_radial=n_radial, angular="gl110",
                                 potential=lambda p: -1.0 / np.linalg.norm(p, axis=1))


def test_hydrogen_eigenproblem_closes_the_loop():
    """The exact ground state is in the span: the lowest generalised eigenvalue is -1/2; the
    next is a variational upper bound of the exact 2s level -1/8.  P of one electron, fed
    back through the density path, gives N = 1 and E = E_V + E_T = -1/2."""
    inst = hydrogen_multi_s()
    o = GridOracle(inst)
    H, S = o.integrate_h(inst.v)
    r = density_matrix(H, S, 1.0)
    assert abs(r["eps"][0] + 0.5) < 1e-8
    assert r["eps"][1] > -0.125 - 1e-8
    assert np.allclose(r["f"], [1.0, 0.0, 0.0, 0.0])
    d = o.density(r["P"], inst.v)
    assert abs(d["N"] - 1.0) < 1e-10
    assert abs(d["E_V"] + d["E_T"] + 0.5) < 1e-8
    # the ground state is e^{-r} alone: the rest of the vector is small in the S-norm (of the
    # order of the square root of the quadrature's eigenvalue error; S is ill-conditioned)
    c = r["C"][:, 0]
    d = c.copy()
    d[0] = 0.0
    assert math.sqrt(d @ S @ d) < 5e-5 * math.sqrt(c @ S @ c)


def _random_problem(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    S = A @ A.T / n + 0.5 * np.eye(n)
    Hs = rng.standard_normal((n, n))
    return Hs + Hs.T + 0.3 * (rng.standard_normal((n, n))), S


def test_invariants_aufbau():
    H, S = _random_problem(12, 1)
    r = density_matrix(H, S, 6.0)
    P, C, eps, f = r["P"], r["C"], r["eps"], r["f"]
    assert np.allclose(C.T @ S @ C, np.eye(12), atol=1e-12)
    assert np.allclose(symmetric_part(H) @ C, S @ C * eps[None, :], atol=1e-11)
    assert np.allclose(P, P.T, atol=1e-14)
    assert abs(np.trace(P @ S) - 6.0) < 1e-12
    assert np.allclose(P @ S @ P, 2.0 * P, atol=1e-11)          # closed-shell idempotency
    assert abs(np.sum(P * symmetric_part(H)) - np.sum(f * eps)) < 1e-11
    assert np.all(np.diff(eps) >= 0)
    assert r["eps"][2] < r["mu"] < r["eps"][3]


def test_invariants_fermi_and_limits():
    H, S = _random_problem(12, 2)
    r0 = density_matrix(H, S, 7.0)                  # odd: the 4th state holds one electron
    assert np.allclose(r0["f"][:5], [2, 2, 2, 1, 0])
    for kT in (0.5, 0.05):
        r = density_matrix(H, S, 7.0, kT)
        assert abs(r["f"].sum() - 7.0) < 1e-12
        assert np.all((r["f"] >= 0) & (r["f"] <= 2)) and np.all(np.diff(r["f"]) <= 1e-15)
        assert abs(np.trace(r["P"] @ S) - 7.0) < 1e-11
    # a tiny smearing reproduces aufbau when the Fermi level sits in a gap
    ra = density_matrix(H, S, 8.0)
    gap = ra["eps"][4] - ra["eps"][3]
    assert gap > 1e-3
    rs = density_matrix(H, S, 8.0, kT=gap * 1e-3)
    assert np.allclose(rs["P"], ra["P"], atol=1e-10)


def test_empty_and_full():
    H, S = _random_problem(9, 3)
    assert np.array_equal(density_matrix(H, S, 0.0)["P"], np.zeros((9, 9)))
    full = density_matrix(H, S, 18.0)["P"]
    assert np.allclose(full, 2.0 * np.linalg.inv(S), atol=1e-11)
    with pytest.raises(ValueError):
        occupations(np.zeros(3), 7.0)
