"""The FP64 oracle against closed forms and library routines.

Each case is chosen so that a plausible slip in the oracle (a wrong harmonic sign or
normalisation, a dropped kinetic term, a wrong radial weight, a transposed operand) fails it."""
import math

import numpy as np
import pytest
from scipy.special import erf, gamma, sph_harm_y

import synth
from oracle import GridOracle, real_ylm
from oracle.harmonics import lm_list, real_ylm_grad
from oracle.radial import RadialSplines, knots


# ---------------------------------------------------------------------------------------------
# real spherical harmonics
# ---------------------------------------------------------------------------------------------
def _scipy_real(u):
    """Real harmonics from scipy's complex ones: Y_l,m>0 = sqrt2 (-1)^m Re Y_l^m,
    Y_l,m<0 = sqrt2 (-1)^m Im Y_l^|m|, Y_l0 = Y_l^0 (removes the Condon-Shortley phase)."""
    th = np.arccos(np.clip(u[:, 2], -1, 1))
    ph = np.arctan2(u[:, 1], u[:, 0])
    cols = []
    for l, m in lm_list():
        c = sph_harm_y(l, abs(m), th, ph)
        if m > 0:
            cols.append(math.sqrt(2) * (-1) ** m * c.real)
        elif m < 0:
            cols.append(math.sqrt(2) * (-1) ** m * c.imag)
        else:
            cols.append(c.real)
    return np.stack(cols, -1)


def test_ylm_matches_scipy():
    rng = np.random.default_rng(0)
    u = rng.standard_normal((4000, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    u = np.vstack([u, [[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, 1, 0]]])
    assert np.max(np.abs(real_ylm(u) - _scipy_real(u))) < 3e-14


def test_ylm_low_order_explicit_forms():
    # l = 1 is (y, z, x) times sqrt(3/(4 pi)); Y_20 = sqrt(5/(16 pi)) (3z^2 - 1);
    # Y_3,-3 = sqrt(35/(32 pi)) y (3x^2 - y^2)
    rng = np.random.default_rng(1)
    u = rng.standard_normal((50, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    x, y, z = u.T
    Y = real_ylm(u)
    c1 = math.sqrt(3 / (4 * math.pi))
    assert np.allclose(Y[:, 1:4], c1 * np.stack([y, z, x], -1), atol=1e-15, rtol=0)
    assert np.allclose(Y[:, 6], math.sqrt(5 / (16 * math.pi)) * (3 * z * z - 1), atol=1e-15)
    assert np.allclose(Y[:, 9], math.sqrt(35 / (32 * math.pi)) * y * (3 * x * x - y * y), atol=1e-15)


def test_ylm_gradient_by_finite_differences():
    rng = np.random.default_rng(2)
    u = rng.standard_normal((20, 3))
    G = real_ylm_grad(u)          # gradient of the homogeneous polynomial at u (not normalised)
    h = 1e-6
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        fd = (real_ylm(u + e) - real_ylm(u - e)) / (2 * h)
        assert np.max(np.abs(fd - G[:, :, c])) < 1e-7


# ---------------------------------------------------------------------------------------------
# radial splines
# ---------------------------------------------------------------------------------------------
def test_spline_interpolates_knots_and_approximates_function(c1):
    spl = RadialSplines(c1)
    rk = knots(c1.n_log, c1.r0, c1.rc)
    off = c1.species_shell_offset()
    for s in range(len(c1.species_nshell)):
        Rv, Kv = spl.eval(s, rk[:-1])
        assert np.allclose(Rv, c1.shell_R[off[s]:off[s + 1], :-1].T, rtol=1e-13, atol=1e-15)
        assert np.allclose(Kv, c1.shell_K[off[s]:off[s + 1], :-1].T, rtol=1e-13, atol=1e-12)
        # between knots the natural spline is O(h^4) close to the analytic function
        mid = np.sqrt(rk[1:-1] * rk[2:])[40:-5]
        Rv, _ = spl.eval(s, mid)
        for j, k in enumerate(range(off[s], off[s + 1])):
            Ra, _ = synth.instances.slater_cut_RK(int(c1.shell_l[k]), float(c1.shell_zeta[k]), mid)
            assert np.max(np.abs(Rv[:, j] - Ra)) < 2e-5 * np.max(np.abs(Ra))
    # zero at and beyond rc
    Rv, Kv = spl.eval(0, np.array([c1.rc, c1.rc * 1.5]))
    assert np.all(Rv == 0) and np.all(Kv == 0)


def test_spline_natural_end_conditions(c1):
    spl = RadialSplines(c1)
    for s in range(len(c1.species_nshell)):
        d2 = spl.R[s](spl.s[[0, -1]], 2)
        assert np.max(np.abs(d2)) < 1e-9 * max(1.0, np.max(np.abs(c1.shell_R)))


def test_spline_torch_twin_matches():
    import torch
    inst = synth.make_instance("c1")
    spl = RadialSplines(inst)
    r = np.concatenate([np.geomspace(1e-5, 9.44, 500), [9.45, 12.0]])
    for s in range(len(inst.species_nshell)):
        R1, K1 = spl.eval(s, r)
        R2, K2 = spl.eval_torch(s, torch.from_numpy(r))
        assert np.max(np.abs(R1 - R2.numpy())) < 1e-14 * np.max(np.abs(R1))
        assert np.max(np.abs(K1 - K2.numpy())) < 1e-14 * np.max(np.abs(K1))


# ---------------------------------------------------------------------------------------------
# closed-form integrals
# ---------------------------------------------------------------------------------------------
def _gauss_RK(l, a):
    """R = r^l exp(-a r^2) and K = -1/2[R'' + 2R'/r - l(l+1)R/r^2] = R a [(2l+3) - 2 a r^2]."""
    def f(r):
        R = r ** l * np.exp(-a * r * r)
        return R, R * a * ((2 * l + 3) - 2 * a * r * r)
    return f


GAUSS_PAIRS = [(0.6, 2.2), (1.1, 0.45)]


def _erf_potential(p):
    r = np.linalg.norm(p, axis=1)
    return -erf(r / 0.3) / r


@pytest.fixture(scope="module")
def one_centre_gauss():
    shells, funcs = [], []
    for l in range(4):
        for a in GAUSS_PAIRS[l % 2]:
            shells.append(l)
            funcs.append(_gauss_RK(l, a))
    inst = synth.custom_instance(np.zeros((1, 3)), [0], [shells], funcs, n_log=1000,
                                 n_radial=75, angular="lobatto302",
                                 potential=_erf_potential)
    return inst, shells


def test_one_centre_gaussian_overlap_and_kinetic(one_centre_gauss):
    inst, shells = one_centre_gauss
    o = GridOracle(inst)
    T, S = o.integrate_h(np.zeros(inst.n_points))
    # function index of (shell k, m)
    idx, k0 = {}, 0
    for k, l in enumerate(shells):
        for m in range(-l, l + 1):
            idx[(k, m)] = k0
            k0 += 1
    worst_S = worst_T = 0.0
    for l in range(4):
        ka, kb = 2 * l, 2 * l + 1
        a, b = GAUSS_PAIRS[l % 2]
        g = a + b
        S_ref = gamma(l + 1.5) / (2 * g ** (l + 1.5))
        T_ref = S_ref * (2 * l + 3) * a * b / g
        for m in range(-l, l + 1):
            i, j = idx[(ka, m)], idx[(kb, m)]
            worst_S = max(worst_S, abs(S[i, j] / S_ref - 1))
            worst_T = max(worst_T, abs(T[i, j] / T_ref - 1), abs(T[j, i] / T_ref - 1))
            # different m of the same shells are orthogonal
            for m2 in range(-l, l + 1):
                if m2 != m:
                    assert abs(S[i, idx[(kb, m2)]]) < 1e-12
    assert worst_S < 1e-7
    assert worst_T < 1e-6
    # functions of different l never overlap on an exact angular rule
    assert abs(S[idx[(0, 0)], idx[(2, 0)]]) < 1e-13


def test_one_centre_erf_nuclear_attraction(one_centre_gauss):
    # V = int e^{-a r^2} e^{-b r^2} Y00^2 (-erf(r/sigma)/r) d^3r = -1/(2 g sigma sqrt(g + sigma^-2))
    inst, shells = one_centre_gauss
    o = GridOracle(inst)
    H, _ = o.integrate_h(inst.v, want_S=False)
    T, _ = o.integrate_h(np.zeros(inst.n_points), want_S=False)
    V = H - T
    a, b = GAUSS_PAIRS[0]
    g, sig = a + b, 0.3
    V_ref = -1.0 / (2 * g * sig * math.sqrt(g + sig ** -2))
    assert abs(V[0, 1] / V_ref - 1) < 1e-7
    assert abs(V[0, 1] - V[1, 0]) < 1e-14 * np.max(np.abs(H))


def test_two_centre_s_gaussians_exercise_partition():
    a, b = 0.9, 1.3
    RB = np.array([0.5, -0.7, 1.1])
    Rab2 = float(RB @ RB)
    inst = synth.custom_instance(np.array([[0.0, 0, 0], RB]), [0, 1], [[0], [0]],
                                 [_gauss_RK(0, a), _gauss_RK(0, b)], n_log=1000, n_radial=75,
                                 angular="lobatto302")
    o = GridOracle(inst)
    T, S = o.integrate_h(np.zeros(inst.n_points))
    g = a + b
    S_ref = (1 / (4 * math.pi)) * (math.pi / g) ** 1.5 * math.exp(-a * b * Rab2 / g)
    T_ref = (a * b / g) * (3 - 2 * a * b * Rab2 / g) * S_ref
    assert abs(S[0, 1] / S_ref - 1) < 1e-6
    assert abs(T[0, 1] / T_ref - 1) < 1e-5
    assert abs(T[1, 0] / T_ref - 1) < 1e-5


@pytest.mark.parametrize("n_log,n_radial,tol", [(200, 50, 1e-6), (1000, 75, 1e-9)])
def test_hydrogen_1s_energy(n_log, n_radial, tol):
    # R = e^{-r}, K = -1/2 (1 - 2/r) e^{-r}, v = -1/r: <T + V>/<S> = -1/2 hartree
    def f(r):
        e = np.exp(-r)
        return e, -0.5 * (1 - 2 / r) * e
    inst = synth.custom_instance(np.zeros((1, 3)), [0], [[0]], [f], n_log=n_log, rc=40.0,
                                 n_radial=n_radial, angular="gl110",
                                 potential=lambda p: -1.0 / np.linalg.norm(p, axis=1))
    o = GridOracle(inst)
    H, S = o.integrate_h(inst.v)
    assert abs(H[0, 0] / S[0, 0] + 0.5) < tol
    # the same number through the density path: P = 1/S gives N = 1 and E = -1/2
    d = o.density(np.array([[1.0 / S[0, 0]]]), inst.v)
    assert abs(d["N"] - 1.0) < 1e-12
    assert abs(d["E_V"] + d["E_T"] + 0.5) < tol
