"""The FP64 oracle against invariants, special cases and brute force."""
import numpy as np
import pytest

import synth
from oracle import GridOracle
from oracle.integrate import phi_bruteforce


@pytest.fixture(scope="module")
def c1_results(c1, c1_oracle):
    dens = c1_oracle.density(c1.P, c1.v)
    H, S = c1_oracle.integrate_h(c1.v)
    return dens, H, S


def test_electron_count_equals_trace_PS(c1, c1_results):
    dens, H, S = c1_results
    trPS = float(np.sum(c1.P * S))
    assert abs(dens["N"] - trPS) < 1e-12 * abs(trPS)
    # and the energy equals tr(P H): the density path and the H path agree
    trPH = float(np.sum(c1.P * H))
    assert abs(dens["E_V"] + dens["E_T"] - trPH) < 1e-12 * abs(trPH)


def test_symmetry_of_S_and_V(c1, c1_oracle, c1_results):
    _, H, S = c1_results
    T, _ = c1_oracle.integrate_h(np.zeros(c1.n_points), want_S=False)
    V = H - T
    assert np.max(np.abs(S - S.T)) < 1e-15 * np.max(np.abs(S)) * 10
    assert np.max(np.abs(V - V.T)) < 1e-13 * np.max(np.abs(V))
    # T is not symmetric on a finite grid, but close to it (quadrature diagnostic)
    asym = np.max(np.abs(T - T.T)) / np.max(np.abs(T))
    assert 0 < asym < 1e-2


def test_special_cases(c1, c1_oracle, c1_results):
    _, H, S = c1_results
    nb = c1.n_basis
    i = 7
    P1 = np.zeros((nb, nb))
    P1[i, i] = 1.0
    d = c1_oracle.density(P1, c1.v)
    Phi, _, cols = c1_oracle.basis_values(c1.pt_xyz, atoms=np.arange(c1.n_atoms))
    assert np.max(np.abs(d["n"] - Phi[:, i] ** 2)) < 1e-15 * np.max(Phi[:, i] ** 2) * 10
    assert abs(d["N"] - S[i, i]) < 1e-13 * S[i, i]
    # constant potential: H(c) - H(0) = c S
    T, _ = c1_oracle.integrate_h(np.zeros(c1.n_points), want_S=False)
    Hc, _ = c1_oracle.integrate_h(np.full(c1.n_points, 2.5), want_S=False)
    assert np.max(np.abs(Hc - T - 2.5 * S)) < 1e-13 * np.max(np.abs(Hc))
    # empty density matrix
    d0 = c1_oracle.density(np.zeros((nb, nb)), c1.v)
    assert np.all(d0["n"] == 0) and d0["N"] == 0 and d0["E_V"] == 0 and d0["E_T"] == 0


def test_translation_invariance(c1, c1_results):
    dens, H, S = c1_results
    sh = c1.translated([0.3, -1.1, 2.7])
    o = GridOracle(sh)
    d2 = o.density(sh.P, sh.v)
    H2, S2 = o.integrate_h(sh.v)
    assert np.max(np.abs(d2["n"] - dens["n"])) < 1e-10 * np.max(np.abs(dens["n"]))
    assert np.max(np.abs(H2 - H)) < 1e-10 * np.max(np.abs(H))
    assert np.max(np.abs(S2 - S)) < 1e-10 * np.max(np.abs(S))


def test_chunked_screened_equals_bruteforce(c1, c1_oracle):
    rng = np.random.default_rng(5)
    sel = rng.choice(c1.n_points, 12, replace=False)
    pts = c1.pt_xyz[sel]
    pts = np.vstack([pts, [[0.0, 0.0, 12.0]]])            # beyond rc of every atom
    Phi, _, cols = c1_oracle.basis_values(pts, atoms=np.arange(c1.n_atoms))
    bf = np.array([phi_bruteforce(c1, p) for p in pts])
    assert np.array_equal(cols, np.arange(c1.n_basis))
    assert np.max(np.abs(Phi - bf)) < 5e-15 * max(1.0, np.max(np.abs(bf)))
    assert np.all(bf[-1] == 0)
    # n from the brute-force values
    n_bf = np.einsum("pi,ij,pj->p", bf[:-1], c1.P, bf[:-1])
    d = c1_oracle.density(c1.P, c1.v, points=sel)
    assert np.max(np.abs(d["n"] - n_bf)) < 1e-13 * np.max(np.abs(n_bf))


def test_chunk_size_independence(c1, c1_results):
    dens, H, S = c1_results
    o = GridOracle(c1, chunk=333)
    d2 = o.density(c1.P, c1.v)
    H2, S2 = o.integrate_h(c1.v)
    assert np.max(np.abs(d2["n"] - dens["n"])) < 1e-13 * np.max(np.abs(dens["n"]))
    assert np.max(np.abs(H2 - H)) < 1e-13 * np.max(np.abs(H))
    assert abs(d2["E_T"] - dens["E_T"]) < 1e-12 * abs(dens["E_T"])


def test_small_cluster_c2_rules():
    # a 6-atom cluster with the l <= 3 basis and the 302-point angular grid
    inst = synth.make_instance("c2", n_atoms=6, box=6.0)
    o = GridOracle(inst)
    d = o.density(inst.P, inst.v)
    H, S = o.integrate_h(inst.v)
    assert abs(d["N"] - np.sum(inst.P * S)) < 1e-12 * abs(d["N"])
    assert abs(d["E_V"] + d["E_T"] - np.sum(inst.P * H)) < 1e-12 * abs(d["E_V"] + d["E_T"])
    ev = np.linalg.eigvalsh(S)
    assert ev.min() > 0       # the quadrature overlap of a non-degenerate basis is positive definite
