"""Density matrix of the occupied subspace from H and S: the step that follows the H
integration in an s.c.f. iteration (the eigensolver stage that the paper names as the
bottleneck for large systems, *Development Priorities*).  TEST INFRASTRUCTURE ONLY (see the
package docstring).

For one system with basis size n:

* H_s = (H + H^T) / 2.  The raw quadrature H is not exactly symmetric; its symmetric part is
  the operator whose generalised eigenproblem is solved.
* H_s c_k = eps_k S c_k with c_k^T S c_j = delta_kj (generalised symmetric-definite problem,
  ``scipy.linalg.eigh``), eps ascending.
* Spin-restricted occupations 0 <= f_k <= 2 with sum_k f_k = N_e:
    - kT = 0: aufbau, the lowest floor(N_e / 2) states hold 2 electrons, a remaining fraction
      goes into the next state;
    - kT > 0: Fermi-Dirac, f_k = 2 / (1 + exp((eps_k - mu) / kT)), with the chemical potential
      mu fixed by sum_k f_k = N_e (bisection to machine precision).
* P = C diag(f) C^T, i.e. P_ij = sum_k f_k c_k(i) c_k(j).
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np
import scipy.linalg
import scipy.special


def symmetric_part(H: np.ndarray) -> np.ndarray:
    H = np.asarray(H, dtype=np.float64)
    return 0.5 * (H + H.T)


def _fermi(eps: np.ndarray, mu: float, kT: float) -> np.ndarray:
    # 2 / (1 + exp((eps - mu) / kT)) = 2 expit(-(eps - mu) / kT), free of overflow
    return 2.0 * scipy.special.expit(-(eps - mu) / kT)


def occupations(eps: np.ndarray, n_elec: float, kT: float = 0.0) -> Tuple[np.ndarray, float]:
    """(f, mu) for ascending eigenvalues ``eps`` and ``n_elec`` electrons."""
    eps = np.asarray(eps, dtype=np.float64)
    n = eps.size
    if not (0.0 <= n_elec <= 2.0 * n):
        raise ValueError(f"{n_elec} electrons do not fit {n} states")
    if kT == 0.0:
        f = np.zeros(n)
        full = int(math.floor(n_elec / 2.0))
        f[:full] = 2.0
        rest = n_elec - 2.0 * full
        if rest > 0.0:
            f[full] = rest
        # mu: midway between the highest (partly) occupied and the lowest empty level
        occ = np.nonzero(f > 0)[0]
        emp = np.nonzero(f < 2.0)[0]
        hi = eps[occ[-1]] if occ.size else -math.inf
        lo = eps[emp[0]] if emp.size else math.inf
        if rest > 0.0:
            mu = float(eps[full])
        elif math.isfinite(hi) and math.isfinite(lo):
            mu = 0.5 * float(hi + lo)
        else:
            mu = float(hi if math.isfinite(hi) else lo)
        return f, mu
    if n_elec == 0.0:
        return np.zeros(n), -math.inf
    if n_elec == 2.0 * n:
        return np.full(n, 2.0), math.inf
    a = float(eps[0]) - 50.0 * kT - 1.0
    b = float(eps[-1]) + 50.0 * kT + 1.0
    while _fermi(eps, a, kT).sum() > n_elec:
        a -= (b - a)
    while _fermi(eps, b, kT).sum() < n_elec:
        b += (b - a)
    for _ in range(2000):
        m = 0.5 * (a + b)
        if m == a or m == b:
            break
        if _fermi(eps, m, kT).sum() < n_elec:
            a = m
        else:
            b = m
    mu = 0.5 * (a + b)
    return _fermi(eps, mu, kT), mu


def density_matrix(H: np.ndarray, S: np.ndarray, n_elec: float, kT: float = 0.0) -> Dict:
    """{"P", "eps", "f", "mu", "C"} of one system (C holds the eigenvectors as columns)."""
    Hs = symmetric_part(H)
    S = np.asarray(S, dtype=np.float64)
    eps, C = scipy.linalg.eigh(Hs, S)
    f, mu = occupations(eps, n_elec, kT)
    P = (C * f[None, :]) @ C.T
    return {"P": P, "eps": eps, "f": f, "mu": mu, "C": C}
