"""Hartree potential of the grid density by an atom-centred multipole expansion of the
partitioned density (the electrostatic step of an s.c.f. iteration, which the paper notes is
not yet accelerated on GPUs, *Development Priorities*).  TEST INFRASTRUCTURE ONLY (see the
package docstring).  Derived from textbook electrostatics:

* Partition.  n = sum_a n_a with n_a = p_a n (p_a the grid's partition function), so each atom's
  piece is integrated on that atom's own product grid: w_p = W_k w_ang p_a for a point on radial
  node k of atom a.
* Multipoles per radial node.  rho_{a,lm}(r_k) = int dOmega n_a Y_lm
  = sum_{p in node k of a} w_p n_p Y_lm(u_p) / W_k,  u_p = (p - R_a)/|p - R_a|  (l <= l_max,
  real orthonormal Y_lm).
* Radial Poisson equation.  The potential of one multipole component is
      V_lm(r) = 4 pi / (2l+1) [ r^-(l+1) int_0^r rho_lm s^(l+2) ds + r^l int_r^inf rho_lm s^(1-l) ds ].
  The radial nodes are Becke's map r = r_m cot^2(theta/2) on uniform theta_k = (k+1) pi/(K+1),
  so rho_lm is interpolated by a natural cubic spline in theta and each interval's integrals
  are taken by 6-point Gauss-Legendre in theta (Jacobian |dr/dtheta| = r_m cot(t/2) csc^2(t/2)).
  Inside the innermost node rho_lm is taken as rho_lm(r_min) (r/r_min)^l.
* Compact support.  An atom's piece of the density lives on that atom's points only, and the
  partition weights vanish exactly beyond a finite radius, so the outer radial nodes of an atom
  can carry no point.  With k_o the outermost node that carries a point of atom a, the spline
  runs over the nodes from the innermost one out to the edge node k_e = k_o + 1 outwards (the
  first empty node, where rho_lm = 0; the outermost node itself when k_o is it), and rho_lm = 0
  beyond it: atom a's support ends at R_a = r(k_e).  q_lm = int_0^{R_a} rho_lm s^(l+2) ds is
  the multipole moment, and for r >= R_a the Poisson solution is exactly the exterior form
  4 pi q_lm / ((2l+1) r^(l+1)).
* Potential at any point.  v_H(p) = sum_a sum_lm V_{a,lm}(|p - R_a|) Y_lm(u), with V_lm from a
  natural cubic spline in theta through its node values from the innermost node out to the edge
  node, the exterior form beyond the edge node (no spline: an atom whose support a point lies
  outside costs only its moments), and V_lm(r_min) (r/r_min)^l inside the innermost node.
* Hartree energy E_H = 1/2 sum_p w_p n_p v_H(p).

Pinned in tests/test_oracle_hartree.py by Gaussian charge distributions (closed forms
erf(sqrt(a) r)/r and the Coulomb self-energy) and the convergence of the expansion with l_max.
"""
from __future__ import annotations

import math
from typing import Dict

import numpy as np
import scipy.interpolate

from .harmonics import lm_list, real_ylm

GL_X, GL_W = np.polynomial.legendre.leggauss(6)


def radial_nodes(n_radial: int, r_map: float):
    """(theta_k, r_k, W_k): Becke's map on Gauss-Chebyshev (second kind) nodes and its radial
    weights with the r^2 Jacobian, W_k = pi/(K+1) sin(t) 2 r_m/(1 - cos t)^2 r_k^2."""
    k = np.arange(1, n_radial + 1, dtype=np.float64)
    th = k * np.pi / (n_radial + 1)
    x = np.cos(th)
    r = r_map * (1.0 + x) / (1.0 - x)
    W = np.pi / (n_radial + 1) * np.sin(th) * 2.0 * r_map / (1.0 - x) ** 2 * r ** 2
    return th, r, W


def _r_of(t, r_map):
    return r_map / np.tan(0.5 * t) ** 2


def _jac(t, r_map):
    c = 1.0 / np.tan(0.5 * t)
    return r_map * c / np.sin(0.5 * t) ** 2


def multipoles(inst, n: np.ndarray, pt_shell: np.ndarray, n_radial: int, r_map: float,
               l_max: int) -> np.ndarray:
    """rho [n_atoms, n_radial, (l_max+1)^2]."""
    _, _, W = radial_nodes(n_radial, r_map)
    own = np.asarray(inst.pt_atom)
    d = inst.pt_xyz - inst.atom_xyz[own]
    r = np.linalg.norm(d, axis=1)
    u = d / np.maximum(r, 1e-300)[:, None]
    Y = real_ylm(u, l_max)
    rho = np.zeros((inst.n_atoms, n_radial, (l_max + 1) ** 2))
    np.add.at(rho, (own, pt_shell), (inst.pt_w * n)[:, None] * Y)
    return rho / W[None, :, None]


def edge_nodes(inst, pt_shell: np.ndarray, n_radial: int) -> np.ndarray:
    """k_e per atom: one node outwards of the outermost node that carries a point of the atom
    (node 0 is the outermost); 0 for an atom without points."""
    own = np.asarray(inst.pt_atom)
    ke = np.zeros(inst.n_atoms, dtype=np.int64)
    for a in range(inst.n_atoms):
        nodes = np.asarray(pt_shell)[own == a]
        if nodes.size:
            ke[a] = max(0, int(nodes.min()) - 1)
    return ke


def radial_potentials(rho: np.ndarray, n_radial: int, r_map: float, l_max: int,
                      edge: np.ndarray = None) -> Dict:
    """{"V": [n_atoms, K, nlm] node values, "q": [n_atoms, nlm] moments} from the node
    multipoles; rho_lm of atom a is splined over nodes edge[a]..K-1 and zero beyond (edge
    None: every node).  V at the nodes outside the edge node is the exterior form."""
    th, r, _ = radial_nodes(n_radial, r_map)
    h = th[1] - th[0]
    na, K, nlm = rho.shape
    if edge is None:
        edge = np.zeros(na, dtype=np.int64)
    ls = np.array([l for l, _ in lm_list(l_max)])
    V = np.zeros_like(rho)
    q = np.zeros((na, nlm))
    # Gauss-Legendre abscissae of every interval [th_k, th_k+1]
    tg = 0.5 * (th[:-1, None] + th[1:, None]) + 0.5 * h * GL_X[None, :]
    wg = 0.5 * h * GL_W[None, :]
    sg = _r_of(tg, r_map)
    jg = _jac(tg, r_map)
    for a in range(na):
        e = int(edge[a])
        for c in range(nlm):
            l = int(ls[c])
            S = scipy.interpolate.CubicSpline(th[e:], rho[a, e:, c], bc_type="natural")
            f = S(tg[e:])
            A = np.sum(wg * f * sg[e:] ** (l + 2) * jg[e:], axis=1)     # int over r in [r_k+1, r_k]
            B = np.sum(wg * f * sg[e:] ** (1 - l) * jg[e:], axis=1)
            tail = rho[a, -1, c] * r[-1] ** (l + 3) / (2 * l + 3)
            inner = tail + np.concatenate([np.cumsum(A[::-1])[::-1], [0.0]])   # int_0^{r_k}
            outer = np.concatenate([[0.0], np.cumsum(B)])                      # int_{r_k}^{R_a}
            pref = 4 * math.pi / (2 * l + 1)
            V[a, e:, c] = pref * (r[e:] ** (-l - 1) * inner + r[e:] ** l * outer)
            q[a, c] = inner[0]
            V[a, :e, c] = pref * q[a, c] / r[:e] ** (l + 1)
    return {"V": V, "q": q, "edge": np.asarray(edge)}


def potential_at(points: np.ndarray, atom_xyz: np.ndarray, pot: Dict, n_radial: int,
                 r_map: float, l_max: int) -> np.ndarray:
    """v_H at arbitrary points from the per-atom node potentials."""
    th, r, _ = radial_nodes(n_radial, r_map)
    ls = np.array([l for l, _ in lm_list(l_max)])
    V, q = pot["V"], pot["q"]
    edge = pot.get("edge", np.zeros(atom_xyz.shape[0], dtype=np.int64))
    out = np.zeros(points.shape[0])
    for a in range(atom_xyz.shape[0]):
        e = int(edge[a])
        d = points - atom_xyz[a]
        ra = np.linalg.norm(d, axis=1)
        u = d / np.maximum(ra, 1e-300)[:, None]
        Y = real_ylm(u, l_max)
        far = ra >= r[e]
        inner = ra < r[-1]
        mid = ~far & ~inner
        t = 2.0 * np.arctan(np.sqrt(r_map / np.maximum(ra, 1e-300)))
        for c in range(len(ls)):
            l = int(ls[c])
            val = np.zeros_like(ra)
            val[far] = 4 * math.pi / (2 * l + 1) * q[a, c] / ra[far] ** (l + 1)
            S = scipy.interpolate.CubicSpline(th[e:], V[a, e:, c], bc_type="natural")
            val[mid] = S(t[mid])
            val[inner] = V[a, -1, c] * (ra[inner] / r[-1]) ** l
            out += val * Y[:, c]
    return out


def hartree(inst, n: np.ndarray, pt_shell: np.ndarray, n_radial: int, r_map: float,
            l_max: int) -> Dict:
    """{"v": v_H at the instance's points, "E_H", "rho", "V", "q"}."""
    rho = multipoles(inst, n, pt_shell, n_radial, r_map, l_max)
    pot = radial_potentials(rho, n_radial, r_map, l_max, edge_nodes(inst, pt_shell, n_radial))
    v = potential_at(inst.pt_xyz, inst.atom_xyz, pot, n_radial, r_map, l_max)
    return {"v": v, "E_H": 0.5 * float(np.sum(inst.pt_w * n * v)), "rho": rho, **pot}
