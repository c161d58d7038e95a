"""Exchange-correlation of the spin-unpolarised electron gas, evaluated pointwise on the grid
(the potential step before the H integration in an s.c.f. iteration; the paper names the
semilocal functionals as the method's scope, *Background and Current Status*).
TEST INFRASTRUCTURE ONLY (see the package docstring).

LDA = Slater exchange + the Perdew-Wang (1992) parametrisation of the correlation energy:

    eps_x(n) = -(3/4) (3 n / pi)^(1/3)                        (energy per electron)
    rs = (3 / (4 pi n))^(1/3)
    eps_c(n) = -2 A (1 + a1 rs) ln(1 + 1 / (2 A (b1 rs^(1/2) + b2 rs + b3 rs^(3/2) + b4 rs^2)))
    A = 0.031091, a1 = 0.21370, b1 = 7.5957, b2 = 3.5876, b3 = 1.6382, b4 = 0.49294  (zeta = 0)
    v_xc = d(n eps_xc)/dn,   E_xc = sum_p w_p n_p eps_xc(n_p)

Points with n <= N_MIN (including the negative densities of unphysical P) contribute nothing:
eps = v = 0 there.  The derivative is taken by torch autograd in float64, not by a formula, so
the oracle's potential is the exact derivative of its energy density.

``density_gradient`` gives n and grad n = sum_ij P_ij grad(phi_i phi_j) at the grid points, the
input of the gradient-corrected functionals, by autograd with respect to the point positions.

``vector_term`` is the matrix B_ij = sum_p w_p phi_i(p) u_p . grad phi_j(p) of a vector field u
on the grid: the gradient-corrected part of H is B + B^T with u = 2 v_sigma grad n.
"""
from __future__ import annotations

import math
from typing import Dict

import numpy as np

N_MIN = 1e-14
PW92 = dict(A=0.031091, a1=0.21370, b1=7.5957, b2=3.5876, b3=1.6382, b4=0.49294)


def _eps_xc_torch(n):
    import torch
    A, a1, b1, b2, b3, b4 = (PW92[k] for k in ("A", "a1", "b1", "b2", "b3", "b4"))
    ex = -0.75 * (3.0 * n / math.pi) ** (1.0 / 3.0)
    rs = (3.0 / (4.0 * math.pi * n)) ** (1.0 / 3.0)
    q = 2.0 * A * (b1 * torch.sqrt(rs) + b2 * rs + b3 * rs ** 1.5 + b4 * rs * rs)
    ec = -2.0 * A * (1.0 + a1 * rs) * torch.log1p(1.0 / q)
    return ex, ec


def lda(n: np.ndarray) -> Dict[str, np.ndarray]:
    """{"eps_x", "eps_c", "eps", "v"} per point for densities ``n``."""
    import torch
    n = np.asarray(n, dtype=np.float64)
    ok = n > N_MIN
    nt = torch.tensor(np.where(ok, n, 1.0), dtype=torch.float64, requires_grad=True)
    ex, ec = _eps_xc_torch(nt)
    (nt * (ex + ec)).sum().backward()
    z = lambda t: np.where(ok, t.detach().numpy(), 0.0)
    return {"eps_x": z(ex), "eps_c": z(ec), "eps": z(ex + ec), "v": z(nt.grad)}


def lda_energy(n: np.ndarray, w: np.ndarray) -> Dict[str, float]:
    """E_xc = sum w n eps_xc and sum w n v_xc."""
    r = lda(n)
    n = np.asarray(n, dtype=np.float64)
    return {"E_xc": float(np.sum(w * n * r["eps"])), "nv": float(np.sum(w * n * r["v"]))}


def density_gradient(oracle, P: np.ndarray, chunk: int = 2048):
    """(n [n_points], grad n [n_points, 3]) of ``oracle.inst`` for the density matrix P:
    n = sum_ij P_ij phi_i phi_j, differentiated with respect to each point's position through
    the basis (torch autograd, float64)."""
    import torch
    inst = oracle.inst
    R = torch.tensor(inst.atom_xyz, dtype=torch.float64)
    Pt = torch.from_numpy(np.ascontiguousarray(P, dtype=np.float64))
    n_all = np.zeros(inst.n_points)
    g_all = np.zeros((inst.n_points, 3))
    for s0 in range(0, inst.n_points, chunk):
        idx = np.arange(s0, min(inst.n_points, s0 + chunk))
        atoms = oracle.relevant_atoms(inst.pt_xyz[idx], inst.atom_xyz)
        if atoms.size == 0:
            continue
        pts = torch.tensor(inst.pt_xyz[idx], dtype=torch.float64, requires_grad=True)
        Phi, _, cols = oracle._basis_torch(pts, R[torch.from_numpy(atoms)], atoms)
        n = ((Phi @ Pt[np.ix_(cols, cols)]) * Phi).sum(1)
        (g,) = torch.autograd.grad(n.sum(), pts)
        n_all[idx] = n.detach().numpy()
        g_all[idx] = g.numpy()
    return n_all, g_all


def vector_term(oracle, u: np.ndarray, chunk: int = 4096) -> np.ndarray:
    """B [nb, nb] with B_ij = sum_p w_p phi_i(p) u_p . grad phi_j(p) (closed-form basis
    gradients), for u [n_points, 3]."""
    inst = oracle.inst
    B = np.zeros((oracle.nb, oracle.nb))
    for s0 in range(0, inst.n_points, chunk):
        idx = np.arange(s0, min(inst.n_points, s0 + chunk))
        Phi, _, cols, GPhi, _ = oracle.basis_values(inst.pt_xyz[idx], grad=True)
        if cols.size == 0:
            continue
        D = np.einsum("pjc,pc->pj", GPhi, u[idx])
        B[np.ix_(cols, cols)] += (Phi * inst.pt_w[idx][:, None]).T @ D
    return B
