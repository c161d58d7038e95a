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

PBE (Perdew-Burke-Ernzerhof 1996, spin-unpolarised) adds the gradient of the density through
sigma = |grad n|^2:

    f(n, sigma) = n eps_x(n) F_x(s) + n (eps_c(n) + H(rs, t))
    F_x(s) = 1 + kappa - kappa / (1 + mu s^2 / kappa),    s^2 = sigma / (4 k_F^2 n^2)
    H = gamma ln(1 + (beta/gamma) t^2 (1 + A t^2) / (1 + A t^2 + A^2 t^4)),
    t^2 = sigma / (4 k_s^2 n^2),  A = (beta/gamma) / (exp(-eps_c / gamma) - 1)
    k_F = (3 pi^2 n)^(1/3),  k_s = (4 k_F / pi)^(1/2),  gamma = (1 - ln 2) / pi^2,
    kappa = 0.804,  beta = 0.06672455060314922,  mu = beta pi^2 / 3
    v_n = df/dn,  v_sigma = df/dsigma (autograd)

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


PBE = dict(kappa=0.804, beta=0.06672455060314922)


def _pbe_H_torch(n, sigma, ec):
    """(H, t^2): the gradient correction of the PBE correlation energy per electron, and the
    reduced gradient t^2 = sigma / (4 k_s^2 n^2) it is a function of (with eps_c = ec)."""
    import torch
    beta = PBE["beta"]
    gamma = (1.0 - math.log(2.0)) / math.pi ** 2
    kF = (3.0 * math.pi ** 2 * n) ** (1.0 / 3.0)
    ks2 = 4.0 * kF / math.pi
    t2 = sigma / (4.0 * ks2 * n * n)
    A = (beta / gamma) / torch.expm1(-ec / gamma)
    At2 = A * t2
    H = gamma * torch.log1p((beta / gamma) * t2 * (1.0 + At2) / (1.0 + At2 + At2 * At2))
    return H, t2


def _pbe_f_torch(n, sigma):
    kappa, beta = PBE["kappa"], PBE["beta"]
    mu = beta * math.pi ** 2 / 3.0
    ex, ec = _eps_xc_torch(n)
    kF = (3.0 * math.pi ** 2 * n) ** (1.0 / 3.0)
    s2 = sigma / (4.0 * kF * kF * n * n)
    Fx = 1.0 + kappa - kappa / (1.0 + mu * s2 / kappa)
    H, _ = _pbe_H_torch(n, sigma, ec)
    return n * ex * Fx + n * (ec + H)


def pbe(n: np.ndarray, sigma: np.ndarray) -> Dict[str, np.ndarray]:
    """{"f", "v_n", "v_sigma"} per point: the energy density f(n, sigma) (E_xc = sum w f) and
    its partial derivatives; zero where n <= N_MIN."""
    import torch
    n = np.asarray(n, dtype=np.float64)
    ok = n > N_MIN
    nt = torch.tensor(np.where(ok, n, 1.0), dtype=torch.float64, requires_grad=True)
    st = torch.tensor(np.where(ok, np.asarray(sigma, dtype=np.float64), 0.0), dtype=torch.float64,
                      requires_grad=True)
    f = _pbe_f_torch(nt, st)
    f.sum().backward()
    z = lambda t: np.where(ok, t.detach().numpy(), 0.0)
    return {"f": z(f), "v_n": z(nt.grad), "v_sigma": z(st.grad)}


def pbe_energy_and_matrix(oracle, P: np.ndarray, chunk: int = 2048):
    """(E_xc, H_xc [nb, nb]) of PBE for the density matrix P: E_xc = sum_p w f(n, |grad n|^2)
    with n = sum_ij P_ij phi_i phi_j and grad n = sum_ij P_ij grad(phi_i phi_j) (closed-form
    basis gradients), and H_xc = dE_xc/dP by autograd (entries independent)."""
    import torch
    inst = oracle.inst
    Pt = torch.tensor(np.ascontiguousarray(P, dtype=np.float64), requires_grad=True)
    E = 0.0
    for s0 in range(0, inst.n_points, chunk):
        idx = np.arange(s0, min(inst.n_points, s0 + chunk))
        Phi, _, cols, GPhi, _ = oracle.basis_values(inst.pt_xyz[idx], grad=True)
        if cols.size == 0:
            continue
        Ph = torch.from_numpy(Phi)
        G = torch.from_numpy(GPhi)
        Pb = Pt[np.ix_(cols, cols)]
        n = ((Ph @ Pb) * Ph).sum(1)
        # grad n = sum_ij P_ij (grad phi_i phi_j + phi_i grad phi_j)
        gn = torch.einsum("pic,ij,pj->pc", G, Pb, Ph) + torch.einsum("pi,ij,pjc->pc", Ph, Pb, G)
        sigma = (gn * gn).sum(1)
        ok = n > N_MIN
        w = torch.from_numpy(inst.pt_w[idx])
        f = _pbe_f_torch(torch.where(ok, n, torch.ones_like(n)),
                         torch.where(ok, sigma, torch.zeros_like(sigma)))
        Ec = (w * torch.where(ok, f, torch.zeros_like(f))).sum()
        Ec.backward()
        E += float(Ec.detach())
    return E, Pt.grad.numpy().copy()
