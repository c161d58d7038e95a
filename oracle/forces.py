"""Total (moving-grid) energy gradient, FP64, by reverse-mode automatic differentiation.
TEST INFRASTRUCTURE ONLY (see the package docstring).

Here every ingredient of the energy follows the atoms, as it does when the whole calculation
is repeated at displaced nuclei:

    E(R) = sum_p w_p(R) [ v(p; R) n(p; R) + sum_ij P_ij phi_i(p) tphi_j(p) ]

* point p = R_o + d_p belongs to the atom-centred grid of its owner o and moves with it (the
  offset d_p is fixed);
* w_p = g_p s_o(p) / sum_b s_b(p): the radial x angular weight g_p of the owner's grid times the
  Stratmann-Scuseria-Frisch partition, s_b(p) = prod_{c != b} s(mu_bc(p)),
  mu_bc = (|p - R_b| - |p - R_c|) / |R_b - R_c|, s(mu) = (1 - z(mu / a)) / 2 with
  z(x) = (35 x - 35 x^3 + 21 x^5 - 5 x^7) / 16 on [-1, 1] and sign(x) beyond, a = 0.64;
* v(p; R) = sum_a -Z_a erf(|p - R_a| / sigma) / |p - R_a|, sigma = 0.3 (the nuclear potential
  the inputs use);
* phi_i, tphi_i are centred on their atoms as in the package docstring; P is held fixed.

The gradient is taken by torch autograd (float64) through all four dependences; the partition
products run over all atoms (no neighbour truncation).  It is pinned in the tests by
translation invariance (sum_a dE/dR_a = 0) and by finite differences of E over grids rebuilt
from scratch at displaced atoms.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

PARTITION_A = 0.64
NUCLEAR_SIGMA = 0.3


def _partition_torch(pts, R, own, a: float):
    """Stratmann partition weight of each point's owner, as a differentiable torch function
    of the point positions ``pts`` [c, 3] and atom positions ``R`` [na, 3]."""
    import torch
    na = R.shape[0]
    if na == 1:
        return torch.ones(pts.shape[0], dtype=pts.dtype)
    d = pts[:, None, :] - R[None, :, :]
    D = torch.sqrt((d * d).sum(-1))                                   # [c, na]
    eye = torch.eye(na, dtype=torch.bool)
    dR = R[:, None, :] - R[None, :, :]
    RAB = torch.sqrt((dR * dR).sum(-1) + eye.to(R.dtype))            # diagonal kept at 1
    mu = (D[:, :, None] - D[:, None, :]) / RAB[None]                  # [c, b, c']
    x = torch.clamp(mu / a, -1.0, 1.0)
    x2 = x * x
    z = x * (35.0 + x2 * (-35.0 + x2 * (21.0 - 5.0 * x2))) / 16.0
    s = torch.where(eye[None], torch.ones_like(z), 0.5 * (1.0 - z))
    Pb = torch.prod(s, dim=2)                                         # [c, na]
    return Pb[torch.arange(pts.shape[0]), own] / Pb.sum(dim=1)


def _nuclear_torch(pts, R, Z, sigma: float):
    import torch
    d = pts[:, None, :] - R[None, :, :]
    r = torch.sqrt((d * d).sum(-1))
    return -(torch.erf(r / sigma) / r * Z[None, :]).sum(dim=1)


def moving_grid_gradient(oracle, P: np.ndarray, a: float = PARTITION_A,
                         sigma: float = NUCLEAR_SIGMA, chunk: int = 1024,
                         points: Optional[np.ndarray] = None):
    """(E, dE/dR [n_atoms, 3]) of the moving-grid energy above for ``oracle.inst`` (which must
    carry the pre-partition weights ``pt_wgrid``).  ``points`` restricts both to a subset of
    the grid (the sums are over points, so subsets add up)."""
    import torch
    inst = oracle.inst
    if inst.pt_wgrid is None:
        raise ValueError("the instance has no pre-partition grid weights")
    R = torch.tensor(inst.atom_xyz, dtype=torch.float64, requires_grad=True)
    Z = torch.tensor(np.asarray(inst.atom_Z, dtype=np.float64))
    Pt = torch.from_numpy(np.ascontiguousarray(P, dtype=np.float64))
    own_all = np.asarray(inst.pt_atom, dtype=np.int64)
    off_all = inst.pt_xyz - inst.atom_xyz[own_all]
    idx_all = np.arange(inst.n_points) if points is None else np.asarray(points)
    E = 0.0
    for s0 in range(0, idx_all.size, chunk):
        idx = idx_all[s0:s0 + chunk]
        own = torch.from_numpy(own_all[idx])
        pts = R[own] + torch.from_numpy(off_all[idx])
        w = torch.from_numpy(inst.pt_wgrid[idx]) * _partition_torch(pts, R, own, a)
        v = _nuclear_torch(pts, R, Z, sigma)
        atoms = oracle.relevant_atoms(inst.pt_xyz[idx], inst.atom_xyz)
        if atoms.size:
            Phi, TPhi, cols = oracle._basis_torch(pts, R[torch.from_numpy(atoms)], atoms)
            Xm = Phi @ Pt[np.ix_(cols, cols)]
            n = (Xm * Phi).sum(1)
            dens_t = (Xm * TPhi).sum(1)
            Ec = (w * (v * n + dens_t)).sum()
        else:
            Ec = (w * v * 0.0).sum()
        Ec.backward()
        E += float(Ec.detach())
    return E, R.grad.numpy().copy()
