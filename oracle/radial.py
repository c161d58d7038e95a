"""Radial functions of the NAO basis as natural cubic splines in s = ln r (test oracle).

Each shell's radial function R and kinetic radial function K are tabulated at the logarithmic
knots r_k = r0 (rc/r0)^(k/(n_log-1)).  They are interpolated by the natural cubic spline in
s = ln r through those values (``scipy.interpolate.CubicSpline`` with ``bc_type='natural'``), the
first cubic piece is used below r0, and both vanish for r >= rc.  Distances below 1e-12 bohr
are clamped to 1e-12.
"""
from __future__ import annotations

import numpy as np
from scipy.interpolate import CubicSpline

R_MIN = 1e-12


def knots(n_log: int, r0: float, rc: float) -> np.ndarray:
    k = np.arange(n_log, dtype=np.float64)
    r = r0 * (rc / r0) ** (k / (n_log - 1))
    r[-1] = rc
    return r


class RadialSplines:
    """Splines of R and K for every shell of every species of an instance."""

    def __init__(self, inst):
        self.rc = float(inst.rc)
        self.s = np.log(knots(inst.n_log, inst.r0, inst.rc))
        off = np.concatenate([[0], np.cumsum(inst.species_nshell)]).astype(np.int64)
        self.shells = [np.arange(off[i], off[i + 1]) for i in range(len(inst.species_nshell))]
        self.R = [CubicSpline(self.s, inst.shell_R[sh].T, bc_type="natural") for sh in self.shells]
        self.K = [CubicSpline(self.s, inst.shell_K[sh].T, bc_type="natural") for sh in self.shells]

    def eval(self, species: int, r: np.ndarray, deriv: int = 0):
        """(R, K) of every shell of ``species`` at distances r[...] -> two arrays [..., nshell].
        ``deriv=1`` returns dR/dr and dK/dr instead."""
        r = np.maximum(np.asarray(r, dtype=np.float64), R_MIN)
        s = np.log(r)
        inside = (r < self.rc)[..., None]
        if deriv == 0:
            Rv = self.R[species](s)
            Kv = self.K[species](s)
        else:
            Rv = self.R[species](s, 1) / r[..., None]
            Kv = self.K[species](s, 1) / r[..., None]
        return np.where(inside, Rv, 0.0), np.where(inside, Kv, 0.0)

    # --- torch twin for automatic differentiation (same piecewise cubics) -------------------
    def torch_tables(self, species: int):
        import torch
        cR = torch.from_numpy(np.ascontiguousarray(self.R[species].c))  # [4, n-1, nshell]
        cK = torch.from_numpy(np.ascontiguousarray(self.K[species].c))
        return torch.from_numpy(self.s), cR, cK

    def eval_torch(self, species: int, r):
        """Differentiable (R, K) at torch distances r[...] -> [..., nshell] each."""
        import torch
        x, cR, cK = self.torch_tables(species)
        r = torch.clamp(r, min=R_MIN)
        s = torch.log(r)
        k = torch.clamp(torch.searchsorted(x, s.detach(), right=True) - 1, 0, x.numel() - 2)
        dt = (s - x[k])[..., None]
        out = []
        for c in (cR, cK):
            ck = c[:, k, :]                                  # [4, ..., nshell]
            val = ((ck[0] * dt + ck[1]) * dt + ck[2]) * dt + ck[3]
            out.append(torch.where((r < self.rc)[..., None], val, torch.zeros_like(val)))
        return out[0], out[1]
