"""Direct FP64 quadrature of density, Hamiltonian, overlap, energy and gradients (test oracle).

Everything is evaluated straight from the definitions listed in the package docstring, in
chunks of points taken in the caller's order.  A chunk only carries the functions of atoms
closer than rc to at least one of its points: every other function is exactly zero on the
chunk, so this screening changes no result (a brute-force test checks it).  There is no other
blocking, fusion or reordering.
"""
from __future__ import annotations

import math
from typing import Dict, Optional

import numpy as np

from .harmonics import lm_list, real_ylm, real_ylm_grad
from .radial import R_MIN, RadialSplines


class GridOracle:
    def __init__(self, inst, chunk: int = 4096):
        self.inst = inst
        self.chunk = int(chunk)
        self.spl = RadialSplines(inst)
        self.lm = {lm: k for k, lm in enumerate(lm_list())}
        off = inst.species_shell_offset()
        # per species: (local shell index, lm index, l) of each function in contract order
        self.fn_shell, self.fn_lm, self.fn_l = [], [], []
        for s in range(len(inst.species_nshell)):
            sh, lmi, ll = [], [], []
            for k in range(off[s], off[s + 1]):
                l = int(inst.shell_l[k])
                for m in range(-l, l + 1):
                    sh.append(k - off[s])
                    lmi.append(self.lm[(l, m)])
                    ll.append(l)
            self.fn_shell.append(np.array(sh, dtype=np.int64))
            self.fn_lm.append(np.array(lmi, dtype=np.int64))
            self.fn_l.append(np.array(ll, dtype=np.float64))
        self.atom_off = inst.atom_basis_offset()
        self.nb = int(self.atom_off[-1])

    # ------------------------------------------------------------------------------------
    def relevant_atoms(self, pts: np.ndarray, atom_xyz: np.ndarray) -> np.ndarray:
        """Atoms with at least one point of ``pts`` closer than rc."""
        d = np.sqrt(((pts[:, None, :] - atom_xyz[None, :, :]) ** 2).sum(-1))
        return np.nonzero(d.min(axis=0) < self.inst.rc)[0]

    def basis_values(self, pts: np.ndarray, atom_xyz: Optional[np.ndarray] = None,
                     atoms: Optional[np.ndarray] = None, grad: bool = False):
        """phi and t phi of the functions of ``atoms`` (default: relevant atoms) at ``pts``.
        Returns (Phi [np, nf], TPhi [np, nf], cols [nf]) with cols the global basis indices in
        ascending order; with ``grad`` also (GPhi, GTPhi) [np, nf, 3] = gradients with respect
        to the point (the gradient with respect to the centre is minus this)."""
        inst = self.inst
        X = inst.atom_xyz if atom_xyz is None else atom_xyz
        if atoms is None:
            atoms = self.relevant_atoms(pts, X)
        blocks, tblocks, gblocks, gtblocks, cols = [], [], [], [], []
        for a in atoms:
            s = int(inst.atom_species[a])
            d = pts - X[a]
            r = np.sqrt((d * d).sum(-1))
            rr = np.maximum(r, R_MIN)
            u = d / rr[:, None]
            Y = real_ylm(u)
            Rv, Kv = self.spl.eval(s, r)
            sh, lmi = self.fn_shell[s], self.fn_lm[s]
            blocks.append(Rv[:, sh] * Y[:, lmi])
            tblocks.append(Kv[:, sh] * Y[:, lmi])
            cols.append(self.atom_off[a] + np.arange(sh.size))
            if grad:
                dR, dK = self.spl.eval(s, r, deriv=1)
                G = real_ylm_grad(u)[:, lmi, :]                    # [np, nf, 3]
                l = self.fn_l[s][None, :]
                radial_part = lambda F, dF: ((dF[:, sh] - l * F[:, sh] / rr[:, None])
                                             * Y[:, lmi])[:, :, None] * u[:, None, :] \
                    + (F[:, sh] / rr[:, None])[:, :, None] * G
                gblocks.append(radial_part(Rv, dR))
                gtblocks.append(radial_part(Kv, dK))
        if not cols:
            z = np.zeros((pts.shape[0], 0))
            out = (z, z, np.zeros(0, dtype=np.int64))
            if grad:
                out = out + (np.zeros((pts.shape[0], 0, 3)),) * 2
            return out
        cols = np.concatenate(cols)
        out = (np.concatenate(blocks, 1), np.concatenate(tblocks, 1), cols)
        if grad:
            out = out + (np.concatenate(gblocks, 1), np.concatenate(gtblocks, 1))
        return out

    def _chunks(self):
        n = self.inst.n_points
        for s0 in range(0, n, self.chunk):
            yield slice(s0, min(n, s0 + self.chunk))

    # ------------------------------------------------------------------------------------
    def density(self, P: np.ndarray, v: Optional[np.ndarray] = None,
                points: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
        """n(p) = sum_ij P_ij phi_i phi_j for every point (or the subset ``points`` of indices),
        and the sums N, E_V, E_T over those points."""
        inst = self.inst
        idx_all = np.arange(inst.n_points) if points is None else np.asarray(points)
        n = np.zeros(idx_all.size)
        N = EV = ET = 0.0
        for s0 in range(0, idx_all.size, self.chunk):
            idx = idx_all[s0:s0 + self.chunk]
            Phi, TPhi, cols = self.basis_values(inst.pt_xyz[idx])
            Xm = Phi @ P[np.ix_(cols, cols)]
            nc = (Xm * Phi).sum(1)
            n[s0:s0 + idx.size] = nc
            w = inst.pt_w[idx]
            N += float(w @ nc)
            if v is not None:
                EV += float((w * v[idx]) @ nc)
            ET += float(w @ (Xm * TPhi).sum(1))
        return {"n": n, "N": N, "E_V": EV, "E_T": ET}

    def integrate_h(self, v: np.ndarray, want_S: bool = True,
                    points: Optional[np.ndarray] = None):
        """H_ij = sum_p w_p phi_i (v_p phi_j + tphi_j) and S_ij = sum_p w_p phi_i phi_j, summed
        over every point (or over the subset ``points`` of indices)."""
        inst = self.inst
        H = np.zeros((self.nb, self.nb))
        S = np.zeros((self.nb, self.nb)) if want_S else None
        idx_all = np.arange(inst.n_points) if points is None else np.asarray(points)
        for s0 in range(0, idx_all.size, self.chunk):
            sl = idx_all[s0:s0 + self.chunk]
            Phi, TPhi, cols = self.basis_values(inst.pt_xyz[sl])
            w = inst.pt_w[sl][:, None]
            ix = np.ix_(cols, cols)
            H[ix] += Phi.T @ (w * (v[sl][:, None] * Phi + TPhi))
            if want_S:
                S[ix] += Phi.T @ (w * Phi)
        return H, S

    def energy(self, P: np.ndarray, v: np.ndarray) -> float:
        d = self.density(P, v)
        return d["E_V"] + d["E_T"]

    # ------------------------------------------------------------------------------------
    def gradient(self, P: np.ndarray, v: np.ndarray, atoms: Optional[np.ndarray] = None):
        """E = sum_p w v n + sum_p w sum_ij P_ij phi_i tphi_j and its derivatives:
        dE/dP = H (independent entries), dE/dv = w n, and dE/dR (basis centres move; grid,
        weights and v stay) by reverse-mode automatic differentiation in float64 of the same
        definitions.  ``atoms`` limits dE/dR to those atoms (only points within rc of them are
        visited)."""
        import torch
        inst = self.inst
        dens = self.density(P, v)
        H, _ = self.integrate_h(v, want_S=False)
        gR = np.zeros((inst.n_atoms, 3))
        Pt = torch.from_numpy(P)
        if atoms is None:
            sel_pts = np.arange(inst.n_points)
            want = np.arange(inst.n_atoms)
        else:
            want = np.asarray(atoms)
            d = np.sqrt(((inst.pt_xyz[:, None, :] - inst.atom_xyz[None, want, :]) ** 2).sum(-1))
            sel_pts = np.nonzero(d.min(axis=1) < inst.rc)[0]
        for s0 in range(0, sel_pts.size, self.chunk):
            idx = sel_pts[s0:s0 + self.chunk]
            pts = torch.from_numpy(inst.pt_xyz[idx])
            atoms_c = self.relevant_atoms(inst.pt_xyz[idx], inst.atom_xyz)
            Rt = torch.from_numpy(inst.atom_xyz[atoms_c].copy()).requires_grad_(True)
            Phi, TPhi, cols = self._basis_torch(pts, Rt, atoms_c)
            Xm = Phi @ Pt[np.ix_(cols, cols)]
            w = torch.from_numpy(inst.pt_w[idx])
            vv = torch.from_numpy(v[idx])
            E = ((w * vv) * (Xm * Phi).sum(1)).sum() + (w * (Xm * TPhi).sum(1)).sum()
            E.backward()
            gR[atoms_c] += Rt.grad.numpy()
        out_R = np.zeros_like(gR)
        out_R[want] = gR[want]
        return {"E": dens["E_V"] + dens["E_T"], "dE_dP": H, "dE_dv": inst.pt_w * dens["n"],
                "dE_dR": out_R, "n": dens["n"]}

    def _basis_torch(self, pts, Rt, atoms):
        import torch
        inst = self.inst
        blocks, tblocks, cols = [], [], []
        for j, a in enumerate(atoms):
            s = int(inst.atom_species[a])
            d = pts - Rt[j]
            r = torch.sqrt((d * d).sum(-1))
            u = d / torch.clamp(r, min=R_MIN)[:, None]
            Y = real_ylm(u, xp=torch)
            Rv, Kv = self.spl.eval_torch(s, r)
            sh = torch.from_numpy(self.fn_shell[s])
            lmi = torch.from_numpy(self.fn_lm[s])
            blocks.append(Rv[:, sh] * Y[:, lmi])
            tblocks.append(Kv[:, sh] * Y[:, lmi])
            cols.append(self.atom_off[a] + np.arange(sh.numel()))
        return torch.cat(blocks, 1), torch.cat(tblocks, 1), np.concatenate(cols)

    def gradient_closed_form(self, P: np.ndarray, v: np.ndarray,
                             atoms: Optional[np.ndarray] = None) -> np.ndarray:
        """dE/dR_a = -sum_p w_p sum_{i in a} [(2 v_p X_pi + Y_pi) grad phi_i + X_pi grad tphi_i]
        with X = Phi P and Y = (T Phi) P, using the analytic basis gradient
        grad phi = (R' - l R/r) Y_lm u + (R/r) grad S_lm(u).  Cross-check of ``gradient``.
        ``atoms`` limits dE/dR to those atoms: only points within rc of one of them are visited,
        and X, Y and the basis gradients are formed for their functions only (the other rows
        of the result are zero)."""
        inst = self.inst
        g = np.zeros((inst.n_atoms, 3))
        if atoms is None:
            want = None
            sel = np.arange(inst.n_points)
        else:
            want = np.asarray(atoms)
            d = np.sqrt(((inst.pt_xyz[:, None, :] - inst.atom_xyz[None, want, :]) ** 2).sum(-1))
            sel = np.nonzero(d.min(axis=1) < inst.rc)[0]
        for s0 in range(0, sel.size, self.chunk):
            idx = sel[s0:s0 + self.chunk]
            pts = inst.pt_xyz[idx]
            if want is None:
                Phi, TPhi, cols, G, GT = self.basis_values(pts, grad=True)
                gcols = cols
            else:
                Phi, TPhi, cols = self.basis_values(pts)
                _, _, gcols, G, GT = self.basis_values(pts, atoms=want, grad=True)
            Pc = P[np.ix_(cols, gcols)]
            Xm = Phi @ Pc
            Ym = TPhi @ Pc
            w = inst.pt_w[idx][:, None]
            coef = w * (2.0 * v[idx][:, None] * Xm + Ym)
            contrib = (coef[:, :, None] * G + (w * Xm)[:, :, None] * GT).sum(0)   # [nf, 3]
            host = np.searchsorted(self.atom_off, gcols, side="right") - 1
            np.add.at(g, host, -contrib)
        return g


def phi_bruteforce(inst, p) -> np.ndarray:
    """All basis functions at one point by plain loops: scipy natural splines evaluated per
    shell and real harmonics from ``scipy.special.sph_harm_y`` (no screening, no vectorising).
    Used on tiny inputs to check the chunked evaluation."""
    from scipy.interpolate import CubicSpline
    from scipy.special import sph_harm_y
    from .radial import knots
    s_knots = np.log(knots(inst.n_log, inst.r0, inst.rc))
    out = []
    off = inst.species_shell_offset()
    for a in range(inst.n_atoms):
        d = np.asarray(p, dtype=np.float64) - inst.atom_xyz[a]
        r = max(math.sqrt(float(d @ d)), R_MIN)
        theta = math.acos(max(-1.0, min(1.0, d[2] / r)))
        azim = math.atan2(d[1], d[0])
        sp = int(inst.atom_species[a])
        for k in range(off[sp], off[sp + 1]):
            l = int(inst.shell_l[k])
            if r < inst.rc:
                Rv = float(CubicSpline(s_knots, inst.shell_R[k], bc_type="natural")(math.log(r)))
            else:
                Rv = 0.0
            for m in range(-l, l + 1):
                c = complex(sph_harm_y(l, abs(m), theta, azim))
                if m > 0:
                    y = math.sqrt(2.0) * (-1) ** m * c.real
                elif m < 0:
                    y = math.sqrt(2.0) * (-1) ** m * c.imag
                else:
                    y = c.real
                out.append(Rv * y)
    return np.array(out)
