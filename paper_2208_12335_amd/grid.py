"""Python front of the HIP library: ``AimsGrid`` (one handle, device tensors in and out) and
``AimsEnergy`` (a ``torch.autograd.Function`` whose backward is the library's backward kernel).

PyTorch is used only for device memory and the stream; every step of the computation runs in
the library's kernels.
"""
from __future__ import annotations

import ctypes
from ctypes import POINTER, byref, c_double, c_int32, c_int64, c_void_p
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import (DM_METHOD, PRECISION, XC_FUNCTIONAL, AimsError, AimsHartreeGrid, AimsMovingGrid,
                   AimsSystem, AimsTuning)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if t.dtype != torch.float64:
        raise TypeError("expected a float64 tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return c_void_p(t.data_ptr())


def _np_ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(POINTER(ctype))


class AimsGrid:
    """One library handle over one or several systems.

    ``systems``: objects with the fields atom_xyz, atom_species, species_nshell, shell_l, n_log,
    r0, rc, shell_R, shell_K, pt_xyz, pt_w, max_batch (e.g. ``synth.Instance``)."""

    def __init__(self, systems, device: int = 0, stream: Optional[torch.cuda.Stream] = None,
                 screen_margin: float = 1e-2):
        if not isinstance(systems, (list, tuple)):
            systems = [systems]
        self._L = _lib.load()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        keep = []
        arr = (AimsSystem * len(systems))()
        for k, s in enumerate(systems):
            f64 = lambda x: np.ascontiguousarray(x, dtype=np.float64)
            i32 = lambda x: np.ascontiguousarray(x, dtype=np.int32)
            fields = dict(atom_xyz=f64(s.atom_xyz), atom_species=i32(s.atom_species),
                          species_nshell=i32(s.species_nshell), shell_l=i32(s.shell_l),
                          shell_R=f64(s.shell_R), shell_K=f64(s.shell_K), pt_xyz=f64(s.pt_xyz),
                          pt_w=f64(s.pt_w))
            keep.append(fields)
            a = arr[k]
            a.n_atoms = fields["atom_xyz"].shape[0]
            a.atom_xyz = _np_ptr(fields["atom_xyz"], c_double)
            a.atom_species = _np_ptr(fields["atom_species"], c_int32)
            a.n_species = fields["species_nshell"].shape[0]
            a.species_nshell = _np_ptr(fields["species_nshell"], c_int32)
            a.shell_l = _np_ptr(fields["shell_l"], c_int32)
            a.n_log = int(s.n_log)
            a.r0 = float(s.r0)
            a.rc = float(s.rc)
            a.shell_R = _np_ptr(fields["shell_R"], c_double)
            a.shell_K = _np_ptr(fields["shell_K"], c_double)
            a.n_points = fields["pt_xyz"].shape[0]
            a.pt_xyz = _np_ptr(fields["pt_xyz"], c_double)
            a.pt_w = _np_ptr(fields["pt_w"], c_double)
            a.max_batch = int(s.max_batch)
            a.screen_margin = float(screen_margin)
        h = c_void_p()
        with torch.cuda.device(self.device):
            st = self._L.aims_grid_setup_many(arr, len(systems), device,
                                              c_void_p(self.stream.cuda_stream), byref(h))
        if st != 0:
            raise AimsError(st, self._L.aims_last_error(None).decode())
        self._h = h
        self._systems = list(systems)
        self.n_sys = len(systems)
        self.nb_sys = [self._nb_of(s) for s in systems]
        self.n_basis = int(self._L.aims_n_basis(h))
        self.n_points = int(self._L.aims_n_points(h))
        self.n_atoms = int(self._L.aims_n_atoms(h))
        self.mat_elems = int(sum(nb * nb for nb in self.nb_sys))

    @staticmethod
    def _nb_of(s) -> int:
        off = np.concatenate([[0], np.cumsum(s.species_nshell)]).astype(int)
        sl = np.asarray(s.shell_l)
        nfn = [int(np.sum(2 * sl[off[i]:off[i + 1]] + 1)) for i in range(len(s.species_nshell))]
        return int(sum(nfn[int(sp)] for sp in np.asarray(s.atom_species)))

    # ------------------------------------------------------------------------------------------
    def _check(self, st):
        if st != 0:
            raise AimsError(st, self._L.aims_last_error(self._h).decode())

    def _new(self, *shape):
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    def _arg(self, t: Optional[torch.Tensor], n: int, name: str, at_least: bool = False):
        """Pointer of a caller tensor after checking it holds exactly ``n`` float64 values
        (``at_least``: n or more), contiguous, on this handle's device (None passes through)."""
        if t is None:
            return None
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name}: expected a torch tensor")
        if t.device != self.device:
            raise ValueError(f"{name}: on {t.device}, the handle is on {self.device}")
        k = t.numel()
        if k < n or (k != n and not at_least):
            raise ValueError(f"{name}: {k} elements, {'at least ' if at_least else ''}{n} expected")
        return _ptr(t)

    def update_density(self, P: torch.Tensor, v: Optional[torch.Tensor] = None,
                       prec: str = "fp64", atom_xyz=None, n_out=None, sums_out=None):
        """n [n_points] (caller order) and sums [n_sys, 3] = (N, E_V, E_T)."""
        n = self._new(self.n_points) if n_out is None else n_out
        sums = self._new(self.n_sys, 3) if sums_out is None else sums_out
        with torch.cuda.device(self.device):
            self._check(self._L.aims_update_density(
                self._h, PRECISION[prec], self._xyz(atom_xyz), self._arg(P, self.mat_elems, "P"),
                self._arg(v, self.n_points, "v"), self._arg(n, self.n_points, "n_out"),
                self._arg(sums, 3 * self.n_sys, "sums_out")))
        return n, sums

    def update_density_noalloc(self, P: torch.Tensor, v: Optional[torch.Tensor] = None,
                               prec: str = "fp64", n_out=None, sums_out=None):
        """``update_density`` through the allocation-free entry point (setup positions)."""
        n = self._new(self.n_points) if n_out is None else n_out
        sums = self._new(self.n_sys, 3) if sums_out is None else sums_out
        with torch.cuda.device(self.device):
            self._check(self._L.aims_update_density_noalloc(
                self._h, PRECISION[prec], self._arg(P, self.mat_elems, "P"),
                self._arg(v, self.n_points, "v"), self._arg(n, self.n_points, "n_out"),
                self._arg(sums, 3 * self.n_sys, "sums_out")))
        return n, sums

    def integrate_h(self, v: torch.Tensor, prec: str = "fp64", want_S: bool = False,
                    atom_xyz=None, H_out=None, S_out=None):
        """Flat H (and S) buffers of mat_elems entries; use ``blocks`` to view per system."""
        H = self._new(self.mat_elems) if H_out is None else H_out
        S = (self._new(self.mat_elems) if S_out is None else S_out) if want_S else None
        with torch.cuda.device(self.device):
            self._check(self._L.aims_integrate_h(
                self._h, PRECISION[prec], self._xyz(atom_xyz), self._arg(v, self.n_points, "v"),
                self._arg(H, self.mat_elems, "H_out"), self._arg(S, self.mat_elems, "S_out")))
        return H, S

    def backward(self, P, v, gE, prec: str = "fp64", atom_xyz=None, want=("P", "v", "R")):
        dP = self._new(self.mat_elems) if "P" in want else None
        dv = self._new(self.n_points) if "v" in want else None
        dR = self._new(self.n_atoms, 3) if "R" in want else None
        with torch.cuda.device(self.device):
            self._check(self._L.aims_integrate_h_backward(
                self._h, PRECISION[prec], self._xyz(atom_xyz), self._arg(P, self.mat_elems, "P"),
                self._arg(v, self.n_points, "v"), self._arg(gE, 1, "gE", at_least=True),
                self._arg(dP, self.mat_elems, "dE_dP"), self._arg(dv, self.n_points, "dE_dv"),
                self._arg(dR, 3 * self.n_atoms, "dE_dR")))
        return dP, dv, dR

    def set_moving_grid(self, systems=None, sigma: float = 0.3, partition_a: float = 0.64):
        """Moving-grid model of each system for ``total_forces``: the owner atom and the
        pre-partition weight of every point (``pt_atom``, ``pt_wgrid`` of the systems), the
        nuclear charges (``atom_Z``), the erf width and the partition parameter."""
        systems = self._systems if systems is None else systems
        for k, s in enumerate(systems):
            owner = np.ascontiguousarray(s.pt_atom, dtype=np.int32)
            wgrid = np.ascontiguousarray(s.pt_wgrid, dtype=np.float64)
            Z = np.ascontiguousarray(s.atom_Z, dtype=np.float64)
            npt, nat = len(self._systems[k].pt_xyz), len(self._systems[k].atom_xyz)
            if owner.size != npt or wgrid.size != npt or Z.size != nat:
                raise ValueError(f"system {k}: moving-grid arrays need {npt} points and {nat} atoms")
            m = AimsMovingGrid()
            m.pt_owner = _np_ptr(owner, c_int32)
            m.pt_wgrid = _np_ptr(wgrid, c_double)
            m.atom_Z = _np_ptr(Z, c_double)
            m.nuc_sigma = float(sigma)
            m.partition_a = float(partition_a)
            self._check(self._L.aims_grid_set_moving(self._h, k, byref(m)))

    def total_forces(self, P: torch.Tensor, gE: Optional[torch.Tensor] = None, prec: str = "fp64",
                     sums_out=None):
        """(dE/dR [n_atoms, 3], sums [n_sys, 3]) of the moving-grid energy (grid points,
        partition weights, nuclear potential and basis centres all follow the atoms)."""
        gE = torch.ones(1, dtype=torch.float64, device=self.device) if gE is None else gE
        dR = self._new(self.n_atoms, 3)
        sums = self._new(self.n_sys, 3) if sums_out is None else sums_out
        with torch.cuda.device(self.device):
            self._check(self._L.aims_total_forces(
                self._h, PRECISION[prec], self._arg(P, self.mat_elems, "P"),
                self._arg(gE, 1, "gE", at_least=True), self._arg(sums, 3 * self.n_sys, "sums_out"),
                self._arg(dR, 3 * self.n_atoms, "dE_dR")))
        return dR, sums

    def integrate_h_gga(self, v: torch.Tensor, u: torch.Tensor, prec: str = "fp64", H_out=None):
        """H_ij = sum_p w phi_i (v phi_j + t phi_j + u . grad phi_j), u [n_points, 3]."""
        H = self._new(self.mat_elems) if H_out is None else H_out
        with torch.cuda.device(self.device):
            self._check(self._L.aims_integrate_h_gga(
                self._h, PRECISION[prec], self._arg(v, self.n_points, "v"),
                self._arg(u, 3 * self.n_points, "u"), self._arg(H, self.mat_elems, "H_out")))
        return H

    def xc_gga(self, n: torch.Tensor, grad_n: torch.Tensor, functional: str = "pbe"):
        """(v [n_points], u [n_points, 3], sums [n_sys, 2]) of a gradient-corrected functional:
        v = df/dn, u = 4 (df/dsigma) grad n (for ``integrate_h_gga``), sums = (E_xc,
        tr(P H_xc))."""
        v = self._new(self.n_points)
        u = self._new(self.n_points, 3)
        sums = self._new(self.n_sys, 2)
        with torch.cuda.device(self.device):
            self._check(self._L.aims_xc_gga(
                self._h, XC_FUNCTIONAL[functional], self._arg(n, self.n_points, "n"),
                self._arg(grad_n, 3 * self.n_points, "grad_n"), self._arg(v, self.n_points, "v_out"),
                self._arg(u, 3 * self.n_points, "u_out"), self._arg(sums, 2 * self.n_sys, "sums_out")))
        return v, u, sums

    def density_gradient(self, P: torch.Tensor, n_out=None, grad_out=None, want_n: bool = True):
        """(n [n_points] or None, grad n [n_points, 3]) in caller order (FP64)."""
        n = (self._new(self.n_points) if n_out is None else n_out) if want_n else None
        grad = self._new(self.n_points, 3) if grad_out is None else grad_out
        with torch.cuda.device(self.device):
            self._check(self._L.aims_density_gradient(
                self._h, self._arg(P, self.mat_elems, "P"), self._arg(n, self.n_points, "n_out"),
                self._arg(grad, 3 * self.n_points, "grad_out")))
        return n, grad

    def set_hartree_grid(self, radial, l_max: int = 6, systems=None):
        """Radial structure of every system's grid for ``hartree``: ``radial[k]`` = (pt_node,
        n_radial, r_map) of system k, pt_node the radial node of each point (caller order) on
        its owner's Becke grid; owners from the systems' ``pt_atom``."""
        systems = self._systems if systems is None else systems
        for k, s in enumerate(systems):
            node, n_radial, r_map = radial[k]
            owner = np.ascontiguousarray(s.pt_atom, dtype=np.int32)
            node = np.ascontiguousarray(node, dtype=np.int32)
            npt = len(self._systems[k].pt_xyz)
            if owner.size != npt or node.size != npt:
                raise ValueError(f"system {k}: Hartree grid arrays need {npt} points")
            h = AimsHartreeGrid()
            h.pt_owner = _np_ptr(owner, c_int32)
            h.pt_node = _np_ptr(node, c_int32)
            h.n_radial = int(n_radial)
            h.r_map = float(r_map)
            h.l_max = int(l_max)
            self._check(self._L.aims_grid_set_hartree(self._h, k, byref(h)))

    def hartree(self, n: torch.Tensor, v_out=None, E_out=None):
        """(v_H [n_points], E_H [n_sys]) of the density n (caller order)."""
        v = self._new(self.n_points) if v_out is None else v_out
        E = self._new(self.n_sys) if E_out is None else E_out
        with torch.cuda.device(self.device):
            self._check(self._L.aims_hartree(self._h, self._arg(n, self.n_points, "n"),
                                             self._arg(v, self.n_points, "v_out"),
                                             self._arg(E, self.n_sys, "E_out")))
        return v, E

    def xc(self, n: torch.Tensor, functional: str = "lda", v_out=None, sums_out=None):
        """(v_xc [n_points], sums [n_sys, 2] = (E_xc, sum w n v_xc)) of the density n (caller
        order)."""
        v = self._new(self.n_points) if v_out is None else v_out
        sums = self._new(self.n_sys, 2) if sums_out is None else sums_out
        with torch.cuda.device(self.device):
            self._check(self._L.aims_xc(self._h, XC_FUNCTIONAL[functional],
                                        self._arg(n, self.n_points, "n"),
                                        self._arg(v, self.n_points, "v_out"),
                                        self._arg(sums, 2 * self.n_sys, "sums_out")))
        return v, sums

    def density_matrix(self, H: torch.Tensor, S: torch.Tensor, n_electrons, kT: float = 0.0,
                       method: str = "eigen", P_out=None, want_eps: bool = True):
        """(P, eps or None, mu [n_sys]) of the occupied subspace: the generalised eigenproblem of
        the symmetric part of H against S ("eigen"), or trace-correcting purification
        ("purify", aufbau with an even electron count, no eigenvalues).  H, S, P hold the
        concatenated per-system blocks; ``n_electrons`` has one count per system."""
        ne = np.ascontiguousarray(np.broadcast_to(np.asarray(n_electrons, dtype=np.float64),
                                                  (self.n_sys,)))
        P = self._new(self.mat_elems) if P_out is None else P_out
        eps = self._new(int(sum(self.nb_sys))) if (want_eps and method == "eigen") else None
        mu = np.zeros(self.n_sys)
        with torch.cuda.device(self.device):
            self._check(self._L.aims_density_matrix(
                self._h, DM_METHOD[method], self._arg(H, self.mat_elems, "H"),
                self._arg(S, self.mat_elems, "S"), _np_ptr(ne, c_double), float(kT),
                self._arg(P, self.mat_elems, "P_out"), self._arg(eps, int(sum(self.nb_sys)), "eps_out"),
                _np_ptr(mu, c_double)))
        return P, eps, mu

    def last_purify_products(self) -> int:
        return int(self._L.aims_last_purify_products(self._h))

    def blocks(self, flat: torch.Tensor):
        """Views of a flat matrix buffer as one nb_s x nb_s matrix per system."""
        out, off = [], 0
        for nb in self.nb_sys:
            out.append(flat[off:off + nb * nb].view(nb, nb))
            off += nb * nb
        return out

    def work_stats(self):
        nbt = c_int64()
        s1 = c_double()
        s2 = c_double()
        self._check(self._L.aims_work_stats(self._h, byref(nbt), byref(s1), byref(s2)))
        return {"n_batches": nbt.value, "sum_np_nb2": s1.value, "sum_nb2": s2.value,
                "flops_per_step": 4.0 * s1.value}

    def get_tuning(self, prec="fp64"):
        t = AimsTuning()
        self._check(self._L.aims_get_tuning(self._h, PRECISION[prec], byref(t)))
        return {"h_merge": t.h_merge, "density_pblocks": t.density_pblocks,
                "persistent": t.persistent, "h_flops_per_atomic": t.h_flops_per_atomic,
                "h_tile32_mask": t.h_tile32_mask,
                "density_bucket_pblocks": list(t.density_bucket_pblocks)}

    def set_tuning(self, h_merge: Optional[int] = None, density_pblocks: Optional[int] = None,
                   prec="fp64", persistent: Optional[int] = None,
                   h_flops_per_atomic: Optional[int] = None, h_tile32_mask: Optional[int] = None,
                   density_bucket_pblocks: Optional[Sequence[int]] = None):
        cur = self.get_tuning(prec)
        t = AimsTuning()
        t.h_merge = int(cur["h_merge"] if h_merge is None else h_merge)
        t.density_pblocks = int(cur["density_pblocks"] if density_pblocks is None else density_pblocks)
        t.persistent = int(cur["persistent"] if persistent is None else persistent)
        t.h_flops_per_atomic = int(cur["h_flops_per_atomic"] if h_flops_per_atomic is None
                                   else h_flops_per_atomic)
        t.h_tile32_mask = int(cur["h_tile32_mask"] if h_tile32_mask is None else h_tile32_mask)
        bp = cur["density_bucket_pblocks"] if density_bucket_pblocks is None else density_bucket_pblocks
        if len(bp) != 8:
            raise ValueError("density_bucket_pblocks needs 8 entries")
        for b, x in enumerate(bp):
            t.density_bucket_pblocks[b] = int(x)
        self._check(self._L.aims_set_tuning(self._h, PRECISION[prec], byref(t)))

    def bucket_stats(self, prec="fp64", which="density"):
        """(batches, flops) per tile-shape bucket of the density partition (8) or of the
        precision's H partition (16)."""
        nbk = 8 if which == "density" else 16
        nb = (c_int64 * nbk)()
        fl = (c_double * nbk)()
        self._check(self._L.aims_bucket_stats(self._h, PRECISION[prec], 0 if which == "density" else 1,
                                              nb, fl))
        return list(nb), list(fl)

    def positions_status(self):
        """Raises AimsError (AIMS_ERR_STALE) if the last positions given as a device tensor
        failed the screening check (that call's outputs are NaN)."""
        self._check(self._L.aims_positions_status(self._h))

    def profile(self, on: bool = True):
        self._check(self._L.aims_profile_enable(self._h, 1 if on else 0))

    def profile_read(self, kernel: str):
        """(launches, total_ms, algorithmic flops) of one kernel family since profiling began."""
        n = c_int64()
        ms = c_double()
        w = c_double()
        self._check(self._L.aims_profile_read(self._h, kernel.encode(), byref(n), byref(ms), byref(w)))
        return n.value, ms.value, w.value

    def step_graph(self, P, v, n_out, sums_out, H_out, prec="fp64"):
        return StepGraph(self, P, v, n_out, sums_out, H_out, prec)

    def _xyz(self, atom_xyz):
        if atom_xyz is None:
            return None
        if isinstance(atom_xyz, torch.Tensor):
            if atom_xyz.is_cuda:
                return self._arg(atom_xyz.contiguous(), 3 * self.n_atoms, "atom_xyz")
            atom_xyz = atom_xyz.numpy()
        self._xyz_keep = np.ascontiguousarray(atom_xyz, dtype=np.float64)
        if self._xyz_keep.size != 3 * self.n_atoms:
            raise ValueError(f"atom_xyz: {self._xyz_keep.size} values, {3 * self.n_atoms} expected")
        return c_void_p(self._xyz_keep.ctypes.data)

    def close(self):
        if getattr(self, "_h", None):
            self._L.aims_grid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class StepGraph:
    """One s.c.f. step (density update + H integration) captured in a HIP graph."""

    def __init__(self, grid: AimsGrid, P, v, n_out, sums_out, H_out, prec="fp64"):
        self.grid = grid
        self._keep = (P, v, n_out, sums_out, H_out)
        h = c_void_p()
        with torch.cuda.device(grid.device):
            grid._check(grid._L.aims_step_graph_create(
                grid._h, PRECISION[prec], grid._arg(P, grid.mat_elems, "P"),
                grid._arg(v, grid.n_points, "v"), grid._arg(n_out, grid.n_points, "n_out"),
                grid._arg(sums_out, 3 * grid.n_sys, "sums_out"),
                grid._arg(H_out, grid.mat_elems, "H_out"), byref(h)))
        self._g = h

    def launch(self):
        st = self.grid._L.aims_step_graph_launch(self._g)
        if st != 0:
            raise AimsError(st, "graph launch failed")

    def __del__(self):
        try:
            if self._g:
                self.grid._L.aims_step_graph_destroy(self._g)
        except Exception:
            pass


class AimsEnergy(torch.autograd.Function):
    """E(P, v, R) = sum_p w_p v_p n(p) + sum_p w_p sum_ij P_ij phi_i tphi_j through the library.

    forward(grid, P_flat, v, R, prec) -> E (0-d float64 tensor, single system);
    backward returns dE/dP, dE/dv and dE/dR from the library's backward kernels."""

    @staticmethod
    def forward(ctx, grid: AimsGrid, P, v, R, prec="fp64"):
        if grid.n_sys != 1:
            raise ValueError("AimsEnergy handles one system per handle")
        # The backward's dE/dR takes X = Phi P and Y = (T Phi) P, which is the gradient only for
        # a symmetric P (a general P needs Phi (P + P^T)/2 and (T Phi) P^T), so another P is refused.
        # (checked outside stream capture, where reading the result back is allowed)
        nb = grid.nb_sys[0]
        Pm = P.detach().reshape(nb, nb)
        if Pm.numel() and not torch.cuda.is_current_stream_capturing():
            scale = float(Pm.abs().max())
            if float((Pm - Pm.T).abs().max()) > 1e-12 * max(scale, 1e-300):
                raise ValueError("AimsEnergy needs a symmetric P (max|P - P^T| above 1e-12 max|P|)")
        _, sums = grid.update_density(P.detach().contiguous(), v.detach().contiguous(), prec=prec,
                                      atom_xyz=R.detach())
        ctx.grid, ctx.prec = grid, prec
        ctx.save_for_backward(P, v, R)
        return sums[0, 1] + sums[0, 2]

    @staticmethod
    def backward(ctx, gE):
        P, v, R = ctx.saved_tensors
        grid = ctx.grid
        gE = gE.detach().reshape(1).to(torch.float64).contiguous()
        dP, dv, dR = grid.backward(P.detach().contiguous(), v.detach().contiguous(), gE,
                                   prec=ctx.prec, atom_xyz=R.detach())
        return None, dP.view_as(P), dv.view_as(v), dR.view_as(R), None
