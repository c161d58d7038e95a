"""A whole self-consistent-field loop through the C ABI: density -> Hartree (multipole) + LDA
exchange-correlation + the nuclear potential -> H -> density matrix -> mixed P, until the energy
and P stop changing, against the same loop on the oracle.  Both sides iterate the same map, so
their converged energies agree to the per-step parity (~1e-12), well inside the 1e-9 Ha bar."""
import numpy as np
import pytest
import torch

import synth
from oracle import GridOracle
from oracle.hartree import hartree
from oracle.scf import density_matrix
from oracle.xc import lda
from paper_2208_12335_amd import AimsGrid

pytestmark = pytest.mark.gpu

ALPHA, L_MAX, TOL_E, TOL_P, MAX_IT = 0.5, 4, 1e-10, 1e-7, 80


def _oracle_scf(inst):
    o = GridOracle(inst)
    N = float(np.sum(inst.atom_Z))
    node, K, rm = synth.radial_shells(inst)
    H0, S = o.integrate_h(inst.v)
    P = density_matrix(H0, S, N)["P"]
    E_old = None
    for it in range(MAX_IT):
        d = o.density(P, inst.v)
        n = d["n"]
        h = hartree(inst, n, node, K, rm, L_MAX)
        x = lda(n)
        E = d["E_V"] + d["E_T"] + h["E_H"] + float(np.sum(inst.pt_w * n * x["eps"]))
        H, _ = o.integrate_h(inst.v + h["v"] + x["v"], want_S=False)
        P_new = density_matrix(H, S, N)["P"]
        if E_old is not None and abs(E - E_old) < TOL_E and np.abs(P_new - P).max() < TOL_P:
            return E, it
        E_old = E
        P = (1 - ALPHA) * P + ALPHA * P_new
    raise AssertionError("oracle loop did not converge")


def _gpu_scf(inst, gpu):
    g = AimsGrid(inst, device=gpu.index)
    g.set_hartree_grid([synth.radial_shells(inst)], l_max=L_MAX)
    N = float(np.sum(inst.atom_Z))
    v_nuc = torch.from_numpy(inst.v).to(gpu)
    H0, S = g.integrate_h(v_nuc, want_S=True)
    P, _, _ = g.density_matrix(H0, S, N)
    E_old = None
    for it in range(MAX_IT):
        n, sums = g.update_density(P, v_nuc)
        vh, EH = g.hartree(n)
        vx, sx = g.xc(n)
        s = sums.cpu().numpy()[0]
        E = s[1] + s[2] + EH.item() + sx[0, 0].item()
        H, _ = g.integrate_h(v_nuc + vh + vx)
        P_new, _, _ = g.density_matrix(H, S, N, want_eps=False)
        if E_old is not None and abs(E - E_old) < TOL_E and \
                (P_new - P).abs().max().item() < TOL_P:
            return E, it
        E_old = E
        P = (1 - ALPHA) * P + ALPHA * P_new
    raise AssertionError("GPU loop did not converge")


def test_lda_hartree_scf_matches_oracle(gpu):
    inst = synth.make_instance("c1")
    E_gpu, it_gpu = _gpu_scf(inst, gpu)
    E_ref, it_ref = _oracle_scf(inst)
    print(f"[scf] triatomic LDA: E {E_gpu:.12f} ({it_gpu} iterations) vs {E_ref:.12f} "
          f"({it_ref})", flush=True)
    assert abs(E_gpu - E_ref) < 1e-9
    assert abs(it_gpu - it_ref) <= 2
