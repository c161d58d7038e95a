"""Total (moving-grid) energy gradient through the C ABI against the oracle.

The energy is E(R) = sum_p w_p(R) [v(p; R) n(p; R) + sum_ij P_ij phi_i tphi_j] with the grid
points, their Stratmann partition weights, the erf nuclear potential and the basis centres all
following the atoms.  Bars: FP64 gradient within 1e-9 of the largest component of the oracle's
autograd gradient and E within 1e-10 relative; translation invariance and finite differences
over grids rebuilt at displaced atoms for a 10-atom cluster; the FP32 form's deviation from
FP64 is stated.

The finite-difference bar is 1e-7 of max|F|, not tighter: the natural cubic spline in ln r
ends at the cutoff rc with a small nonzero slope (dR/dr up to ~3e-4, dK/dr up to ~6e-2 for
these radial functions), so E(R) has tiny derivative jumps wherever a grid point crosses another
atom's cutoff sphere, and a difference quotient over +-2h averages over them.  The oracle's own
gradient shows the same ~2e-8 max|F| scatter against these quotients at h = 2e-3, 1e-3, 5e-4."""
import numpy as np
import pytest
import torch

import synth
from oracle import GridOracle
from oracle.forces import moving_grid_gradient
from paper_2208_12335_amd import AimsError, AimsGrid

pytestmark = pytest.mark.gpu


def _gpu_forces(inst, gpu, prec="fp64"):
    g = AimsGrid(inst, device=gpu.index)
    g.set_moving_grid()
    P = torch.from_numpy(inst.P).to(gpu).reshape(-1)
    dR, sums = g.total_forces(P, prec=prec)
    torch.cuda.synchronize()
    s = sums.cpu().numpy()[0]
    return g, dR.cpu().numpy(), s[1] + s[2]


@pytest.mark.parametrize("path", ["wave", "thread"])
@pytest.mark.parametrize("which", ["triatomic", "grown5"])
def test_total_forces_match_oracle(gpu, which, path, monkeypatch):
    # the thread-per-point kernel serves systems above 512 atoms; the switch (read at setup)
    # runs it on small systems too
    monkeypatch.setenv("AIMS_FORCES_THREAD_PATH", "1" if path == "thread" else "0")
    inst = (synth.make_instance("c1") if which == "triatomic" else
            synth.make_molecule_set(n_mol=1, seed=3, n_min=5, n_max=5)[0])
    print(f"[forces] {which} ({path}): {inst.n_points} points, {inst.n_atoms} atoms", flush=True)
    g, F, E = _gpu_forces(inst, gpu)
    E_ref, F_ref = moving_grid_gradient(GridOracle(inst), inst.P)
    err = np.max(np.abs(F - F_ref)) / np.max(np.abs(F_ref))
    print(f"[forces] {which}: max|dF|/max|F| = {err:.2e}, E {E:.12f} vs {E_ref:.12f}", flush=True)
    assert err <= 1e-9
    assert abs(E - E_ref) <= 1e-10 * abs(E_ref)
    # the moving-grid terms are not negligible: the fixed-grid (Pulay) gradient differs
    _, _, dRp = g.backward(torch.from_numpy(inst.P).to(gpu).reshape(-1),
                           torch.from_numpy(inst.v).to(gpu),
                           torch.ones(1, dtype=torch.float64, device=gpu), want=("R",))
    assert np.max(np.abs(dRp.cpu().numpy() - F)) > 1e-4 * np.max(np.abs(F))


def test_total_forces_cluster_invariance_and_finite_differences(gpu, monkeypatch):
    with synth.generator_device(gpu):
        inst = synth.make_instance("c2", n_atoms=10, box=7.5, seed=4)
    print(f"[forces] cluster: {inst.n_points} points, {inst.n_atoms} atoms", flush=True)
    _, F, E = _gpu_forces(inst, gpu)
    tot = F.sum(axis=0)
    Fmax = np.max(np.abs(F))
    print(f"[forces] cluster: sum of forces {tot}, max|F| {Fmax:.3e}", flush=True)
    assert np.max(np.abs(tot)) <= 1e-9 * Fmax + 1e-9
    E_ref, F_ref = moving_grid_gradient(GridOracle(inst), inst.P, chunk=4096)
    err = np.max(np.abs(F - F_ref)) / np.max(np.abs(F_ref))
    print(f"[forces] cluster vs oracle: max|dF|/max|F| = {err:.2e}, E {E:.10f} vs {E_ref:.10f}",
          flush=True)
    assert err <= 1e-9
    assert abs(E - E_ref) <= 1e-10 * abs(E_ref)
    # repeatability: the moving-grid sums are added in a fixed order, the Pulay pass's per-point
    # atomics may still change the last bits
    _, F2, _ = _gpu_forces(inst, gpu)
    assert np.max(np.abs(F2 - F)) <= 1e-13 * Fmax
    monkeypatch.setenv("AIMS_FORCES_THREAD_PATH", "1")
    _, F3, _ = _gpu_forces(inst, gpu)
    monkeypatch.delenv("AIMS_FORCES_THREAD_PATH")
    print(f"[forces] cluster thread vs wave kernel: {np.max(np.abs(F3 - F)) / Fmax:.2e}", flush=True)
    assert np.max(np.abs(F3 - F)) <= 1e-12 * Fmax

    P = torch.from_numpy(inst.P).to(gpu).reshape(-1)

    def energy(xyz):
        with synth.generator_device(gpu):
            r = synth.regrid(inst, xyz)
        g = AimsGrid(r, device=gpu.index)
        _, s = g.update_density(P, torch.from_numpy(r.v).to(gpu))
        s = s.cpu().numpy()[0]
        return s[1] + s[2]

    rng = np.random.default_rng(21)
    h = 1e-3
    for a in rng.choice(inst.n_atoms, 3, replace=False):
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        e = np.zeros_like(inst.atom_xyz)
        e[a] = u
        d1 = (energy(inst.atom_xyz + h * e) - energy(inst.atom_xyz - h * e)) / (2 * h)
        d2 = (energy(inst.atom_xyz + 2 * h * e) - energy(inst.atom_xyz - 2 * h * e)) / (4 * h)
        fd = (4 * d1 - d2) / 3
        an = float(F[a] @ u)
        print(f"[forces] atom {a}: analytic {an:.9f}, finite difference {fd:.9f}", flush=True)
        assert abs(an - fd) <= 1e-7 * Fmax


def test_total_forces_grouped_molecules(gpu):
    """One handle over several molecules: per-system ranges and slots, each system against its
    own oracle gradient."""
    mols = synth.make_molecule_set(n_mol=4, seed=11, n_min=2, n_max=6)
    g = AimsGrid(mols, device=gpu.index)
    g.set_moving_grid()
    P = torch.cat([torch.from_numpy(m.P).reshape(-1) for m in mols]).to(gpu)
    dR, sums = g.total_forces(P)
    dR = dR.cpu().numpy()
    sums = sums.cpu().numpy()
    a = 0
    for k, m in enumerate(mols):
        E_ref, F_ref = moving_grid_gradient(GridOracle(m), m.P)
        F = dR[a:a + m.n_atoms]
        a += m.n_atoms
        err = np.max(np.abs(F - F_ref)) / np.max(np.abs(F_ref))
        print(f"[forces] molecule {k} ({m.n_atoms} atoms): max|dF|/max|F| = {err:.2e}", flush=True)
        assert err <= 1e-9
        assert abs(sums[k, 1] + sums[k, 2] - E_ref) <= 1e-10 * abs(E_ref)


def test_total_forces_fp32_stated_and_errors(gpu):
    inst = synth.make_instance("c2", n_atoms=6, box=6.0, seed=7)
    _, F64, E64 = _gpu_forces(inst, gpu, "fp64")
    _, F32, E32 = _gpu_forces(inst, gpu, "fp32")
    err = np.max(np.abs(F32 - F64)) / np.max(np.abs(F64))
    print(f"[forces] fp32 vs fp64: max|dF|/max|F| = {err:.2e}, |dE| = {abs(E32 - E64):.2e}", flush=True)
    assert err <= 1e-3
    g = AimsGrid(inst, device=gpu.index)
    P = torch.from_numpy(inst.P).to(gpu).reshape(-1)
    with pytest.raises(AimsError) as e:            # no model set yet
        g.total_forces(P)
    assert e.value.status == -1
    g.set_moving_grid()
    with pytest.raises(AimsError) as e:
        g.total_forces(P, prec="bf16x3")
    assert e.value.status == -5
