"""Library against the oracle on the three larger workload families at full size: the 512-atom
water cluster, the 256-molecule grouped set and the 128-atom cluster with the backward.

The oracle cannot integrate these whole in test time, so it checks outputs it can compute one
by one (n at sampled points, H/S blocks of sampled atom pairs, whole small molecules of the
set), and properties that hold at any size are checked on everything (N = tr(PS),
E = tr(PH), S symmetric, dE/dP = H, dE/dv = w n, a directional finite difference of E for
dE/dR).  Inputs are generated with the generator's arithmetic on the GPU (same definitions as
on the CPU, agreeing to rounding)."""
import numpy as np
import pytest
import torch

import synth
from conftest import pair_block, relerr
from oracle import GridOracle
from paper_2208_12335_amd import AimsGrid

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _forward(inst_list, gpu, want_S=True, prec="fp64"):
    g = AimsGrid(inst_list, device=gpu.index)
    P = torch.cat([torch.from_numpy(m.P).reshape(-1) for m in inst_list]).to(gpu)
    v = torch.cat([torch.from_numpy(m.v) for m in inst_list]).to(gpu)
    n, sums = g.update_density(P, v, prec=prec)
    H, S = g.integrate_h(v, prec=prec, want_S=want_S)
    torch.cuda.synchronize()
    return g, P, v, n, sums, H, S


def _sampled_checks(inst, n, H, S, seed, n_pts=2000, n_pairs=4):
    o = GridOracle(inst)
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(inst.n_points, min(n_pts, inst.n_points), replace=False))
    d = o.density(inst.P, inst.v, points=idx)
    en = relerr(n[idx], d["n"])
    worst_H = worst_S = 0.0
    # pairs of near atoms (nonzero blocks), plus one diagonal block
    for _ in range(n_pairs):
        a = int(rng.integers(inst.n_atoms))
        dist = np.linalg.norm(inst.atom_xyz - inst.atom_xyz[a], axis=1)
        near = np.nonzero((dist < inst.rc) & (dist > 0))[0]
        b = int(rng.choice(near)) if near.size else a
        ca, cb, Hr, Sr = pair_block(o, inst, a, b, inst.v)
        worst_H = max(worst_H, relerr(H[np.ix_(ca, cb)], Hr))
        if S is not None:
            worst_S = max(worst_S, relerr(S[np.ix_(ca, cb)], Sr))
    ca, cb, Hr, Sr = pair_block(o, inst, 0, 0, inst.v)
    worst_H = max(worst_H, relerr(H[np.ix_(ca, cb)], Hr))
    if S is not None:
        worst_S = max(worst_S, relerr(S[np.ix_(ca, cb)], Sr))
    return en, worst_H, worst_S


def test_c3_water_cluster_full_size(gpu):
    with synth.generator_device(gpu):
        inst = synth.make_instance("c3", seed=0)
    print(f"[c3] {inst.n_points} points, {inst.n_basis} functions", flush=True)
    g, P, v, n, sums, H, S = _forward([inst], gpu)
    nb = inst.n_basis
    n = n.cpu().numpy()
    s = sums.cpu().numpy()[0]
    Hh = H.cpu().numpy().reshape(nb, nb)
    Sh = S.cpu().numpy().reshape(nb, nb)
    del H, S
    en, eH, eS = _sampled_checks(inst, n, Hh, Sh, seed=31)
    print(f"[c3] n {en:.2e}, H blocks {eH:.2e}, S blocks {eS:.2e}", flush=True)
    assert en < TOL and eH < TOL and eS < TOL
    assert abs(s[0] - np.sum(inst.P * Sh)) < 1e-11 * abs(s[0])
    assert abs(s[1] + s[2] - np.sum(inst.P * Hh)) < 1e-10 * abs(s[1] + s[2])
    assert np.max(np.abs(Sh - Sh.T)) < 1e-13 * np.max(np.abs(Sh))
    st = g.work_stats()
    assert st["n_batches"] >= 16384


def test_c4_molecule_set_full_size(gpu):
    with synth.generator_device(gpu):
        mols = synth.make_molecule_set(n_mol=256, seed=0)
    npts = sum(m.n_points for m in mols)
    print(f"[c4] {len(mols)} molecules, {npts} points, {sum(m.n_basis for m in mols)} functions",
          flush=True)
    g, P, v, n, sums, H, S = _forward(mols, gpu)
    g.set_tuning(persistent=1, prec="fp64")
    n2, sums2 = g.update_density(P, v)
    H2, _ = g.integrate_h(v)
    torch.cuda.synchronize()
    assert relerr(n2.cpu().numpy(), n.cpu().numpy()) < 1e-13
    assert relerr(H2.cpu().numpy(), H.cpu().numpy()) < 1e-13
    Hb = [h.cpu().numpy() for h in g.blocks(H)]
    Sb = [x.cpu().numpy() for x in g.blocks(S)]
    sums = sums.cpu().numpy()
    n = n.cpu().numpy()
    # properties of every molecule
    off = np.concatenate([[0], np.cumsum([m.n_points for m in mols])])
    for k, m in enumerate(mols):
        assert abs(sums[k, 0] - np.sum(m.P * Sb[k])) < 1e-11 * abs(sums[k, 0]), k
        assert abs(sums[k, 1] + sums[k, 2] - np.sum(m.P * Hb[k])) < 1e-10 * abs(sums[k, 1] + sums[k, 2]), k
    # whole molecules against the oracle: the smallest, the largest and two random ones
    rng = np.random.default_rng(41)
    sizes = [m.n_atoms for m in mols]
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)),
                   *[int(x) for x in rng.choice(len(mols), 2, replace=False)]})
    for k in pick:
        m = mols[k]
        o = GridOracle(m)
        if m.n_points <= 60000:
            d = o.density(m.P, m.v)
            Hr, Sr = o.integrate_h(m.v)
            errs = (relerr(n[off[k]:off[k + 1]], d["n"]), relerr(Hb[k], Hr), relerr(Sb[k], Sr))
        else:
            errs = _sampled_checks(m, n[off[k]:off[k + 1]], Hb[k], Sb[k], seed=k, n_pts=1000,
                                   n_pairs=2)
        print(f"[c4] molecule {k} ({m.n_atoms} atoms): n {errs[0]:.2e} H {errs[1]:.2e} "
              f"S {errs[2]:.2e}", flush=True)
        assert max(errs) < TOL, (k, errs)


def test_c5_forward_and_backward_full_size(gpu):
    with synth.generator_device(gpu):
        inst = synth.make_instance("c5", seed=0)
    print(f"[c5] {inst.n_points} points, {inst.n_basis} functions", flush=True)
    g, P, v, n, sums, H, S = _forward([inst], gpu, want_S=False)
    nb = inst.n_basis
    Hh = H.cpu().numpy().reshape(nb, nb)
    en, eH, _ = _sampled_checks(inst, n.cpu().numpy(), Hh, None, seed=51, n_pairs=3)
    print(f"[c5] n {en:.2e}, H blocks {eH:.2e}", flush=True)
    assert en < TOL and eH < TOL
    gE = torch.full((1,), 0.75, dtype=torch.float64, device=gpu)
    dP, dv, dR = g.backward(P, v, gE)
    torch.cuda.synchronize()
    # dE/dP = gE H, dE/dv = gE w n (same kernels' arithmetic up to summation order)
    assert relerr(dP.cpu().numpy(), 0.75 * H.cpu().numpy()) < 1e-13
    w = torch.from_numpy(inst.pt_w).to(gpu)
    assert relerr(dv.cpu().numpy(), (0.75 * w * n).cpu().numpy()) < 1e-13
    # dE/dR along two random directions (every atom moves) against a Richardson-extrapolated
    # central difference of the library's FP64 energy (steps 2h and h: truncation O(h^4));
    # E's rounding noise over the steps bounds the bar
    dR = dR.cpu().numpy() / 0.75
    rng = np.random.default_rng(52)
    h = 1e-3

    def energy(x):
        _, s = g.update_density(P, v, atom_xyz=x)
        s = s.cpu().numpy()[0]
        return s[1] + s[2]

    for _ in range(2):
        u = rng.standard_normal(inst.atom_xyz.shape)
        u /= np.linalg.norm(u)
        d1 = (energy(inst.atom_xyz + h * u) - energy(inst.atom_xyz - h * u)) / (2 * h)
        d2 = (energy(inst.atom_xyz + 2 * h * u) - energy(inst.atom_xyz - 2 * h * u)) / (4 * h)
        fd = (4 * d1 - d2) / 3
        an = float(np.sum(dR * u))
        print(f"[c5] directional dE/dR: analytic {an:.10f}, finite difference {fd:.10f} "
              f"(central {d1:.10f})", flush=True)
        assert abs(an - fd) < 1e-4 + 1e-5 * abs(an)
