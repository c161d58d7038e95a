"""Library (HIP, through the C ABI) against the FP64 oracle on small systems.

Bar: H, S and n norm-wise within 1e-10 relative; N, E_V, E_T within 1e-10 relative."""
import numpy as np
import pytest
import torch

import synth
from oracle import GridOracle
from paper_2208_12335_amd import AimsError, AimsGrid
from conftest import relerr

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _run(inst, dev, prec="fp64", want_S=True):
    g = AimsGrid(inst, device=dev.index)
    P = torch.from_numpy(inst.P).to(dev)
    v = torch.from_numpy(inst.v).to(dev)
    n, sums = g.update_density(P.reshape(-1), v, prec=prec)
    H, S = g.integrate_h(v, prec=prec, want_S=want_S)
    torch.cuda.synchronize()
    nb = inst.n_basis
    return (g, n.cpu().numpy(), sums.cpu().numpy()[0], H.cpu().numpy().reshape(nb, nb),
            None if S is None else S.cpu().numpy().reshape(nb, nb))


def _check_against_oracle(inst, dev, tol=TOL):
    print(f"[parity] {inst.name}: {inst.n_points} points, {inst.n_basis} functions", flush=True)
    g, n, sums, H, S = _run(inst, dev)
    o = GridOracle(inst)
    d = o.density(inst.P, inst.v)
    Hr, Sr = o.integrate_h(inst.v)
    errs = {"n": relerr(n, d["n"]), "H": relerr(H, Hr), "S": relerr(S, Sr),
            "N": abs(sums[0] - d["N"]) / abs(d["N"]), "E_V": abs(sums[1] - d["E_V"]) / abs(d["E_V"]),
            "E_T": abs(sums[2] - d["E_T"]) / abs(d["E_T"])}
    print("[parity]", inst.name, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e <= tol, (k, e)
    return g, n, sums, H, S


def test_c1_fp64_parity(gpu, c1):
    g, n, sums, H, S = _check_against_oracle(c1, gpu)
    st = g.work_stats()
    assert st["n_batches"] >= 64 and st["sum_np_nb2"] > 0


@pytest.mark.parametrize("n_atoms,box,seed", [(10, 7.0, 1), (24, 11.0, 2)])
def test_small_cluster_fp64_parity_multi_tile(gpu, n_atoms, box, seed):
    # l <= 3 basis, 302-point angular grid: batches with 100-700 functions span several 64-wide
    # tiles with ragged tails in both the basis and the point dimension
    inst = synth.make_instance("c2", n_atoms=n_atoms, box=box, seed=seed)
    g, n, sums, H, S = _check_against_oracle(inst, gpu)
    # invariants on the library's own outputs
    assert abs(sums[0] - np.sum(inst.P * S)) < 1e-11 * abs(sums[0])
    assert abs(sums[1] + sums[2] - np.sum(inst.P * H)) < 1e-10 * abs(sums[1] + sums[2])


@pytest.mark.parametrize("max_batch", [1, 512])
def test_extreme_batch_sizes(gpu, max_batch):
    """Single-point batches (every tile ragged, K = 1 point in H) and the largest supported
    batch (512 points: H tiles with K = 512, density point tiles split into equal blocks)."""
    import dataclasses
    base = synth.make_instance("c2", n_atoms=6, box=6.0, seed=7)
    if max_batch == 1:           # keep the oracle fast: a random subset of 3000 points
        idx = np.sort(np.random.default_rng(3).choice(base.n_points, 3000, replace=False))
        base = dataclasses.replace(base, pt_xyz=base.pt_xyz[idx], pt_w=base.pt_w[idx],
                                   pt_atom=base.pt_atom[idx], v=base.v[idx])
    inst = dataclasses.replace(base, max_batch=max_batch)
    g, n, sums, H, S = _check_against_oracle(inst, gpu)
    assert g.work_stats()["n_batches"] == (inst.n_points if max_batch == 1 else
                                          g.work_stats()["n_batches"])


def test_determinism_and_repeat(gpu, c1):
    _, n1, s1, H1, _ = _run(c1, gpu, want_S=False)
    _, n2, s2, H2, _ = _run(c1, gpu, want_S=False)
    assert relerr(n2, n1) < 1e-15 * 10 and relerr(H2, H1) < 1e-15 * 10
    assert np.max(np.abs(s2 - s1) / np.abs(s1)) < 1e-14


def test_special_inputs(gpu, c1):
    g = AimsGrid(c1, device=gpu.index)
    nb = c1.n_basis
    P0 = torch.zeros(nb * nb, dtype=torch.float64, device=gpu)
    v = torch.from_numpy(c1.v).to(gpu)
    n, sums = g.update_density(P0, v)
    assert torch.count_nonzero(n).item() == 0 and torch.count_nonzero(sums).item() == 0
    # v = const: H(c) - H(0) = c S
    H0, S = g.integrate_h(torch.zeros_like(v), want_S=True)
    Hc, _ = g.integrate_h(torch.full_like(v, 2.5))
    assert relerr((Hc - H0).cpu().numpy(), 2.5 * S.cpu().numpy()) < 1e-12
    # P = e_i e_i^T: N = S_ii
    Pi = torch.zeros(nb, nb, dtype=torch.float64, device=gpu)
    Pi[5, 5] = 1.0
    _, sums = g.update_density(Pi.reshape(-1), v)
    assert abs(sums[0, 0].item() - S.view(nb, nb)[5, 5].item()) < 1e-12 * S.view(nb, nb)[5, 5].item()


def test_positions_and_errors(gpu, c1):
    g = AimsGrid(c1, device=gpu.index)
    P = torch.from_numpy(c1.P).to(gpu).reshape(-1)
    v = torch.from_numpy(c1.v).to(gpu)
    with pytest.raises(AimsError) as e:
        g.update_density(P, v, atom_xyz=c1.atom_xyz + np.array([0.5, 0, 0]))
    assert "STALE" in str(e.value)
    with pytest.raises(ValueError):
        g.update_density(P.cpu(), v)                       # host tensor: refused by the binding
    import ctypes
    from paper_2208_12335_amd import _lib
    Ph = P.cpu()                                           # and by the C ABI itself
    st = g._L.aims_update_density(g._h, 0, None, ctypes.c_void_p(Ph.data_ptr()),
                                  ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                                  ctypes.c_void_p(P.data_ptr()))
    assert st == _lib.AIMS_ERR_ARG and "device memory" in g._L.aims_last_error(g._h).decode()
    # moved positions (within the margin) agree with the oracle at those positions
    X = c1.atom_xyz.copy()
    X[1, 0] += 0.004
    n, sums = g.update_density(P, v, atom_xyz=X)
    d = GridOracle(c1.moved(X)).density(c1.P, c1.v)
    assert relerr(n.cpu().numpy(), d["n"]) < TOL
    # and NULL positions go back to the setup geometry
    n0, _ = g.update_density(P, v)
    d0 = GridOracle(c1).density(c1.P, c1.v)
    assert relerr(n0.cpu().numpy(), d0["n"]) < TOL


def test_allocation_failure_is_reported(gpu, c1, monkeypatch):
    """A failed device allocation (forced from the host) surfaces as AIMS_ERR_OOM with a
    message, leaves no handle behind, and a later set-up works."""
    monkeypatch.setenv("AIMS_FAIL_ALLOC", "1")
    with pytest.raises(AimsError) as e:
        AimsGrid(c1, device=gpu.index)
    assert e.value.status == -2 and "alloc" in str(e.value)
    monkeypatch.delenv("AIMS_FAIL_ALLOC")
    g = AimsGrid(c1, device=gpu.index)
    n, _ = g.update_density(torch.from_numpy(c1.P).to(gpu).reshape(-1), torch.from_numpy(c1.v).to(gpu))
    torch.cuda.synchronize()
    assert torch.isfinite(n).all()


def test_empty_grid(gpu, c1):
    import dataclasses
    e = dataclasses.replace(c1, pt_xyz=np.zeros((0, 3)), pt_w=np.zeros(0), v=np.zeros(0))
    g = AimsGrid(e, device=gpu.index)
    P = torch.from_numpy(c1.P).to(gpu).reshape(-1)
    v = torch.zeros(0, dtype=torch.float64, device=gpu)
    n, sums = g.update_density(P, v)
    H, S = g.integrate_h(v, want_S=True)
    assert n.numel() == 0 and torch.count_nonzero(sums).item() == 0
    assert torch.count_nonzero(H).item() == 0 and torch.count_nonzero(S).item() == 0
    # exchange-correlation on the empty grid: empty outputs, zero sums, zero gradient term
    vx, sx = g.xc(n)
    n2, grad = g.density_gradient(P)
    vn, u, sg = g.xc_gga(n2, grad)
    Hg = g.integrate_h_gga(v, u)
    torch.cuda.synchronize()
    assert vx.numel() == 0 and grad.numel() == 0 and u.numel() == 0
    assert torch.count_nonzero(sx).item() == 0 and torch.count_nonzero(sg).item() == 0
    assert torch.count_nonzero(Hg).item() == 0


@pytest.mark.parametrize("merge,ratio", [(0, 0), (1, 0), (2, 0), (3, 0), (0, 64), (0, 4096)])
def test_h_merge_levels_same_result(gpu, merge, ratio):
    # coarser H batches (the bisection stopped earlier, at fixed levels or where the cost model
    # prefers fewer scatter-adds) change only the rounding order
    inst = synth.make_instance("c2", n_atoms=10, box=7.0, seed=1)
    g = AimsGrid(inst, device=gpu.index)
    g.set_tuning(merge, prec="fp64", h_flops_per_atomic=ratio)
    t = g.get_tuning("fp64")
    assert t["h_merge"] == merge and t["h_flops_per_atomic"] == ratio
    v = torch.from_numpy(inst.v).to(gpu)
    H, S = g.integrate_h(v, want_S=True)
    torch.cuda.synchronize()
    nb = inst.n_basis
    Hr, Sr = GridOracle(inst).integrate_h(inst.v)
    assert relerr(H.cpu().numpy().reshape(nb, nb), Hr) < TOL
    assert relerr(S.cpu().numpy().reshape(nb, nb), Sr) < TOL


@pytest.mark.parametrize("pblocks", [2, 3, 4, 5])
def test_density_tile_widths_same_result(gpu, pblocks):
    # the density work tiles span 64 .. 160 points; every width gives the oracle's n
    inst = synth.make_instance("c2", n_atoms=10, box=7.0, seed=1)
    g = AimsGrid(inst, device=gpu.index)
    g.set_tuning(density_pblocks=pblocks, prec="fp64")
    assert g.get_tuning("fp64")["density_pblocks"] == pblocks
    P = torch.from_numpy(inst.P).to(gpu).reshape(-1)
    v = torch.from_numpy(inst.v).to(gpu)
    n, sums = g.update_density(P, v)
    torch.cuda.synchronize()
    d = GridOracle(inst).density(inst.P, inst.v)
    assert relerr(n.cpu().numpy(), d["n"]) < TOL
    s = sums.cpu().numpy()[0]
    assert abs(s[2] - d["E_T"]) < TOL * abs(d["E_T"])
