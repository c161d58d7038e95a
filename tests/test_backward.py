"""The library's backward (dE/dP, dE/dv, dE/dR) against the oracle's derivatives and against
central finite differences of the library's own energy (h = 1e-4 bohr, basis centres moved,
grid, weights and v fixed), and the torch.autograd.Function built on it."""
import numpy as np
import pytest
import torch

import synth
from oracle import GridOracle
from paper_2208_12335_amd import AimsEnergy, AimsGrid
from conftest import relerr

pytestmark = pytest.mark.gpu


def _backward(g, inst, dev, prec="fp64", gE=1.0, X=None):
    P = torch.from_numpy(inst.P).to(dev).reshape(-1)
    v = torch.from_numpy(inst.v).to(dev)
    ge = torch.tensor([gE], dtype=torch.float64, device=dev)
    dP, dv, dR = g.backward(P, v, ge, prec=prec, atom_xyz=X)
    torch.cuda.synchronize()
    nb = inst.n_basis
    return dP.cpu().numpy().reshape(nb, nb), dv.cpu().numpy(), dR.cpu().numpy()


def _energy(g, inst, dev, X, prec="fp64"):
    P = torch.from_numpy(inst.P).to(dev).reshape(-1)
    v = torch.from_numpy(inst.v).to(dev)
    _, sums = g.update_density(P, v, prec=prec, atom_xyz=X)
    s = sums.cpu().numpy()[0]
    return s[1] + s[2]


@pytest.mark.parametrize("case", ["c1", "cluster"])
def test_backward_matches_oracle_fp64(gpu, case):
    inst = synth.make_instance("c1") if case == "c1" else synth.make_instance("c2", n_atoms=8, box=7.0, seed=3)
    print(f"[backward] {inst.name}: {inst.n_points} points, {inst.n_basis} functions", flush=True)
    g = AimsGrid(inst, device=gpu.index)
    dP, dv, dR = _backward(g, inst, gpu, gE=1.7)
    ref = GridOracle(inst).gradient(inst.P, inst.v)
    e = {"dP": relerr(dP, 1.7 * ref["dE_dP"]), "dv": relerr(dv, 1.7 * ref["dE_dv"]),
         "dR": relerr(dR, 1.7 * ref["dE_dR"])}
    print(f"[backward] {inst.name} fp64 vs oracle: " + ", ".join(f"{k} {v:.2e}" for k, v in e.items()), flush=True)
    assert e["dP"] < 1e-10 and e["dv"] < 1e-10 and e["dR"] < 1e-9


def _fd_worst(g, inst, dev, dR, atoms, h=1e-4):
    worst = 0.0
    for a in atoms:
        for c in range(3):
            Xp = inst.atom_xyz.copy()
            Xp[a, c] += h
            Xm = inst.atom_xyz.copy()
            Xm[a, c] -= h
            fd = (_energy(g, inst, dev, Xp) - _energy(g, inst, dev, Xm)) / (2 * h)
            worst = max(worst, abs(fd - dR[a, c]))
    return worst


def test_backward_vs_finite_differences_triatomic(gpu, c1):
    g = AimsGrid(c1, device=gpu.index)
    _, _, dR = _backward(g, c1, gpu)
    worst = _fd_worst(g, c1, gpu, dR, range(3))
    print(f"[backward] c1: max |dE/dR - FD| = {worst:.2e} Ha/bohr", flush=True)
    assert worst < 1e-6


def test_backward_vs_finite_differences_cluster(gpu):
    # the 128-atom differentiation workload's density (16 atoms in a 12.6 bohr box).  With a
    # randomly signed P the energy is a sum of terms far larger than itself, so its FP64
    # rounding noise (~1e-8 Ha here) divided by h, plus the O(h^2) truncation, bounds how well
    # any FD can agree: the bar is 1e-6 + 1e-8 max|dE/dR| (the analytic gradient is held to
    # the oracle's at 1e-9 relative in test_backward_matches_oracle_fp64).
    inst = synth.make_instance("c2", n_atoms=16, box=12.6, seed=4)
    g = AimsGrid(inst, device=gpu.index)
    _, _, dR = _backward(g, inst, gpu)
    rng = np.random.default_rng(7)
    atoms = rng.choice(inst.n_atoms, 8, replace=False)
    worst = _fd_worst(g, inst, gpu, dR, atoms)
    bar = 1e-6 + 1e-8 * np.max(np.abs(dR))
    print(f"[backward] 16-atom cluster, 8 atoms: max |dE/dR - FD| = {worst:.2e} Ha/bohr "
          f"(bar {bar:.1e}, max |dE/dR| {np.max(np.abs(dR)):.1e})", flush=True)
    assert worst < bar


@pytest.mark.parametrize("prec,bound", [("fp32", 1e-4), ("bf16x3", 1e-2)])
def test_backward_mixed_error_stated(gpu, prec, bound):
    inst = synth.make_instance("c2", n_atoms=8, box=7.0, seed=3)
    g = AimsGrid(inst, device=gpu.index)
    dP64, dv64, dR64 = _backward(g, inst, gpu)
    dP, dv, dR = _backward(g, inst, gpu, prec=prec)
    e = {"dP": relerr(dP, dP64), "dv": relerr(dv, dv64), "dR": relerr(dR, dR64),
         "dR_abs": float(np.max(np.abs(dR - dR64)))}
    print(f"[backward] {prec} vs fp64: " + ", ".join(f"{k} {v:.2e}" for k, v in e.items()), flush=True)
    assert e["dP"] < bound and e["dv"] < bound and e["dR"] < bound


def test_autograd_function(gpu):
    inst = synth.make_instance("c1")
    g = AimsGrid(inst, device=gpu.index)
    P = torch.from_numpy(inst.P).to(gpu).requires_grad_(True)
    v = torch.from_numpy(inst.v).to(gpu).requires_grad_(True)
    R = torch.from_numpy(inst.atom_xyz.copy()).to(gpu).requires_grad_(True)
    E = AimsEnergy.apply(g, P, v, R, "fp64")
    E.backward()
    ref = GridOracle(inst).gradient(inst.P, inst.v)
    assert abs(E.item() - ref["E"]) < 1e-10 * abs(ref["E"])
    assert relerr(P.grad.cpu().numpy(), ref["dE_dP"]) < 1e-10
    assert relerr(v.grad.cpu().numpy(), ref["dE_dv"]) < 1e-10
    assert relerr(R.grad.cpu().numpy(), ref["dE_dR"]) < 1e-9
    # second use of the same handle with moved centres (within the screening margin)
    R2 = (R.detach() + 0.003).requires_grad_(True)
    E2 = AimsEnergy.apply(g, P.detach(), v.detach(), R2, "fp64")
    ref2 = GridOracle(inst.moved(R2.detach().cpu().numpy())).energy(inst.P, inst.v)
    assert abs(E2.item() - ref2) < 1e-10 * abs(ref2)


def test_short_buffers_and_asymmetric_P_refused(gpu):
    """Caller buffers shorter than the call needs are refused on the host, by the binding and by
    the C ABI itself (allocation range of the device pointer), before any launch; AimsEnergy
    refuses a density matrix that is not symmetric (its backward assumes P = P^T)."""
    import ctypes
    from paper_2208_12335_amd import _lib
    inst = synth.make_instance("c1")
    g = AimsGrid(inst, device=gpu.index)
    P = torch.from_numpy(inst.P).to(gpu).reshape(-1)
    v = torch.from_numpy(inst.v).to(gpu)
    with pytest.raises(ValueError):
        g.update_density(P[:-1].contiguous(), v)
    L = _lib.load()
    # a buffer of its own allocation, half of n_points, straight through the C ABI
    hip = ctypes.CDLL("libamdhip64.so")
    raw = ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(raw), ctypes.c_size_t(8 * (inst.n_points // 2))) == 0
    try:
        sums = torch.empty(3, dtype=torch.float64, device=gpu)
        st = L.aims_update_density(g._h, 0, None, ctypes.c_void_p(P.data_ptr()),
                                   ctypes.c_void_p(v.data_ptr()), raw, ctypes.c_void_p(sums.data_ptr()))
        msg = L.aims_last_error(g._h).decode()
        print(f"[abi] short n_out: status {st}, {msg}", flush=True)
        assert st == _lib.AIMS_ERR_ARG and "n_out" in msg
    finally:
        torch.cuda.synchronize()
        hip.hipFree(raw)
    nb = inst.n_basis
    Pa = inst.P.copy()
    Pa[0, 1] += 1e-3
    with pytest.raises(ValueError, match="symmetric"):
        AimsEnergy.apply(g, torch.from_numpy(Pa).to(gpu).reshape(-1), v,
                         torch.from_numpy(inst.atom_xyz).to(gpu).reshape(-1, 3))
    assert nb > 0


def test_device_positions_checked_on_device(gpu):
    """Positions given as a device tensor are copied and checked on the device with no host
    synchronisation: valid ones give the host-array result; an atom beyond screen_margin makes
    the call's outputs NaN and aims_positions_status report AIMS_ERR_STALE; NULL positions
    restore the set-up geometry and clear the flag."""
    from paper_2208_12335_amd import AimsError
    inst = synth.make_instance("c1")
    g = AimsGrid(inst, device=gpu.index)
    P = torch.from_numpy(inst.P).to(gpu).reshape(-1)
    v = torch.from_numpy(inst.v).to(gpu)
    X = inst.atom_xyz.copy()
    X[1, 2] += 0.004
    n_h, s_h = g.update_density(P, v, atom_xyz=X)
    n_d, s_d = g.update_density(P, v, atom_xyz=torch.from_numpy(X).to(gpu))
    torch.cuda.synchronize()
    assert relerr(n_d.cpu().numpy(), n_h.cpu().numpy()) < 1e-14
    g.positions_status()
    Xs = inst.atom_xyz.copy()
    Xs[0, 0] += 0.5
    n_s, s_s = g.update_density(P, v, atom_xyz=torch.from_numpy(Xs).to(gpu))
    H_s, _ = g.integrate_h(v, atom_xyz=torch.from_numpy(Xs).to(gpu))
    torch.cuda.synchronize()
    assert torch.isnan(n_s).all() and torch.isnan(s_s).all() and torch.isnan(H_s).all()
    with pytest.raises(AimsError) as e:
        g.positions_status()
    assert e.value.status == -4
    n0, _ = g.update_density(P, v)
    torch.cuda.synchronize()
    g.positions_status()
    ref = GridOracle(inst).density(inst.P, inst.v)
    assert relerr(n0.cpu().numpy(), ref["n"]) < 1e-10


def test_autograd_step_captured_in_a_graph(gpu):
    """One AimsEnergy forward + backward captured with torch.cuda.graph on the handle's stream
    (positions as a device tensor, no host synchronisation inside) and replayed three times at
    new positions written into the captured tensor: E and every gradient match eager calls."""
    inst = synth.make_instance("c1")
    s = torch.cuda.Stream(device=gpu)
    g = AimsGrid(inst, device=gpu.index, stream=s)
    P = torch.from_numpy(inst.P).to(gpu).reshape(-1).clone().requires_grad_(True)
    v = torch.from_numpy(inst.v).to(gpu).clone().requires_grad_(True)
    R = torch.from_numpy(inst.atom_xyz).to(gpu).clone().requires_grad_(True)

    def step():
        for t in (P, v, R):
            t.grad = None
        E = AimsEnergy.apply(g, P, v, R)
        E.backward()
        return E

    with torch.cuda.stream(s):
        for _ in range(2):                   # warm-up: buffers of the backward, work lists
            step()
    s.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        E_cap = step()
    gP, gv, gR = P.grad, v.grad, R.grad
    rng = np.random.default_rng(7)
    for rep in range(3):
        X = inst.atom_xyz + rng.uniform(-3e-3, 3e-3, inst.atom_xyz.shape)
        with torch.no_grad():
            R.copy_(torch.from_numpy(X))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        E_g, dP_g, dv_g, dR_g = (float(E_cap), gP.cpu().numpy().copy(), gv.cpu().numpy().copy(),
                                 gR.cpu().numpy().copy())
        with torch.cuda.stream(s):
            E_e = step()
        s.synchronize()
        print(f"[graph] replay {rep}: E {E_g:.12f} eager {float(E_e):.12f}", flush=True)
        assert abs(E_g - float(E_e)) <= 1e-12 * abs(float(E_e))
        assert relerr(dP_g, P.grad.cpu().numpy()) < 1e-12
        assert relerr(dv_g, v.grad.cpu().numpy()) < 1e-12
        assert relerr(dR_g, R.grad.cpu().numpy()) < 1e-12
