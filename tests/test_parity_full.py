"""Library against the oracle at the full size of the 64-atom cluster workload (the benchmark's
configuration), on outputs the oracle can compute one by one: n at sampled points, H and S
blocks of sampled atom pairs.  Properties that hold at any size are checked on everything."""
import numpy as np
import pytest
import torch

import synth
from oracle import GridOracle
from paper_2208_12335_amd import AimsGrid
from paper_2208_12335_amd.autotune import autotune
from conftest import pair_block, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2_run(gpu):
    inst = synth.make_instance("c2", seed=0)
    print(f"[full] c2: {inst.n_points} points, {inst.n_basis} functions", flush=True)
    g = AimsGrid(inst, device=gpu.index)
    P = torch.from_numpy(inst.P).to(gpu).reshape(-1)
    v = torch.from_numpy(inst.v).to(gpu)
    # the launch configuration the benchmark times: the autotuner's choice on this device
    r = autotune(g, P, v, prec="fp64", reps=1, cache="")
    print(f"[full] tuning {g.get_tuning('fp64')}", flush=True)
    n, sums = g.update_density(P, v)
    H, S = g.integrate_h(v, want_S=True)
    torch.cuda.synchronize()
    nb = inst.n_basis
    out = {"n": n.cpu().numpy(), "sums": sums.cpu().numpy()[0],
           "H": H.cpu().numpy().reshape(nb, nb), "S": S.cpu().numpy().reshape(nb, nb)}
    return inst, g, out


def test_c2_density_sampled_points(c2_run):
    inst, g, out = c2_run
    o = GridOracle(inst)
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(inst.n_points, 3000, replace=False))
    d = o.density(inst.P, inst.v, points=idx)
    e = relerr(out["n"][idx], d["n"])
    print(f"[full] n on 3000 sampled points: {e:.2e}", flush=True)
    assert e < 1e-10


def test_c2_h_and_s_sampled_blocks(c2_run):
    inst, g, out = c2_run
    o = GridOracle(inst)
    rng = np.random.default_rng(12)
    worst_H = worst_S = 0.0
    pairs = [(int(a), int(b)) for a, b in rng.integers(0, inst.n_atoms, size=(6, 2))] + [(3, 3)]
    for a, b in pairs:
        ca, cb, Hr, Sr = pair_block(o, inst, a, b, inst.v)
        worst_H = max(worst_H, relerr(out["H"][np.ix_(ca, cb)], Hr) if np.abs(Hr).max() > 0 else 0)
        worst_S = max(worst_S, relerr(out["S"][np.ix_(ca, cb)], Sr) if np.abs(Sr).max() > 0 else 0)
    print(f"[full] sampled H blocks {worst_H:.2e}, S blocks {worst_S:.2e}", flush=True)
    assert worst_H < 1e-10 and worst_S < 1e-10


def test_c2_whole_output_properties(c2_run):
    inst, g, out = c2_run
    N, EV, ET = out["sums"]
    assert abs(N - np.sum(inst.P * out["S"])) < 1e-11 * abs(N)
    assert abs(EV + ET - np.sum(inst.P * out["H"])) < 1e-10 * abs(EV + ET)
    S = out["S"]
    assert np.max(np.abs(S - S.T)) < 1e-13 * np.max(np.abs(S))
    assert np.all(np.isfinite(out["n"])) and np.all(np.isfinite(out["H"]))


def test_c2_whole_sums_against_oracle(c2_run):
    """N, E_V and E_T over every point of the workload against the oracle's full density pass
    (about a minute on the host cores)."""
    inst, g, out = c2_run
    d = GridOracle(inst).density(inst.P, inst.v)
    N, EV, ET = out["sums"]
    errs = {"N": abs(N - d["N"]) / abs(d["N"]), "E_V": abs(EV - d["E_V"]) / abs(d["E_V"]),
            "E_T": abs(ET - d["E_T"]) / abs(d["E_T"]), "n": relerr(out["n"], d["n"])}
    print("[full] whole-workload sums vs oracle: " + ", ".join(f"{k} {e:.2e}" for k, e in errs.items())
          + f"; |dE| = {abs(EV + ET - d['E_V'] - d['E_T']):.2e} Ha", flush=True)
    assert max(errs.values()) < 1e-10
