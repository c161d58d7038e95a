"""Persistent tile launches, step-graph replay, grouped many-molecule handles and the live
autotuner, each checked against the plain per-call / per-molecule path and the FP64 oracle.

Bars: the persistent and graph paths do the same arithmetic as the one-workgroup-per-tile
path, up to the order of the FP64 scatter-adds into H and n: 1e-13 relative.  A grouped handle
computes every molecule exactly as a handle of its own: 1e-12 relative.  Against the oracle:
the FP64 bar of 1e-10."""
import numpy as np
import pytest
import torch

import synth
from conftest import relerr
from oracle import GridOracle
from paper_2208_12335_amd import AimsGrid
from paper_2208_12335_amd.autotune import autotune

pytestmark = pytest.mark.gpu
SAME = 1e-13


def _step(g, P, v, prec="fp64"):
    n, sums = g.update_density(P, v, prec=prec)
    H, S = g.integrate_h(v, prec=prec, want_S=True)
    torch.cuda.synchronize()
    return n.cpu().numpy(), sums.cpu().numpy(), H.cpu().numpy(), S.cpu().numpy()


@pytest.fixture(scope="module")
def cluster():
    # l <= 3 basis, several 64-wide tiles per batch, ragged tails
    return synth.make_instance("c2", n_atoms=12, box=8.0, seed=3)


@pytest.mark.parametrize("prec,scratch_mb", [("fp64", None), ("fp32", None), ("bf16x3", None),
                                              ("fp64", "16"), ("bf16x3", "16")])
def test_persistent_matches_grid_launch(gpu, cluster, prec, scratch_mb, monkeypatch):
    """Persistent launches (resident grid, per-XCD work counters) against one workgroup per
    tile; a 16 MB scratch budget cuts each pass into many groups of batches, so that the
    counters are cleared and reused across many launches of one call."""
    if scratch_mb:
        monkeypatch.setenv("AIMS_SCRATCH_MB", scratch_mb)
    print(f"[persistent] {prec} {cluster.n_points} points, scratch {scratch_mb}", flush=True)
    g = AimsGrid(cluster, device=gpu.index)
    P = torch.from_numpy(cluster.P).to(gpu).reshape(-1)
    v = torch.from_numpy(cluster.v).to(gpu)
    ref = _step(g, P, v, prec)
    g.set_tuning(persistent=1, prec=prec)
    assert g.get_tuning(prec)["persistent"] == 1
    for _ in range(2):                      # the counters are cleared on every call
        out = _step(g, P, v, prec)
        for a, b, name in zip(out, ref, ("n", "sums", "H", "S")):
            assert relerr(a, b) <= SAME, (prec, name, relerr(a, b))
    if prec == "fp64":
        o = GridOracle(cluster)
        d = o.density(cluster.P, cluster.v)
        Hr, Sr = o.integrate_h(cluster.v)
        assert relerr(out[0], d["n"]) <= 1e-10
        assert relerr(out[2], Hr.reshape(-1)) <= 1e-10
        assert relerr(out[3], Sr.reshape(-1)) <= 1e-10


@pytest.mark.parametrize("persistent", [0, 1])
def test_step_graph_replays(gpu, cluster, persistent):
    """Replays with eager work and host syncs in between; every replay matches an eager step
    on the same inputs."""
    print(f"[graph] persistent={persistent}", flush=True)
    g = AimsGrid(cluster, device=gpu.index, stream=torch.cuda.Stream(gpu))
    g.set_tuning(persistent=persistent, h_merge=2, prec="fp64")
    P0 = torch.from_numpy(cluster.P).to(gpu).reshape(-1)
    v0 = torch.from_numpy(cluster.v).to(gpu)
    P = P0.clone()
    v = v0.clone()
    n = torch.empty(g.n_points, dtype=torch.float64, device=gpu)
    sums = torch.empty(1, 3, dtype=torch.float64, device=gpu)
    H = torch.empty(g.mat_elems, dtype=torch.float64, device=gpu)
    with torch.cuda.stream(g.stream):
        graph = g.step_graph(P, v, n, sums, H, prec="fp64")
    for k, scale in enumerate((1.0, 0.5, -1.25, 1.0)):
        with torch.cuda.stream(g.stream):
            P.copy_(P0 * scale)
            v.copy_(v0 * (1.0 + 0.1 * k))
            graph.launch()
        torch.cuda.synchronize()
        got = (n.cpu().numpy().copy(), sums.cpu().numpy().copy(), H.cpu().numpy().copy())
        # eager work between replays, into other buffers, on the same stream
        with torch.cuda.stream(g.stream):
            ne, se = g.update_density(P, v)
            He, _ = g.integrate_h(v)
        torch.cuda.synchronize()
        ref = (ne.cpu().numpy(), se.cpu().numpy(), He.cpu().numpy())
        for a, b, name in zip(got, ref, ("n", "sums", "H")):
            assert relerr(a, b) <= SAME, (k, name, relerr(a, b))
    del graph


@pytest.fixture(scope="module")
def molecules():
    return synth.make_molecule_set(n_mol=6, seed=5, n_min=3, n_max=14)


@pytest.mark.parametrize("persistent", [0, 1])
def test_grouped_handle_matches_single(gpu, molecules, persistent):
    print(f"[grouped] {len(molecules)} molecules, persistent={persistent}", flush=True)
    gg = AimsGrid(molecules, device=gpu.index)
    gg.set_tuning(persistent=persistent, prec="fp64")
    P = torch.cat([torch.from_numpy(m.P).reshape(-1) for m in molecules]).to(gpu)
    v = torch.cat([torch.from_numpy(m.v) for m in molecules]).to(gpu)
    n, sums = gg.update_density(P, v)
    H, S = gg.integrate_h(v, want_S=True)
    torch.cuda.synchronize()
    Hb, Sb = gg.blocks(H), gg.blocks(S)
    pt = 0
    for k, m in enumerate(molecules):
        g1 = AimsGrid(m, device=gpu.index)
        n1, s1, H1, S1 = _step(g1, torch.from_numpy(m.P).to(gpu).reshape(-1),
                               torch.from_numpy(m.v).to(gpu))
        assert relerr(n[pt:pt + m.n_points].cpu().numpy(), n1) <= 1e-12, k
        assert np.max(np.abs(sums[k].cpu().numpy() - s1[0]) / np.abs(s1[0])) <= 1e-12, k
        assert relerr(Hb[k].cpu().numpy().reshape(-1), H1) <= 1e-12, k
        assert relerr(Sb[k].cpu().numpy().reshape(-1), S1) <= 1e-12, k
        pt += m.n_points
    # one molecule against the oracle
    m = molecules[-1]
    o = GridOracle(m)
    d = o.density(m.P, m.v)
    Hr, _ = o.integrate_h(m.v, want_S=False)
    assert relerr(Hb[-1].cpu().numpy(), Hr) <= 1e-10
    assert abs(sums[-1, 0].item() - d["N"]) <= 1e-10 * abs(d["N"])


def test_autotune_live(gpu, cluster, tmp_path):
    g = AimsGrid(cluster, device=gpu.index)
    P = torch.from_numpy(cluster.P).to(gpu).reshape(-1)
    v = torch.from_numpy(cluster.v).to(gpu)
    ref = _step(g, P, v)
    cache = str(tmp_path / "tuning.json")
    r = autotune(g, P, v, prec="fp64", reps=1, cache=cache)
    print("[autotune]", {k: r[k] for k in ("h_merge", "h_flops_per_atomic", "density_pblocks",
                                           "persistent", "key")},
          flush=True)
    # 24 global candidates, then the per-bucket refinement (its timings are labelled by bucket)
    glob = [k for k in r["ms"] if "bucket" not in k and "base" not in k]
    assert r["source"] == "measured" and len(glob) == 24
    t = g.get_tuning("fp64")
    assert t == {k: r[k] for k in ("h_merge", "density_pblocks", "persistent", "h_flops_per_atomic",
                                   "h_tile32_mask", "density_bucket_pblocks")}
    out = _step(g, P, v)
    # a different h_merge changes the H batches (same sums up to rounding)
    assert relerr(out[0], ref[0]) <= 1e-12 and relerr(out[2], ref[2]) <= 1e-12
    g2 = AimsGrid(cluster, device=gpu.index)
    r2 = autotune(g2, P, v, prec="fp64", cache=cache)
    assert r2["source"] == "cache" and r2["key"] == r["key"]
    assert g2.get_tuning("fp64") == t


def test_debug_table_checks(gpu, monkeypatch):
    """AIMS_DEBUG=1 checks every index table of every batch set and work list on the host as it
    is built (set-up, the H partitions of the tunings set below, per-bucket tile lists, the
    allocation-free set); a grouped handle and a cluster pass, and their results are unchanged."""
    monkeypatch.setenv("AIMS_DEBUG", "1")
    mols = synth.make_molecule_set(n_mol=6, seed=4, n_min=3, n_max=12)
    inst = synth.make_instance("c2", n_atoms=12, box=9.0, seed=6)
    for systems in (mols, [inst]):
        g = AimsGrid(systems, device=gpu.index)
        for t in (dict(h_merge=2), dict(h_flops_per_atomic=256, h_tile32_mask=0xffff),
                  dict(density_bucket_pblocks=[5, 4, 3, 2, 5, 4, 3, 2])):
            g.set_tuning(prec="fp64", **t)
        P = torch.cat([torch.from_numpy(m.P).reshape(-1) for m in systems]).to(gpu)
        v = torch.cat([torch.from_numpy(m.v) for m in systems]).to(gpu)
        n, sums = g.update_density(P, v)
        H, _ = g.integrate_h(v)
        torch.cuda.synchronize()
        k = len(systems) - 1
        o = GridOracle(systems[k])
        Hr, _ = o.integrate_h(systems[k].v, want_S=False)
        assert relerr(g.blocks(H)[k].cpu().numpy(), Hr) <= 1e-10


def test_debug_refuses_an_asymmetric_P(gpu, monkeypatch):
    """With AIMS_DEBUG=1 every call that reads P checks on the device that it is symmetric and
    finite, per system of a grouped handle: a symmetric P passes with unchanged results, one
    asymmetric entry in the second system, or one NaN, is refused with AIMS_ERR_ARG by the
    density pass, the backward and the density gradient alike."""
    from paper_2208_12335_amd import AimsError
    monkeypatch.setenv("AIMS_DEBUG", "1")
    mols = synth.make_molecule_set(n_mol=2, seed=9, n_min=2, n_max=4)
    g = AimsGrid(mols, device=gpu.index)
    P = torch.cat([torch.from_numpy(m.P).reshape(-1) for m in mols]).to(gpu)
    v = torch.cat([torch.from_numpy(m.v) for m in mols]).to(gpu)
    gE = torch.ones(1, dtype=torch.float64, device=gpu)
    n, sums = g.update_density(P, v)
    torch.cuda.synchronize()
    monkeypatch.delenv("AIMS_DEBUG")
    g0 = AimsGrid(mols, device=gpu.index)
    n0, sums0 = g0.update_density(P, v)
    assert relerr(sums.cpu().numpy(), sums0.cpu().numpy()) <= 1e-13
    nb1 = g.nb_sys[1]
    off = g.nb_sys[0] ** 2
    bad = P.clone()
    bad[off + 1] += 1e-6 * bad[off:].abs().max()      # entry (0, 1) of system 1 only
    nan = P.clone()
    nan[off + nb1 + 1] = float("nan")                  # entry (1, 1) of system 1
    for Q in (bad, nan):
        for call in (lambda: g.update_density(Q, v), lambda: g.backward(Q, v, gE),
                     lambda: g.density_gradient(Q)):
            with pytest.raises(AimsError) as e:
                call()
            assert "not symmetric" in str(e.value) and "system 1" in str(e.value)
    g.update_density(P, v)                             # the handle still works
