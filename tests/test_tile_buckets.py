"""Tile shapes per (points, basis count) bucket against the oracle: every H bucket on 32 x 32
tiles, per-bucket point-tile caps of the density kernel, mixed masks, a grouped handle of small
molecules (basis counts below 64), and the autotuner's per-bucket choice.  The FP64 bar is the
parity bar (1e-10 norm-wise relative); the FP32 form is held to its stated bounds and compared
with its own 64 x 64 result."""
import numpy as np
import pytest
import torch

import synth
from oracle import GridOracle
from paper_2208_12335_amd import AimsGrid
from paper_2208_12335_amd.autotune import autotune
from conftest import relerr

pytestmark = pytest.mark.gpu

ALL32 = (1 << 16) - 1


@pytest.fixture(scope="module")
def cluster():
    inst = synth.make_instance("c2", n_atoms=16, box=10.0, seed=5)
    o = GridOracle(inst)
    d = o.density(inst.P, inst.v)
    H, S = o.integrate_h(inst.v)
    return inst, d, H, S


def _step(g, inst, dev, prec):
    P = torch.from_numpy(inst.P).to(dev).reshape(-1)
    v = torch.from_numpy(inst.v).to(dev)
    n, sums = g.update_density(P, v, prec=prec)
    H, S = g.integrate_h(v, prec=prec, want_S=True)
    torch.cuda.synchronize()
    return n.cpu().numpy(), sums.cpu().numpy(), H.cpu().numpy(), S.cpu().numpy()


@pytest.mark.parametrize("mask,caps", [(ALL32, [0] * 8), (0b1010101010101010, [2, 3, 4, 5, 2, 3, 4, 5]),
                                       (0, [5, 4, 3, 2, 5, 4, 3, 2])])
def test_fp64_tile_shapes_match_oracle(gpu, cluster, mask, caps):
    inst, d, Hr, Sr = cluster
    nb = inst.n_basis
    g = AimsGrid(inst, device=gpu.index)
    for persistent in (0, 1):
        g.set_tuning(prec="fp64", h_merge=0, h_flops_per_atomic=0, persistent=persistent,
                     h_tile32_mask=mask, density_bucket_pblocks=caps)
        n, sums, H, S = _step(g, inst, gpu, "fp64")
        e = {"n": relerr(n, d["n"]), "H": relerr(H.reshape(nb, nb), Hr), "S": relerr(S.reshape(nb, nb), Sr),
             "E": abs(sums[0, 1] + sums[0, 2] - d["E_V"] - d["E_T"]) / abs(d["E_V"] + d["E_T"])}
        print(f"[tiles] mask {mask:#06x} caps {caps} persistent {persistent}: "
              + ", ".join(f"{k} {x:.2e}" for k, x in e.items()), flush=True)
        assert max(e.values()) < 1e-10, e


def test_fp32_tile32_matches_its_64_tiles(gpu, cluster):
    inst, d, Hr, Sr = cluster
    nb = inst.n_basis
    g = AimsGrid(inst, device=gpu.index)
    g.set_tuning(prec="fp32", h_merge=1, h_tile32_mask=0)
    _, _, H64, S64 = _step(g, inst, gpu, "fp32")
    g.set_tuning(prec="fp32", h_merge=1, h_tile32_mask=ALL32)
    _, _, H32, S32 = _step(g, inst, gpu, "fp32")
    # the same FP32 accumulation per element; only the FP64 scatter-add order differs
    assert relerr(H32, H64) < 1e-13 and relerr(S32, S64) < 1e-13
    assert relerr(H32.reshape(nb, nb), Hr) < 1e-5


def test_grouped_small_molecules_tile32(gpu):
    """Molecules of 3-4 atoms (basis counts 15-56, all below 64): their H batches in bucket 0
    or 1; 32 x 32 tiles against the oracle per molecule."""
    mols = synth.make_molecule_set(n_mol=5, seed=3, n_min=3, n_max=4)
    g = AimsGrid(mols, device=gpu.index)
    g.set_tuning(prec="fp64", h_merge=0, h_tile32_mask=ALL32, density_bucket_pblocks=[3] * 8)
    nb_b, fl = g.bucket_stats("fp64", "h")
    assert sum(nb_b[2:]) == 0 and sum(nb_b[:2]) > 0          # every batch below 64 functions
    P = torch.cat([torch.from_numpy(m.P).reshape(-1) for m in mols]).to(gpu)
    v = torch.cat([torch.from_numpy(m.v) for m in mols]).to(gpu)
    n, sums = g.update_density(P, v)
    H, _ = g.integrate_h(v)
    torch.cuda.synchronize()
    Hs = g.blocks(H)
    off = 0
    for k, m in enumerate(mols):
        o = GridOracle(m)
        Hr, _ = o.integrate_h(m.v, want_S=False)
        dr = o.density(m.P, m.v)
        assert relerr(Hs[k].cpu().numpy(), Hr) < 1e-10
        assert relerr(n[off:off + m.n_points].cpu().numpy(), dr["n"]) < 1e-10
        off += m.n_points


def test_autotuner_picks_per_bucket_shapes(gpu, cluster):
    inst, d, Hr, Sr = cluster
    nb = inst.n_basis
    g = AimsGrid(inst, device=gpu.index)
    P = torch.from_numpy(inst.P).to(gpu).reshape(-1)
    v = torch.from_numpy(inst.v).to(gpu)
    r = autotune(g, P, v, prec="fp64", reps=1, cache="")
    t = g.get_tuning("fp64")
    print(f"[tiles] autotuned: mask {t['h_tile32_mask']:#06x}, bucket caps {t['density_bucket_pblocks']}",
          flush=True)
    assert any(k.startswith("density bucket") or k.startswith("h bucket") for k in r["ms"])
    n, sums, H, S = _step(g, inst, gpu, "fp64")
    assert relerr(n, d["n"]) < 1e-10 and relerr(H.reshape(nb, nb), Hr) < 1e-10
