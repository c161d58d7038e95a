"""Mixed-precision forms against the FP64 oracle: the error of each result is measured and
stated (printed), and held to bounds that follow from the arithmetic:

* FP32: basis values, tables and per-batch accumulation in binary32 (unit roundoff 6e-8); the
  randomly signed density matrix cancels strongly inside n, so n and E carry relative errors of
  order 1e-6, H and S of order 1e-7.
* BF16x3: products of hi/lo bf16 splits keep about 16 significant bits (2^-16 ~ 1.5e-5 per
  product), so the bounds are about 100 times looser.

The total-energy target of 1e-6 Ha is reported, not asserted: these forms do not reach it on
randomly signed density matrices (see the benchmark's mixed_vs_fp64 field)."""
import numpy as np
import pytest
import torch

import synth
from oracle import GridOracle
from paper_2208_12335_amd import AimsGrid
from conftest import relerr

pytestmark = pytest.mark.gpu

BOUNDS = {"fp32": {"n": 1e-4, "H": 1e-5, "S": 1e-5, "N": 1e-5, "E": 1e-5},
          "bf16x3": {"n": 1e-2, "H": 1e-3, "S": 1e-3, "N": 1e-3, "E": 1e-3}}


@pytest.fixture(scope="module")
def cases():
    out = []
    for inst in (synth.make_instance("c1"), synth.make_instance("c2", n_atoms=24, box=11.0, seed=2)):
        o = GridOracle(inst)
        d = o.density(inst.P, inst.v)
        H, S = o.integrate_h(inst.v)
        out.append((inst, d, H, S))
    return out


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_precision_errors_stated(gpu, cases, prec):
    for inst, d, Hr, Sr in cases:
        g = AimsGrid(inst, device=gpu.index)
        P = torch.from_numpy(inst.P).to(gpu).reshape(-1)
        v = torch.from_numpy(inst.v).to(gpu)
        n, sums = g.update_density(P, v, prec=prec)
        H, S = g.integrate_h(v, prec=prec, want_S=True)
        torch.cuda.synchronize()
        nb = inst.n_basis
        s = sums.cpu().numpy()[0]
        E, Er = s[1] + s[2], d["E_V"] + d["E_T"]
        errs = {"n": relerr(n.cpu().numpy(), d["n"]),
                "H": relerr(H.cpu().numpy().reshape(nb, nb), Hr),
                "S": relerr(S.cpu().numpy().reshape(nb, nb), Sr),
                "N": abs(s[0] - d["N"]) / abs(d["N"]), "E": abs(E - Er) / abs(Er)}
        print(f"[mixed] {prec} {inst.name}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items())
              + f", |dE| = {abs(E - Er):.2e} Ha", flush=True)
        for k, e in errs.items():
            assert e < BOUNDS[prec][k], (prec, inst.name, k, e)
