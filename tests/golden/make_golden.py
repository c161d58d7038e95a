"""Writes the stored oracle values for the seeded bent-triatomic case (seed 0).

Calls only the ``synth`` generator and the FP64 ``oracle``; run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import GridOracle  # noqa: E402


def main():
    inst = synth.make_instance("c1", seed=0)
    o = GridOracle(inst)
    d = o.density(inst.P, inst.v)
    H, S = o.integrate_h(inst.v)
    g = o.gradient(inst.P, inst.v)
    sample = [0, 1234, 5000, 9876, inst.n_points - 1]
    out = {
        "case": "bent triatomic O/H/H, 24-function l<=2 basis, 50 x 110 grid, seed 0",
        "n_points": inst.n_points, "n_basis": inst.n_basis,
        "N": d["N"], "E_V": d["E_V"], "E_T": d["E_T"],
        "n_sample_idx": sample, "n_sample": [float(d["n"][i]) for i in sample],
        "H_block": H[:6, :6].tolist(), "S_diag": np.diag(S).tolist(),
        "trace_H": float(np.trace(H)), "dE_dR": g["dE_dR"].tolist(),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_seed0_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
