import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


@pytest.fixture(scope="session")
def c1():
    import synth
    return synth.make_instance("c1")


@pytest.fixture(scope="session")
def c1_oracle(c1):
    from oracle import GridOracle
    return GridOracle(c1)


@pytest.fixture(scope="session")
def gpu():
    """The HIP library on cuda:0.  GPU tests fail (they do not skip) when either is missing."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2208_12335_amd import _lib
    _lib.load()
    return torch.device("cuda", 0)


def relerr(x, ref):
    """Norm-wise relative error max|x - ref| / max|ref| (0 when both are zero)."""
    import numpy as np
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref)) if ref.size else 0.0
    num = np.max(np.abs(x - ref)) if ref.size else 0.0
    return 0.0 if den == 0 and num == 0 else num / den


def pair_block(o, inst, a, b, v):
    """H and S block of atoms (a, b) by the oracle ``o``, over the points within rc of both
    (every other point contributes exactly zero to the block)."""
    import numpy as np
    d = np.linalg.norm(inst.pt_xyz[:, None, :] - inst.atom_xyz[None, [a, b], :], axis=-1)
    idx = np.nonzero((d[:, 0] < inst.rc) & (d[:, 1] < inst.rc))[0]
    Pa, Ta, ca = o.basis_values(inst.pt_xyz[idx], atoms=np.array([a]))
    Pb, Tb, cb = o.basis_values(inst.pt_xyz[idx], atoms=np.array([b]))
    w = inst.pt_w[idx][:, None]
    H = Pa.T @ (w * (v[idx][:, None] * Pb + Tb))
    S = Pa.T @ (w * Pb)
    return ca, cb, H, S
