"""Stored oracle values (written by tests/golden/make_golden.py, which calls only the oracle)
and the code-independence rules between the oracle and the HIP library."""
import ast
import json
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_reproduces_stored_c1_values(c1, c1_oracle):
    with open(os.path.join(ROOT, "tests", "golden", "c1_seed0_oracle.json")) as f:
        ref = json.load(f)
    assert c1.n_points == ref["n_points"] and c1.n_basis == ref["n_basis"]
    d = c1_oracle.density(c1.P, c1.v)
    for k in ("N", "E_V", "E_T"):
        assert abs(d[k] - ref[k]) < 1e-11 * max(1.0, abs(ref[k]))
    assert np.allclose(d["n"][ref["n_sample_idx"]], ref["n_sample"], rtol=1e-11, atol=1e-15)
    H, S = c1_oracle.integrate_h(c1.v)
    assert np.allclose(H[:6, :6], np.array(ref["H_block"]), rtol=1e-11, atol=1e-14)
    assert np.allclose(np.diag(S), ref["S_diag"], rtol=1e-12)


def _imports(path):
    tree = ast.parse(open(path).read())
    names = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            names.update(a.name.split(".")[0] for a in node.names)
        elif isinstance(node, ast.ImportFrom) and node.module and node.level == 0:
            names.add(node.module.split(".")[0])
    return names


def _py_files(d):
    for root, _, files in os.walk(os.path.join(ROOT, d)):
        for f in files:
            if f.endswith(".py"):
                yield os.path.join(root, f)


def test_oracle_and_library_share_no_code():
    for f in _py_files("oracle"):
        assert "paper_2208_12335_amd" not in _imports(f), f
    for f in _py_files("paper_2208_12335_amd"):
        assert "oracle" not in _imports(f), f
    # the generator holds none of the method's arithmetic and imports neither side
    for f in _py_files("synth"):
        imps = _imports(f)
        assert "oracle" not in imps and "paper_2208_12335_amd" not in imps, f
