"""The C-ABI library loads and exports every symbol the header declares; argument validation
happens on the host before any device work (these calls never reach a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "aims_grid.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(aims_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2208_12335_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2208_12335_amd.build import build
        build()
    return _lib.load()


def test_header_symbols_exported(lib):
    from paper_2208_12335_amd._lib import SIGNATURES
    names = _declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
        assert n in SIGNATURES, n


def _system(c1, **over):
    from paper_2208_12335_amd._lib import AimsSystem
    keep = {}
    def arr(name, dt, v):
        keep[name] = np.ascontiguousarray(v, dtype=dt)
        return keep[name].ctypes.data_as(ctypes.POINTER(ctypes.c_double if dt == np.float64 else ctypes.c_int32))
    s = AimsSystem()
    s.n_atoms = c1.n_atoms
    s.atom_xyz = arr("xyz", np.float64, c1.atom_xyz)
    s.atom_species = arr("sp", np.int32, c1.atom_species)
    s.n_species = len(c1.species_nshell)
    s.species_nshell = arr("ns", np.int32, c1.species_nshell)
    s.shell_l = arr("l", np.int32, over.pop("shell_l", c1.shell_l))
    s.n_log = over.pop("n_log", c1.n_log)
    s.r0, s.rc = over.pop("r0", c1.r0), c1.rc
    s.shell_R = arr("R", np.float64, c1.shell_R)
    s.shell_K = arr("K", np.float64, c1.shell_K)
    s.n_points = c1.n_points
    s.pt_xyz = arr("p", np.float64, c1.pt_xyz)
    s.pt_w = arr("w", np.float64, c1.pt_w)
    s.max_batch = over.pop("max_batch", c1.max_batch)
    s.screen_margin = 0.01
    return s, keep


@pytest.mark.parametrize("over,status", [
    ({"shell_l": None}, -5),          # l = 4 -> unsupported
    ({"n_log": 3}, -1),
    ({"r0": 20.0}, -1),               # r0 >= rc
    ({"max_batch": 0}, -5),
    ({"max_batch": 100000}, -5),
])
def test_setup_validation_errors(lib, c1, over, status):
    if "shell_l" in over:
        l = np.array(c1.shell_l)
        l[0] = 4
        over = {"shell_l": l}
    s, keep = _system(c1, **over)
    h = ctypes.c_void_p()
    st = lib.aims_grid_setup(ctypes.byref(s), 0, None, ctypes.byref(h))
    assert st == status
    assert h.value is None
    msg = lib.aims_last_error(None).decode()
    assert len(msg) > 5 and msg != "no error"


def test_null_arguments(lib, c1):
    h = ctypes.c_void_p()
    assert lib.aims_grid_setup(None, 0, None, ctypes.byref(h)) == -1
    assert lib.aims_grid_setup_many(None, 0, 0, None, ctypes.byref(h)) == -1
    assert lib.aims_update_density(None, 0, None, None, None, None, None) == -1
    assert lib.aims_integrate_h(None, 0, None, None, None, None) == -1
    assert lib.aims_work_stats(None, None, None, None) == -1
    assert lib.aims_n_basis(None) == -1
    assert lib.aims_step_graph_launch(None) == -1
    assert lib.aims_grid_set_moving(None, 0, None) == -1
    assert lib.aims_total_forces(None, 0, None, None, None, None) == -1
    assert lib.aims_density_matrix(None, 0, None, None, None, 0.0, None, None, None) == -1
    assert lib.aims_last_purify_products(None) == 0
    assert lib.aims_xc(None, 0, None, None, None) == -1
    assert lib.aims_density_gradient(None, None, None, None) == -1
    assert lib.aims_integrate_h_gga(None, 0, None, None, None) == -1
    assert lib.aims_xc_gga(None, 1, None, None, None, None, None) == -1
    assert lib.aims_grid_set_hartree(None, 0, None) == -1
    assert lib.aims_hartree(None, None, None, None) == -1
    lib.aims_grid_destroy(None)
    lib.aims_step_graph_destroy(None)


def test_basis_count_limit(lib):
    """A system with more than 65535 basis functions is refused at set-up (the tiled kernels
    address P with 32-bit offsets): 293 atoms of a species with 32 f shells, 224 functions
    each, make 65,632."""
    from paper_2208_12335_amd._lib import AimsSystem
    n_atoms, nsh, n_log = 293, 32, 8
    keep = {
        "xyz": np.arange(3 * n_atoms, dtype=np.float64) * 3.0,
        "sp": np.zeros(n_atoms, dtype=np.int32),
        "ns": np.array([nsh], dtype=np.int32),
        "l": np.full(nsh, 3, dtype=np.int32),
        "R": np.zeros(nsh * n_log), "K": np.zeros(nsh * n_log),
    }
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    s = AimsSystem()
    s.n_atoms, s.n_species, s.n_log, s.r0, s.rc = n_atoms, 1, n_log, 1e-4, 9.45
    s.atom_xyz, s.atom_species, s.species_nshell = dp(keep["xyz"]), ip(keep["sp"]), ip(keep["ns"])
    s.shell_l, s.shell_R, s.shell_K = ip(keep["l"]), dp(keep["R"]), dp(keep["K"])
    s.n_points, s.max_batch, s.screen_margin = 0, 256, 0.01
    h = ctypes.c_void_p()
    assert lib.aims_grid_setup(ctypes.byref(s), 0, None, ctypes.byref(h)) == -5
    assert h.value is None
    assert "basis functions" in lib.aims_last_error(None).decode()


def test_binding_refuses_wrong_sizes_on_host():
    """The binding checks every caller tensor (element count, dtype, contiguity, device) before
    it reaches the C ABI, so a short buffer never becomes an out-of-bounds device access."""
    import torch
    from paper_2208_12335_amd.grid import AimsGrid
    g = object.__new__(AimsGrid)
    g.device = torch.device("cpu")
    ok = torch.zeros(12, dtype=torch.float64)
    assert g._arg(ok, 12, "x") is not None
    assert g._arg(None, 12, "x") is None
    assert g._arg(torch.zeros(13, dtype=torch.float64), 12, "gE", at_least=True) is not None
    with pytest.raises(ValueError, match="11 elements"):
        g._arg(torch.zeros(11, dtype=torch.float64), 12, "P")
    with pytest.raises(ValueError, match="13 elements"):
        g._arg(torch.zeros(13, dtype=torch.float64), 12, "H_out")
    with pytest.raises(TypeError):
        g._arg(torch.zeros(12, dtype=torch.float32), 12, "v")
    with pytest.raises(ValueError, match="contiguous"):
        g._arg(torch.zeros(12, 2, dtype=torch.float64)[:, 0], 12, "v")
    g.device = torch.device("cuda", 0)
    with pytest.raises(ValueError, match="handle is on"):
        g._arg(ok, 12, "P")


def test_valid_setup_runs_host_stages_then_needs_a_device(lib, c1):
    """A valid system passes validation, and the host stages of set-up (natural splines of
    every shell, the bisection of the points into batches) run before the first device call;
    without a GPU the call then fails cleanly (a HIP error, no handle).  Under the host
    sanitizers this exercises the host set-up code end to end."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present: set-up would succeed")
    s, keep = _system(c1)
    h = ctypes.c_void_p()
    st = lib.aims_grid_setup(ctypes.byref(s), 0, None, ctypes.byref(h))
    assert st == -3 and h.value is None
    assert len(lib.aims_last_error(None).decode()) > 5
