"""Instance construction for the five workload families of the NAO grid-integration core.

Units are bohr and hartree.  Every random quantity is drawn from one
``numpy.random.default_rng(seed)`` stream in a fixed order (geometry, then radial exponents,
then the density matrix), and instances can be saved to ``.npz`` so that parity never depends
on RNG details.

Workload families (sizes are for seed 0):

* ``c1``  bent triatomic O/H/H, l<=2 basis (14 + 5 + 5 = 24 functions), 50 radial shells x
  110-point angular grid, batches of <= 200 points.
* ``c2``  64-atom random cluster (Z in {1,6,8}, box 20 bohr, separation >= 1.8 bohr), l<=3 basis
  (30 functions per heavy atom, 5 per H), 75 shells x 302 angular points, batches <= 256.
* ``c3``  512-atom water-like cluster (170 H2O + OH) at 1 g/cm^3, c2 basis/grid rules,
  batches <= 300.
* ``c4``  a set of independent grown molecules of 3..40 atoms (Z in {1,6,7,8}), c1 rules.
* ``c5``  128-atom random cluster, c2 basis/grid rules, box 20 * 2^(1/3) bohr.

Radial functions are R(r) = r^l exp(-zeta r) (1 - (r/rc)^2)^3 for r < rc (0 beyond) with one
zeta per (element, shell) drawn log-uniformly in [0.3, 8].  The kinetic radial function
K = -1/2 [R'' + 2R'/r - l(l+1)R/r^2] is tabulated analytically next to R so that
t phi = -1/2 Laplacian(phi) = K(r) Y_lm.
"""
from __future__ import annotations

import dataclasses
import json
import math
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

# --------------------------------------------------------------------------------------------
# constants of the workload families
# --------------------------------------------------------------------------------------------
RC = 9.45            # radial cutoff (bohr)
R0 = 1.0e-4          # first knot of the logarithmic radial grid
N_LOG = 200          # knots of the logarithmic radial grid
ZETA_MIN, ZETA_MAX = 0.3, 8.0
PRUNE_MARGIN = 0.01  # points farther than rc + margin from every atom are dropped
STRATMANN_A = 0.64
NUCLEAR_SIGMA = 0.3  # width of the smeared nuclear potential -Z erf(r/sigma)/r
BECKE_RM = 1.0       # radial map scale of the Becke grid, same for every element
OH_BOND = 1.81
HOH_ANGLE_DEG = 104.5

# shells (angular momenta) per species class; functions = sum(2l+1)
BASIS_RULES = {
    "c1": {"heavy": [0, 0, 0, 1, 1, 2], "light": [0, 0, 1]},            # 3s2p1d / 2s1p
    "c2": {"heavy": [0, 0, 0, 0, 1, 1, 1, 2, 2, 3], "light": [0, 0, 1]},  # 4s3p2d1f / 2s1p
}
GRID_RULES = {
    "c1": {"n_radial": 50, "angular": "gl110"},
    "c2": {"n_radial": 75, "angular": "lobatto302"},
}


_DEVICE = [None]


class generator_device:
    """Context manager choosing the torch device of the generator's bulk arithmetic (distance
    tables, partition weights, potential): ``with generator_device("cuda"): ...``.  The
    default is the CPU.  The instance definition does not depend on the device; values agree
    to floating-point rounding."""

    def __init__(self, device):
        self.device = device

    def __enter__(self):
        self.prev = _DEVICE[0]
        _DEVICE[0] = self.device
        return self

    def __exit__(self, *exc):
        _DEVICE[0] = self.prev
        return False


def _torch_device():
    import torch
    return torch.device(_DEVICE[0]) if _DEVICE[0] is not None else torch.device("cpu")


def _dist(X, A):
    """Distance table |X_i - A_j| (torch, on X's device)."""
    import torch
    if X.device.type == "cpu":
        return torch.cdist(X, A, compute_mode='donot_use_mm_for_euclid_dist')
    d = X[:, None, :] - A[None, :, :]
    return torch.sqrt((d * d).sum(-1))


@dataclasses.dataclass
class Instance:
    """One molecular system with its integration grid, potential and density matrix."""

    name: str
    atom_xyz: np.ndarray          # [na, 3] float64
    atom_Z: np.ndarray            # [na] int32
    atom_species: np.ndarray      # [na] int32 -> index into species_*
    species_Z: np.ndarray         # [ns] int32
    species_nshell: np.ndarray    # [ns] int32
    shell_l: np.ndarray           # [sum nshell] int32, species-major
    shell_zeta: np.ndarray        # [sum nshell] float64 (nan for custom radial functions)
    n_log: int
    r0: float
    rc: float
    shell_R: np.ndarray           # [sum nshell, n_log] float64, R at the knots
    shell_K: np.ndarray           # [sum nshell, n_log] float64, K at the knots
    pt_xyz: np.ndarray            # [n_pts, 3] float64
    pt_w: np.ndarray              # [n_pts] float64, full quadrature weight
    pt_atom: np.ndarray           # [n_pts] int32, atom whose grid produced the point
    v: np.ndarray                 # [n_pts] float64
    P: np.ndarray                 # [nb, nb] float64, symmetric
    max_batch: int
    meta: dict = dataclasses.field(default_factory=dict)
    pt_wgrid: Optional[np.ndarray] = None   # [n_pts] radial x angular weight (before partition)

    # ---- derived basis layout -------------------------------------------------------------
    @property
    def n_atoms(self) -> int:
        return int(self.atom_xyz.shape[0])

    @property
    def n_points(self) -> int:
        return int(self.pt_xyz.shape[0])

    def species_shell_offset(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.species_nshell)]).astype(np.int64)

    def species_nfn(self) -> np.ndarray:
        off = self.species_shell_offset()
        return np.array([int(sum(2 * self.shell_l[k] + 1 for k in range(off[s], off[s + 1])))
                         for s in range(len(self.species_nshell))], dtype=np.int64)

    def atom_basis_offset(self) -> np.ndarray:
        """Offset of each atom's first function in the global basis (atom-major order)."""
        nfn = self.species_nfn()[self.atom_species]
        return np.concatenate([[0], np.cumsum(nfn)]).astype(np.int64)

    @property
    def n_basis(self) -> int:
        return int(self.atom_basis_offset()[-1])

    def basis_table(self) -> np.ndarray:
        """[nb, 4] int64 rows (atom, global shell index, l, m) in the contract's basis order:
        atom-major, then the species' shells in order, then m = -l..l."""
        off = self.species_shell_offset()
        rows = []
        for a in range(self.n_atoms):
            s = int(self.atom_species[a])
            for k in range(off[s], off[s + 1]):
                l = int(self.shell_l[k])
                for m in range(-l, l + 1):
                    rows.append((a, k, l, m))
        return np.array(rows, dtype=np.int64).reshape(-1, 4)

    # ---- persistence ----------------------------------------------------------------------
    def save(self, path: str) -> None:
        arrays = {f.name: getattr(self, f.name) for f in dataclasses.fields(self)
                  if isinstance(getattr(self, f.name), np.ndarray)}
        scalars = {"name": self.name, "n_log": self.n_log, "r0": self.r0, "rc": self.rc,
                   "max_batch": self.max_batch, "meta": self.meta}
        np.savez(path, _scalars=np.array(json.dumps(scalars)), **arrays)

    @staticmethod
    def load(path: str) -> "Instance":
        with np.load(path, allow_pickle=False) as z:
            sc = json.loads(str(z["_scalars"]))
            kw = {k: z[k] for k in z.files if k != "_scalars"}
        return Instance(name=sc["name"], n_log=int(sc["n_log"]), r0=float(sc["r0"]),
                        rc=float(sc["rc"]), max_batch=int(sc["max_batch"]), meta=sc["meta"],
                        **kw)

    def with_P(self, P: np.ndarray) -> "Instance":
        return dataclasses.replace(self, P=np.ascontiguousarray(P, dtype=np.float64))

    def with_v(self, v: np.ndarray) -> "Instance":
        return dataclasses.replace(self, v=np.ascontiguousarray(v, dtype=np.float64))

    def moved(self, atom_xyz: np.ndarray) -> "Instance":
        """Same grid, weights, potential and P; basis centres moved (Pulay convention)."""
        return dataclasses.replace(self, atom_xyz=np.ascontiguousarray(atom_xyz, np.float64))

    def translated(self, shift: Sequence[float]) -> "Instance":
        s = np.asarray(shift, dtype=np.float64)
        return dataclasses.replace(self, atom_xyz=self.atom_xyz + s, pt_xyz=self.pt_xyz + s)


# --------------------------------------------------------------------------------------------
# quadrature rules
# --------------------------------------------------------------------------------------------
def becke_radial(n: int, rm: float = BECKE_RM):
    """Becke's radial map r = rm (1+x)/(1-x) on Gauss-Chebyshev nodes of the second kind,
    x_i = cos(i pi/(n+1)), i = 1..n.  Returns (r, w) with sum w f(r) ~ int_0^inf f(r) r^2 dr."""
    i = np.arange(1, n + 1, dtype=np.float64)
    theta = i * np.pi / (n + 1)
    x = np.cos(theta)
    r = rm * (1.0 + x) / (1.0 - x)
    w = np.pi / (n + 1) * np.sin(theta) * 2.0 * rm / (1.0 - x) ** 2 * r ** 2
    return r, w


def _directions(cos_t: np.ndarray, n_phi: int):
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t ** 2))
    ph = 2.0 * np.pi * np.arange(n_phi) / n_phi
    u = np.stack([np.outer(sin_t, np.cos(ph)), np.outer(sin_t, np.sin(ph)),
                  np.outer(cos_t, np.ones(n_phi))], axis=-1)
    return u.reshape(-1, 3)


def angular_gauss_legendre(n_theta: int = 10, n_phi: int = 11):
    """Product rule: Gauss-Legendre in cos(theta) x uniform azimuth.  10 x 11 = 110 points,
    exact for spherical polynomials up to degree 10.  Weights sum to 4 pi."""
    x, wx = np.polynomial.legendre.leggauss(n_theta)
    u = _directions(x, n_phi)
    w = np.repeat(wx, n_phi) * (2.0 * np.pi / n_phi)
    return u, w


def angular_lobatto(n_theta: int = 14, n_phi: int = 25):
    """Product rule: Gauss-Lobatto in cos(theta) (poles included and collapsed to one point
    each) x uniform azimuth.  12 x 25 + 2 = 302 points, exact up to degree 24."""
    n = n_theta
    pn1 = np.polynomial.legendre.Legendre.basis(n - 1)
    interior = np.sort(pn1.deriv().roots().real)
    x = np.concatenate([[-1.0], interior, [1.0]])
    wx = 2.0 / (n * (n - 1) * pn1(x) ** 2)
    u_int = _directions(x[1:-1], n_phi)
    w_int = np.repeat(wx[1:-1], n_phi) * (2.0 * np.pi / n_phi)
    u = np.concatenate([np.array([[0.0, 0.0, -1.0]]), u_int, np.array([[0.0, 0.0, 1.0]])])
    w = np.concatenate([[wx[0] * 2.0 * np.pi], w_int, [wx[-1] * 2.0 * np.pi]])
    return u, w


ANGULAR = {"gl110": angular_gauss_legendre, "lobatto302": angular_lobatto}


def stratmann_partition(points: np.ndarray, owner: np.ndarray, atoms: np.ndarray,
                        max_neighbors: int = 64, chunk: int = 512) -> np.ndarray:
    """Stratmann-Scuseria-Frisch partition weight w_owner(p) = P_owner / sum_b P_b with
    P_b = prod_{c != b} s(mu_bc), mu_bc = (|p-R_b| - |p-R_c|)/|R_b-R_c|,
    s = (1 - g(mu/0.64))/2 and g the degree-7 switching polynomial (sign(nu) for |nu|>1).

    Exact screening: with D_min the distance to the nearest atom, every atom with
    D_b >= D_min (1+a)/(1-a) has mu_b,nearest >= a and hence P_b = 0, so only nearer atoms are
    candidates (one candidate means weight 1 for the nearest atom and 0 for the others).
    For systems with more than ``max_neighbors`` atoms the candidate set and the products are
    further limited to the ``max_neighbors`` nearest atoms (a point-dependent set, so the
    weights still sum to one at every point); with fewer atoms the formula is exact.
    Runs on the generator's torch device (see :func:`generator_device`)."""
    import torch
    dev = _torch_device()
    na = atoms.shape[0]
    npts = points.shape[0]
    out = np.zeros(npts, dtype=np.float64)
    if na == 1:
        out[:] = 1.0
        return out
    a = STRATMANN_A
    M = min(na, max_neighbors)
    dAA = np.linalg.norm(atoms[:, None, :] - atoms[None, :, :], axis=-1)
    with np.errstate(divide="ignore"):
        inv_aa = np.where(dAA > 0, 1.0 / np.where(dAA > 0, dAA, 1.0), 0.0)
    A = torch.from_numpy(np.ascontiguousarray(atoms)).to(dev)
    Dinv = torch.from_numpy(inv_aa).to(dev)
    big = 65536
    for c0 in range(0, npts, big):
        X = torch.from_numpy(np.ascontiguousarray(points[c0:c0 + big])).to(dev)
        D = _dist(X, A)
        Ds_all, order_all = torch.topk(D, M, dim=1, largest=False)
        del D
        own_all = torch.from_numpy(owner[c0:c0 + big].astype(np.int64)).to(dev)
        res = torch.zeros(X.shape[0], dtype=torch.float64, device=dev)
        ncand = (Ds_all < Ds_all[:, :1] * ((1.0 + a) / (1.0 - a))).sum(dim=1)
        one = ncand <= 1
        res[one] = (order_all[one, 0] == own_all[one]).to(torch.float64)
        k = 2
        lo = 1
        while lo < M:
            hi = min(k, M)
            sel = torch.nonzero((ncand > lo) & (ncand <= hi)).reshape(-1)
            step = max(1, chunk * 64 // hi) if dev.type == "cpu" else 65536
            for s0 in range(0, sel.numel(), step):
                idx = sel[s0:s0 + step]
                Ds = Ds_all[idx]                                       # [c, M]
                order = order_all[idx]                                 # [c, M]
                cand = order[:, :hi]                                   # [c, k]
                inv = Dinv[cand[:, :, None], order[:, None, :]]        # [c, k, M], 0 where b == c
                nu = (Ds[:, :hi, None] - Ds[:, None, :]) * inv / a
                nu.clamp_(-1.0, 1.0)
                nu2 = nu * nu
                g = nu * (35.0 + nu2 * (-35.0 + nu2 * (21.0 - 5.0 * nu2))) / 16.0
                s = 0.5 * (1.0 - g)
                same = cand[:, :, None] == order[:, None, :]
                s = torch.where(same, torch.ones_like(s), s)
                Pb = torch.prod(s, dim=2)                              # [c, k]
                Pown = torch.where(cand == own_all[idx][:, None], Pb, torch.zeros_like(Pb)).sum(dim=1)
                res[idx] = Pown / Pb.sum(dim=1)
            lo = hi
            k *= 2
        out[c0:c0 + X.shape[0]] = res.cpu().numpy()
    return out


# --------------------------------------------------------------------------------------------
# radial tables
# --------------------------------------------------------------------------------------------
def log_knots(n_log: int = N_LOG, r0: float = R0, rc: float = RC) -> np.ndarray:
    """r_k = r0 (rc/r0)^(k/(n_log-1)), k = 0..n_log-1 (last knot = rc)."""
    k = np.arange(n_log, dtype=np.float64)
    r = r0 * (rc / r0) ** (k / (n_log - 1))
    r[-1] = rc
    return r


def slater_cut_RK(l: int, zeta: float, r: np.ndarray, rc: float = RC):
    """R = r^l f, f = exp(-zeta r) (1-x)^3, x = r^2/rc^2 (0 for r >= rc), and the analytic
    kinetic radial function K = -1/2 r^l [f'' + 2 (l+1) f'/r]."""
    r = np.asarray(r, dtype=np.float64)
    inside = r < rc
    x = np.where(inside, r * r / (rc * rc), 1.0)
    one = 1.0 - x
    c = one ** 3
    c1 = -6.0 * r / rc ** 2 * one ** 2
    c2 = -6.0 / rc ** 2 * one ** 2 + 24.0 * r * r / rc ** 4 * one
    e = np.exp(-zeta * r)
    f = e * c
    f1 = e * (c1 - zeta * c)
    f2 = e * (c2 - 2.0 * zeta * c1 + zeta * zeta * c)
    rl = r ** l
    R = np.where(inside, rl * f, 0.0)
    K = np.where(inside, -0.5 * rl * (f2 + 2.0 * (l + 1) * f1 / r), 0.0)
    return R, K


def radial_tables(shell_l: Sequence[int], shell_zeta: Sequence[float], n_log: int = N_LOG,
                  r0: float = R0, rc: float = RC):
    r = log_knots(n_log, r0, rc)
    R = np.zeros((len(shell_l), n_log))
    K = np.zeros((len(shell_l), n_log))
    for k, (l, z) in enumerate(zip(shell_l, shell_zeta)):
        R[k], K[k] = slater_cut_RK(int(l), float(z), r, rc)
    return R, K


# --------------------------------------------------------------------------------------------
# geometries
# --------------------------------------------------------------------------------------------
def triatomic() -> (np.ndarray, np.ndarray):
    ang = math.radians(HOH_ANGLE_DEG)
    xyz = np.array([[0.0, 0.0, 0.0], [OH_BOND, 0.0, 0.0],
                    [OH_BOND * math.cos(ang), OH_BOND * math.sin(ang), 0.0]])
    return xyz, np.array([8, 1, 1], dtype=np.int32)


def random_cluster(rng, n: int, zset: Sequence[int], box: float, dmin: float = 1.8):
    xyz = np.zeros((0, 3))
    Z = rng.choice(np.asarray(zset), size=n).astype(np.int32)
    while xyz.shape[0] < n:
        p = rng.uniform(0.0, box, size=3)
        if xyz.shape[0] == 0 or np.min(np.linalg.norm(xyz - p, axis=1)) >= dmin:
            xyz = np.vstack([xyz, p])
    return xyz, Z


def _random_rotation(rng) -> np.ndarray:
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a*a+b*b-c*c-d*d, 2*(b*c-a*d), 2*(b*d+a*c)],
                     [2*(b*c+a*d), a*a-b*b+c*c-d*d, 2*(c*d-a*b)],
                     [2*(b*d-a*c), 2*(c*d+a*b), a*a-b*b-c*c+d*d]])


def water_cluster(rng, n_water: int = 170, with_oh: bool = True, box: float = 32.56,
                  d_oo: float = 4.8, d_inter: float = 2.5):
    ang = math.radians(HOH_ANGLE_DEG)
    h2o = np.array([[0.0, 0.0, 0.0], [OH_BOND, 0.0, 0.0],
                    [OH_BOND * math.cos(ang), OH_BOND * math.sin(ang), 0.0]])
    oh = h2o[:2]
    mols = [h2o] * n_water + ([oh] if with_oh else [])
    xyz, Z, oxy = [], [], []
    placed = np.zeros((0, 3))
    for m in mols:
        for _ in range(100000):
            o = rng.uniform(0.0, box, size=3)
            cand = (m - m[0]) @ _random_rotation(rng).T + o
            if oxy and np.min(np.linalg.norm(np.array(oxy) - o, axis=1)) < d_oo:
                continue
            if placed.shape[0] and np.min(np.linalg.norm(
                    placed[:, None, :] - cand[None, :, :], axis=-1)) < d_inter:
                continue
            break
        else:
            raise RuntimeError("water placement failed")
        oxy.append(o)
        placed = np.vstack([placed, cand])
        xyz.append(cand)
        Z += [8] + [1] * (len(m) - 1)
    return np.vstack(xyz), np.array(Z, dtype=np.int32)


def grown_molecule(rng, n: int, zset: Sequence[int] = (1, 6, 7, 8), dmin: float = 1.8,
                   dmax: float = 2.9):
    Z = rng.choice(np.asarray(zset), size=n).astype(np.int32)
    xyz = np.zeros((1, 3))
    while xyz.shape[0] < n:
        base = xyz[rng.integers(xyz.shape[0])]
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        p = base + rng.uniform(dmin, dmax) * d
        if np.min(np.linalg.norm(xyz - p, axis=1)) >= dmin - 1e-12:
            xyz = np.vstack([xyz, p])
    return xyz, Z


# --------------------------------------------------------------------------------------------
# assembly
# --------------------------------------------------------------------------------------------
def species_for(zset: Sequence[int], rule: str, rng) -> Dict[str, np.ndarray]:
    """One species per element of ``zset`` (ascending Z); one zeta per (element, shell),
    log-uniform in [0.3, 8], drawn element by element then shell by shell."""
    zs = sorted(set(int(z) for z in zset))
    nshell, ls, zetas = [], [], []
    for z in zs:
        shells = BASIS_RULES[rule]["light" if z == 1 else "heavy"]
        nshell.append(len(shells))
        ls += shells
        zetas += list(np.exp(rng.uniform(math.log(ZETA_MIN), math.log(ZETA_MAX),
                                         size=len(shells))))
    return {"species_Z": np.array(zs, dtype=np.int32),
            "species_nshell": np.array(nshell, dtype=np.int32),
            "shell_l": np.array(ls, dtype=np.int32),
            "shell_zeta": np.array(zetas, dtype=np.float64)}


def build_grid(atom_xyz: np.ndarray, n_radial: int, angular: str, rc: float = RC,
               prune: bool = True, max_neighbors: int = 64):
    """Atom-centred product grids with Stratmann partition weights; returns
    (points, weights, owner, meta, wgrid) with wgrid the radial x angular weight before the
    partition.  Points are atom-major, shell-major, angle-minor."""
    r, wr = becke_radial(n_radial)
    u, wa = ANGULAR[angular]()
    na = atom_xyz.shape[0]
    rel = (r[:, None, None] * u[None, :, :]).reshape(-1, 3)
    wraw = (wr[:, None] * wa[None, :]).reshape(-1)
    pts = (atom_xyz[:, None, :] + rel[None, :, :]).reshape(-1, 3)
    w0 = np.tile(wraw, na)
    owner = np.repeat(np.arange(na, dtype=np.int32), rel.shape[0])
    n_raw = pts.shape[0]
    keep = np.ones(n_raw, dtype=bool)
    if prune:
        # distance screening first (cheap), then the partition weights of the survivors
        keep &= _min_distance(pts, atom_xyz) <= rc + PRUNE_MARGIN
    wpart = np.zeros(n_raw)
    sel = np.nonzero(keep)[0]
    wpart[sel] = stratmann_partition(pts[sel], owner[sel], atom_xyz, max_neighbors)
    w = w0 * wpart
    n_far = int(n_raw - keep.sum())
    if prune:
        zero = keep & (w == 0.0)
        keep &= w != 0.0
    meta = {"n_raw": int(n_raw), "n_beyond_rc": n_far,
            "n_zero_weight": int(zero.sum()) if prune else 0, "n_kept": int(keep.sum())}
    return pts[keep], w[keep], owner[keep], meta, w0[keep]


def _min_distance(points: np.ndarray, atom_xyz: np.ndarray) -> np.ndarray:
    import torch
    dev = _torch_device()
    A = torch.from_numpy(np.ascontiguousarray(atom_xyz)).to(dev)
    out = np.empty(points.shape[0])
    for s0 in range(0, points.shape[0], 65536):
        X = torch.from_numpy(np.ascontiguousarray(points[s0:s0 + 65536])).to(dev)
        out[s0:s0 + 65536] = _dist(X, A).min(1).values.cpu().numpy()
    return out


def nuclear_potential(points: np.ndarray, atom_xyz: np.ndarray, Z: np.ndarray,
                      sigma: float = NUCLEAR_SIGMA) -> np.ndarray:
    """v(p) = sum_a -Z_a erf(r/sigma)/r, with the r -> 0 limit -Z 2/(sigma sqrt(pi))."""
    import torch
    dev = _torch_device()
    A = torch.from_numpy(np.ascontiguousarray(atom_xyz)).to(dev)
    Zt = torch.from_numpy(np.asarray(Z, dtype=np.float64)).to(dev)
    v = np.empty(points.shape[0])
    lim = 2.0 / (sigma * math.sqrt(math.pi))
    for s0 in range(0, points.shape[0], 65536):
        X = torch.from_numpy(np.ascontiguousarray(points[s0:s0 + 65536])).to(dev)
        r = _dist(X, A)
        small = r < 1e-12
        rs = torch.where(small, torch.ones_like(r), r)
        t = torch.where(small, torch.full_like(r, lim), torch.erf(rs / sigma) / rs)
        v[s0:s0 + 65536] = -(t * Zt).sum(1).cpu().numpy()
    return v


def random_density_matrix(rng, atom_xyz: np.ndarray, atom_nfn: np.ndarray,
                          pair_cutoff: Optional[float] = None) -> np.ndarray:
    """P_ij = P_ji = g exp(-d_ab/2), g ~ N(0,1) drawn for i <= j, d_ab the distance of the
    host atoms; atom-pair blocks with d_ab > pair_cutoff are zero."""
    off = np.concatenate([[0], np.cumsum(atom_nfn)]).astype(np.int64)
    nb = int(off[-1])
    host = np.repeat(np.arange(atom_xyz.shape[0]), atom_nfn)
    d = np.linalg.norm(atom_xyz[host][:, None, :] - atom_xyz[host][None, :, :], axis=-1)
    g = rng.standard_normal((nb, nb))
    g = np.triu(g) + np.triu(g, 1).T
    P = g * np.exp(-d / 2.0)
    if pair_cutoff is not None:
        P[d > pair_cutoff] = 0.0
    return np.ascontiguousarray(P)


EXACT_PARTITION_ATOMS = 128   # up to this many atoms the partition products run over all atoms


def _assemble(name, rng, atom_xyz, atom_Z, zset, rule, max_batch, pair_cutoff=None,
              max_neighbors=None):
    if max_neighbors is None:
        n = atom_xyz.shape[0]
        max_neighbors = n if n <= EXACT_PARTITION_ATOMS else 64
    sp = species_for(zset, rule, rng)
    zidx = {int(z): i for i, z in enumerate(sp["species_Z"])}
    atom_species = np.array([zidx[int(z)] for z in atom_Z], dtype=np.int32)
    R, K = radial_tables(sp["shell_l"], sp["shell_zeta"])
    g = GRID_RULES[rule]
    pts, w, owner, meta, wgrid = build_grid(atom_xyz, g["n_radial"], g["angular"],
                                            max_neighbors=max_neighbors)
    v = nuclear_potential(pts, atom_xyz, atom_Z)
    inst = Instance(name=name, atom_xyz=np.ascontiguousarray(atom_xyz, np.float64),
                    atom_Z=atom_Z.astype(np.int32), atom_species=atom_species,
                    species_Z=sp["species_Z"], species_nshell=sp["species_nshell"],
                    shell_l=sp["shell_l"], shell_zeta=sp["shell_zeta"], n_log=N_LOG, r0=R0,
                    rc=RC, shell_R=R, shell_K=K, pt_xyz=np.ascontiguousarray(pts),
                    pt_w=np.ascontiguousarray(w), pt_atom=owner.astype(np.int32), v=v,
                    P=np.zeros((0, 0)), max_batch=int(max_batch), meta=dict(meta),
                    pt_wgrid=np.ascontiguousarray(wgrid))
    nfn = inst.species_nfn()[atom_species]
    inst.P = random_density_matrix(rng, atom_xyz, nfn, pair_cutoff)
    inst.meta.update({"rule": rule, "grid": g, "pair_cutoff": pair_cutoff, "n_radial": g["n_radial"],
                      "r_map": BECKE_RM})
    return inst


def regrid(inst: Instance, atom_xyz: np.ndarray) -> Instance:
    """The same system (species, radial tables, density matrix, batch size) with every atom at
    ``atom_xyz`` and its grid built afresh there: atom-centred grids moved with their atoms,
    partition weights and the nuclear potential recomputed.  Used to take finite differences
    of quantities whose grid moves with the atoms."""
    atom_xyz = np.ascontiguousarray(atom_xyz, dtype=np.float64)
    g = inst.meta["grid"]
    n = atom_xyz.shape[0]
    pts, w, owner, meta, wgrid = build_grid(atom_xyz, g["n_radial"], g["angular"], rc=inst.rc,
                                            max_neighbors=n if n <= EXACT_PARTITION_ATOMS else 64)
    v = nuclear_potential(pts, atom_xyz, inst.atom_Z)
    return dataclasses.replace(inst, atom_xyz=atom_xyz, pt_xyz=np.ascontiguousarray(pts),
                               pt_w=np.ascontiguousarray(w), pt_atom=owner.astype(np.int32),
                               v=v, pt_wgrid=np.ascontiguousarray(wgrid),
                               meta=dict(inst.meta, **meta))


CONFIGS = ("c1", "c2", "c3", "c4", "c5")


def make_instance(config: str, seed: int = 0, n_atoms: Optional[int] = None,
                  box: Optional[float] = None) -> Instance:
    """Build one seeded instance of a workload family (``c1``, ``c2``, ``c3``, ``c5``; ``c4``
    is a set, see :func:`make_molecule_set`).  ``n_atoms``/``box`` shrink the random clusters
    for quick tests (the construction rules stay the same)."""
    rng = np.random.default_rng(seed)
    if config == "c1":
        xyz, Z = triatomic()
        return _assemble("c1", rng, xyz, Z, (1, 8), "c1", 200)
    if config == "c2":
        n = 64 if n_atoms is None else n_atoms
        b = 20.0 if box is None else box
        xyz, Z = random_cluster(rng, n, (1, 6, 8), b)
        return _assemble(f"c2_n{n}", rng, xyz, Z, (1, 6, 8), "c2", 256, pair_cutoff=2 * RC)
    if config == "c3":
        xyz, Z = water_cluster(rng)
        return _assemble("c3", rng, xyz, Z, (1, 8), "c2", 300, pair_cutoff=2 * RC)
    if config == "c5":
        n = 128 if n_atoms is None else n_atoms
        b = 20.0 * 2.0 ** (1.0 / 3.0) if box is None else box
        xyz, Z = random_cluster(rng, n, (1, 6, 8), b)
        return _assemble(f"c5_n{n}", rng, xyz, Z, (1, 6, 8), "c2", 256, pair_cutoff=2 * RC)
    raise ValueError(f"unknown config {config!r}")


def make_molecule_set(n_mol: int = 256, seed: int = 0, n_min: int = 3,
                      n_max: int = 40) -> List[Instance]:
    """Independent grown molecules (sizes uniform in [n_min, n_max]); every molecule uses the
    same species defaults (one zeta per element and shell), c1 basis/grid rules, batches
    of <= 200 points."""
    rng = np.random.default_rng(seed)
    zset = (1, 6, 7, 8)
    sizes = rng.integers(n_min, n_max + 1, size=n_mol)
    out = []
    for k, n in enumerate(sizes):
        xyz, Z = grown_molecule(rng, int(n), zset)
        mol_rng = np.random.default_rng([seed, 2, k])
        # species defaults are shared: draw them from the same stream for every molecule
        inst = _assemble(f"c4_m{k}", np.random.default_rng([seed, 1]), xyz, Z, zset, "c1", 200)
        inst.P = random_density_matrix(mol_rng, xyz, inst.species_nfn()[inst.atom_species])
        out.append(inst)
    return out


def custom_instance(atom_xyz: np.ndarray, atom_species: np.ndarray,
                    species_shells: List[List[int]],
                    radial: List[Callable[[np.ndarray], tuple]], *, n_log: int = N_LOG,
                    r0: float = R0, rc: float = RC, n_radial: int = 50,
                    angular: str = "gl110", potential: Optional[Callable] = None,
                    P: Optional[np.ndarray] = None, max_batch: int = 200,
                    prune: bool = True, rm: float = BECKE_RM, name: str = "custom",
                    atom_Z: Optional[np.ndarray] = None) -> Instance:
    """Instance with caller-chosen radial functions (one ``f(r) -> (R, K)`` per shell, shells
    concatenated species-major), used for closed-form test cases (Gaussian and hydrogenic
    radial functions)."""
    atom_xyz = np.ascontiguousarray(atom_xyz, dtype=np.float64)
    atom_species = np.asarray(atom_species, dtype=np.int32)
    shell_l = np.array([l for sh in species_shells for l in sh], dtype=np.int32)
    rk = log_knots(n_log, r0, rc)
    R = np.zeros((len(shell_l), n_log))
    K = np.zeros((len(shell_l), n_log))
    for k, f in enumerate(radial):
        R[k], K[k] = f(rk)
    r, wr = becke_radial(n_radial, rm)
    u, wa = ANGULAR[angular]()
    na = atom_xyz.shape[0]
    rel = (r[:, None, None] * u[None, :, :]).reshape(-1, 3)
    pts = (atom_xyz[:, None, :] + rel[None, :, :]).reshape(-1, 3)
    w0 = np.tile((wr[:, None] * wa[None, :]).reshape(-1), na)
    owner = np.repeat(np.arange(na, dtype=np.int32), rel.shape[0])
    w = w0 * stratmann_partition(pts, owner, atom_xyz, max_neighbors=max(64, na))
    keep = np.ones(pts.shape[0], dtype=bool)
    if prune:
        d = np.min(np.linalg.norm(pts[:, None, :] - atom_xyz[None], axis=-1), axis=1)
        keep = (w != 0.0) & (d <= rc + PRUNE_MARGIN)
    pts, w, owner, w0 = pts[keep], w[keep], owner[keep], w0[keep]
    nsp = len(species_shells)
    inst = Instance(name=name, atom_xyz=atom_xyz,
                    atom_Z=(np.ones(na, np.int32) if atom_Z is None else np.asarray(atom_Z, np.int32)),
                    atom_species=atom_species, species_Z=np.arange(nsp, dtype=np.int32),
                    species_nshell=np.array([len(s) for s in species_shells], dtype=np.int32),
                    shell_l=shell_l, shell_zeta=np.full(len(shell_l), np.nan), n_log=n_log,
                    r0=r0, rc=rc, shell_R=R, shell_K=K, pt_xyz=np.ascontiguousarray(pts),
                    pt_w=np.ascontiguousarray(w), pt_atom=owner.astype(np.int32),
                    v=np.zeros(pts.shape[0]), P=np.zeros((0, 0)), max_batch=max_batch,
                    meta={"custom": True, "n_radial": int(n_radial), "r_map": float(rm)},
                    pt_wgrid=np.ascontiguousarray(w0))
    if potential is not None:
        inst.v = np.ascontiguousarray(potential(pts), dtype=np.float64)
    nb = inst.n_basis
    inst.P = np.zeros((nb, nb)) if P is None else np.ascontiguousarray(P, dtype=np.float64)
    return inst


def radial_shells(inst: Instance):
    """(pt_shell [n_pts] int32, n_radial, r_map): the index of each point's radial node on its
    owner's Becke radial grid (nodes as ``becke_radial`` orders them), found from the point's
    distance to its owner."""
    n_radial = int(inst.meta["n_radial"])
    rm = float(inst.meta.get("r_map", BECKE_RM))
    r_nodes, _ = becke_radial(n_radial, rm)
    d = np.linalg.norm(inst.pt_xyz - inst.atom_xyz[inst.pt_atom], axis=1)
    order = np.argsort(r_nodes)
    rs = r_nodes[order]
    j = np.clip(np.searchsorted(rs, d), 1, n_radial - 1)
    j = np.where(np.abs(rs[j - 1] - d) < np.abs(rs[j] - d), j - 1, j)
    k = order[j]
    if np.any(np.abs(r_nodes[k] - d) > 1e-9 * np.maximum(1.0, r_nodes[k])):
        raise ValueError("points off the radial nodes")
    return k.astype(np.int32), n_radial, rm
