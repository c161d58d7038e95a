"""Real spherical harmonics from the general real-solid-harmonic expansion (test oracle).

The real solid harmonic of degree l and order m is a homogeneous polynomial in (x, y, z):

    S_lm = N_lm sum_{t=0}^{(l-|m|)/2} sum_{u=0}^{t} sum_{v} C_tuv x^(2t+|m|-2(u+v)) y^(2(u+v)) z^(l-2t-|m|)
    C_tuv = (-1)^(t+v-v_m) 4^(-t) binom(l,t) binom(l-t,|m|+t) binom(t,u) binom(|m|,2v)
    N_lm  = 1/(2^|m| l!) sqrt(2 (l+|m|)! (l-|m|)! / 2^delta(m,0))

with v_m = 0 for m >= 0 and 1/2 for m < 0 (v runs over v_m, v_m + 1, ... up to
floor(|m|/2 - v_m) + v_m).  This is the standard closed form of the real solid harmonics
(Helgaker, Jorgensen and Olsen, "Molecular Electronic-Structure Theory", section 6.4); S_lm(u) on
the unit sphere equals sqrt(4 pi/(2l+1)) Y_lm(u) for the orthonormal real harmonics with no
Condon-Shortley phase, which is the contract's convention (Y_1,-1 ~ y, Y_10 ~ z, Y_11 ~ x).
The tests pin it against ``scipy.special.sph_harm_y``.

Functions take an array module ``xp`` (numpy or torch) so that the same expansion serves both
the plain numpy oracle and its autograd twin used for the atomic-position gradient.
"""
from __future__ import annotations

import math
from functools import lru_cache
from typing import Dict, List, Tuple

import numpy as np

LMAX = 3


@lru_cache(maxsize=None)
def ylm_terms(l: int, m: int) -> Tuple[Tuple[float, int, int, int], ...]:
    """Monomial expansion of the orthonormal real harmonic Y_lm as ((coef, px, py, pz), ...)."""
    am = abs(m)
    vm2 = 0 if m >= 0 else 1                      # 2 v_m
    norm = (1.0 / (2 ** am * math.factorial(l))) * math.sqrt(
        2.0 * math.factorial(l + am) * math.factorial(l - am) / (2.0 if m == 0 else 1.0))
    norm *= math.sqrt((2 * l + 1) / (4.0 * math.pi))
    acc: Dict[Tuple[int, int, int], float] = {}
    v2_max = 2 * ((am - vm2) // 2) + vm2         # 2 * (floor(|m|/2 - v_m) + v_m)
    for t in range((l - am) // 2 + 1):
        for u in range(t + 1):
            for v2 in range(vm2, v2_max + 1, 2):  # v2 = 2v
                sign = -1.0 if ((2 * t + v2 - vm2) // 2) % 2 else 1.0
                c = (sign * 0.25 ** t * math.comb(l, t) * math.comb(l - t, am + t)
                     * math.comb(t, u) * math.comb(am, v2))
                key = (2 * t + am - (2 * u + v2), 2 * u + v2, l - 2 * t - am)
                acc[key] = acc.get(key, 0.0) + norm * c
    return tuple((c, px, py, pz) for (px, py, pz), c in sorted(acc.items()) if c != 0.0)


def lm_list(lmax: int = LMAX) -> List[Tuple[int, int]]:
    return [(l, m) for l in range(lmax + 1) for m in range(-l, l + 1)]


def _powers(xp, a, n):
    out = [xp.ones_like(a)]
    for _ in range(n):
        out.append(out[-1] * a)
    return out


def real_ylm(u, lmax: int = LMAX, xp=np):
    """Y_lm(u) for unit vectors u[..., 3]; returns [..., (lmax+1)^2] ordered l-major, m=-l..l."""
    x, y, z = u[..., 0], u[..., 1], u[..., 2]
    px, py, pz = _powers(xp, x, lmax), _powers(xp, y, lmax), _powers(xp, z, lmax)
    cols = []
    for l, m in lm_list(lmax):
        val = 0.0 * x
        for c, a, b, d in ylm_terms(l, m):
            val = val + c * px[a] * py[b] * pz[d]
        cols.append(val)
    return xp.stack(cols, -1) if xp is not np else np.stack(cols, axis=-1)


def real_ylm_grad(u, lmax: int = LMAX, xp=np):
    """Cartesian gradient of the solid harmonic S_lm = sqrt(4pi/(2l+1)) Y_lm-normalised
    polynomial, evaluated on u: returns [..., (lmax+1)^2, 3] with d/dx, d/dy, d/dz of the
    homogeneous polynomial Y_lm(x, y, z) (not of Y_lm(u/|u|))."""
    x, y, z = u[..., 0], u[..., 1], u[..., 2]
    px, py, pz = _powers(xp, x, lmax), _powers(xp, y, lmax), _powers(xp, z, lmax)
    cols = []
    for l, m in lm_list(lmax):
        gx, gy, gz = 0.0 * x, 0.0 * x, 0.0 * x
        for c, a, b, d in ylm_terms(l, m):
            if a:
                gx = gx + c * a * px[a - 1] * py[b] * pz[d]
            if b:
                gy = gy + c * b * px[a] * py[b - 1] * pz[d]
            if d:
                gz = gz + c * d * px[a] * py[b] * pz[d - 1]
        cols.append(np.stack([gx, gy, gz], axis=-1))
    return np.stack(cols, axis=-2)
