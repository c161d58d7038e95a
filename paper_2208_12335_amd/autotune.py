"""Autotuner of the library's execution parameters, timed on the live device.

Four knobs decide how the batched work of one s.c.f. step maps onto the GPU (the batch
integration scheme itself is fixed by the grid partition):

* ``density_pblocks`` -- the point extent (32 x pblocks) of a density work tile;
* ``h_merge``        -- how many bisection levels the H/S pass merges (bigger batches, fewer
  FP64 scatter-adds into H, more flops);
* ``h_flops_per_atomic`` -- instead of a fixed level, a cost-model partition of the H/S pass
  that charges this many flop-equivalents per scatter-add (0 = fixed level);
* ``persistent``     -- one workgroup per tile, or a resident grid pulling tiles from per-XCD
  work counters.

The density pass depends only on (pblocks, persistent) and the H pass only on its partition
(h_merge or h_flops_per_atomic) and persistent, so the tuner times the two passes separately and picks, per ``persistent`` value,
the best of each, then the better ``persistent``.

Then the tile shapes are refined per (points, basis count) bucket (``refine_buckets``): the
density batches of each basis-size bucket get their own point-tile cap
(``density_bucket_pblocks``), and each H bucket (basis-size class x whether the last 64-wide
tile row is at most half full) runs 64 x 64 or 32 x 32 tiles (``h_tile32_mask``, FP64 and
FP32).  Buckets are visited in decreasing order of their flops, one at a time, keeping a change
only when the pass gets faster by more than ``min_gain``.

Results are cached in a JSON file keyed by (device architecture, precision, workload bucket) so
later handles of a similar workload skip the measurement.
"""
from __future__ import annotations

import json
import math
import os
import tempfile
from typing import Callable, Dict, Iterable, Optional, Sequence, Tuple

DENSITY_PBLOCKS = (2, 3, 4, 5)
H_MERGE = (0, 1, 2, 3)
H_RATIO = (64, 256, 1024, 4096)
PERSISTENT = (0, 1)
KNOBS = ("h_merge", "density_pblocks", "persistent", "h_flops_per_atomic", "h_tile32_mask",
         "density_bucket_pblocks")
BASE_KNOBS = KNOBS[:4]


def default_cache_path() -> str:
    return os.environ.get("AIMS_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2208_12335_amd",
                                       "tuning.json"))


def workload_key(arch: str, prec: str, n_sys: int, n_points: int, sum_np_nb2: float) -> str:
    """Bucket of a workload: systems per handle (power of two), points (power of two) and the
    mean batch basis size sqrt(sum n_p n_b^2 / n_points) (in steps of 32)."""
    sys_b = 1 << max(0, math.ceil(math.log2(max(1, n_sys))))
    pts_b = 1 << max(0, round(math.log2(max(1, n_points))))
    nb_b = 32 * max(1, round(math.sqrt(sum_np_nb2 / max(1, n_points)) / 32))
    return f"{arch}|{prec}|sys{sys_b}|pts{pts_b}|nb{nb_b}"


def search(cost: Callable[[str, dict], float],
           density_pblocks: Iterable[int] = DENSITY_PBLOCKS,
           h_merge: Iterable[int] = H_MERGE,
           persistent: Iterable[int] = PERSISTENT,
           h_ratio: Iterable[int] = H_RATIO) -> Tuple[dict, Dict[str, float]]:
    """Pick the tuning that minimises density time + H time.

    ``cost(kind, cfg)`` returns the time of pass ``kind`` ("density" or "h") under ``cfg``
    (a dict with the knobs that pass depends on).  Returns (best cfg, {candidate label: ms})."""
    log: Dict[str, float] = {}
    best, best_t = None, math.inf
    h_parts = [(m, 0) for m in h_merge] + [(0, r) for r in h_ratio]
    for p in persistent:
        bd, td = None, math.inf
        for pb in density_pblocks:
            t = float(cost("density", {"density_pblocks": pb, "persistent": p}))
            log[f"density pblocks={pb} persistent={p}"] = t
            if t < td:
                bd, td = pb, t
        bh, th = None, math.inf
        for m, r in h_parts:
            t = float(cost("h", {"h_merge": m, "h_flops_per_atomic": r, "persistent": p}))
            log[f"h merge={m} ratio={r} persistent={p}"] = t
            if t < th:
                bh, th = (m, r), t
        if bd is not None and bh is not None and td + th < best_t:
            best = {"h_merge": bh[0], "h_flops_per_atomic": bh[1], "density_pblocks": bd,
                    "persistent": p}
            best_t = td + th
    if best is None:
        raise ValueError("empty candidate set")
    return best, log


def refine_buckets(cost: Callable[[str, dict], float], base: dict, density_flops: Sequence[float],
                   h_flops: Sequence[float], pblocks: Iterable[int] = DENSITY_PBLOCKS,
                   allow_h32: bool = True, min_gain: float = 0.005) -> Tuple[dict, Dict[str, float]]:
    """Per-bucket tile shapes on top of ``base`` by coordinate descent over the buckets that
    hold work.  ``cost(kind, cfg)`` times pass ``kind`` under the full tuning ``cfg``."""
    cfg = dict(base)
    cfg.setdefault("h_tile32_mask", 0)
    cfg["density_bucket_pblocks"] = list(cfg.get("density_bucket_pblocks") or [0] * len(density_flops))
    log: Dict[str, float] = {}
    pbl = list(pblocks)
    if len(pbl) > 1:
        t_best = float(cost("density", cfg))
        log["density base"] = t_best
        for b in sorted(range(len(density_flops)), key=lambda k: -density_flops[k]):
            if density_flops[b] <= 0:
                continue
            for pb in pbl:
                if pb == (cfg["density_bucket_pblocks"][b] or cfg["density_pblocks"]):
                    continue
                trial = dict(cfg, density_bucket_pblocks=list(cfg["density_bucket_pblocks"]))
                trial["density_bucket_pblocks"][b] = pb
                t = float(cost("density", trial))
                log[f"density bucket {b} pblocks={pb}"] = t
                if t < t_best * (1.0 - min_gain):
                    cfg, t_best = trial, t
    if allow_h32:
        t_best = float(cost("h", cfg))
        log["h base"] = t_best
        for b in sorted(range(len(h_flops)), key=lambda k: -h_flops[k]):
            if h_flops[b] <= 0:
                continue
            trial = dict(cfg, h_tile32_mask=cfg["h_tile32_mask"] ^ (1 << b))
            t = float(cost("h", trial))
            log[f"h bucket {b} tile32={(trial['h_tile32_mask'] >> b) & 1}"] = t
            if t < t_best * (1.0 - min_gain):
                cfg, t_best = trial, t
    return cfg, log


def load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store_cache(path: str, key: str, entry: dict) -> None:
    data = load_cache(path)
    data[key] = entry
    d = os.path.dirname(path) or "."
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".tuning.", suffix=".json")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(grid, P, v, prec: str = "fp64", *, reps: int = 3, cache: Optional[str] = None,
             force: bool = False, density_pblocks: Iterable[int] = DENSITY_PBLOCKS,
             h_merge: Iterable[int] = H_MERGE, persistent: Iterable[int] = PERSISTENT,
             h_ratio: Iterable[int] = H_RATIO, buckets: bool = True) -> dict:
    """Time the candidates on ``grid``'s device with inputs P, v (device tensors), apply the
    best tuning for ``prec`` and return {tuning..., "source": "cache"|"measured", "key": ...,
    "ms": {...}}.  ``cache=""`` disables the cache file."""
    import torch

    props = torch.cuda.get_device_properties(grid.device)
    arch = getattr(props, "gcnArchName", props.name).split(":")[0]
    ws = grid.work_stats()
    key = workload_key(arch, prec, grid.n_sys, grid.n_points, ws["sum_np_nb2"])
    path = default_cache_path() if cache is None else cache
    if path and not force:
        hit = load_cache(path).get(key)
        if hit and all(k in hit for k in KNOBS):
            grid.set_tuning(prec=prec, **{k: hit[k] for k in KNOBS})
            return dict(hit, source="cache", key=key)

    n = torch.empty(grid.n_points, dtype=torch.float64, device=grid.device)
    sums = torch.empty(grid.n_sys, 3, dtype=torch.float64, device=grid.device)
    H = torch.empty(grid.mat_elems, dtype=torch.float64, device=grid.device)
    cur = grid.get_tuning(prec)
    stream = grid.stream

    def run(kind):
        if kind == "density":
            grid.update_density(P, v, prec=prec, n_out=n, sums_out=sums)
        else:
            grid.integrate_h(v, prec=prec, H_out=H)

    def cost(kind, cfg):
        grid.set_tuning(h_merge=cfg.get("h_merge", cur["h_merge"]),
                        h_flops_per_atomic=cfg.get("h_flops_per_atomic", cur["h_flops_per_atomic"]),
                        density_pblocks=cfg.get("density_pblocks", cur["density_pblocks"]),
                        persistent=cfg["persistent"], prec=prec,
                        h_tile32_mask=cfg.get("h_tile32_mask", 0),
                        density_bucket_pblocks=cfg.get("density_bucket_pblocks", [0] * 8))
        run(kind)                                   # warm (first use builds the work lists)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            run(kind)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    if prec == "int8x7":            # its density tiles always span 64 points
        density_pblocks = (2,)
    best, log = search(cost, density_pblocks, h_merge, persistent, h_ratio)
    best = dict(best, h_tile32_mask=0, density_bucket_pblocks=[0] * 8)
    grid.set_tuning(prec=prec, **best)
    if buckets:
        _, dfl = grid.bucket_stats(prec, "density")
        _, hfl = grid.bucket_stats(prec, "h")
        best, blog = refine_buckets(cost, best, dfl, hfl, density_pblocks,
                                    allow_h32=prec in ("fp64", "fp32"))
        log.update(blog)
        grid.set_tuning(prec=prec, **best)
    entry = dict(best, ms=log)
    if path:
        store_cache(path, key, entry)
    return dict(entry, source="measured", key=key)
