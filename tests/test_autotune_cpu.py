"""Host logic of the autotuner: candidate search, workload buckets and the JSON cache."""
import json

import pytest

from paper_2208_12335_amd.autotune import load_cache, search, store_cache, workload_key


def test_search_picks_min_of_sum_per_persistent_flag():
    # density favours persistent=1 slightly, H favours persistent=0 strongly
    d = {(2, 0): 5.0, (3, 0): 4.0, (4, 0): 4.5, (5, 0): 6.0,
         (2, 1): 3.9, (3, 1): 3.8, (4, 1): 4.2, (5, 1): 5.0}
    h = {(0, 0): 9.0, (1, 0): 6.0, (2, 0): 7.0, (3, 0): 8.0,
         (0, 1): 9.5, (1, 1): 8.0, (2, 1): 7.5, (3, 1): 8.5}
    calls = []

    def cost(kind, cfg):
        calls.append((kind, dict(cfg)))
        if kind == "density":
            return d[(cfg["density_pblocks"], cfg["persistent"])]
        return h[(cfg["h_merge"], cfg["persistent"])]

    best, log = search(cost, h_ratio=[])
    # persistent=0: 4.0 + 6.0 = 10.0 ; persistent=1: 3.8 + 7.5 = 11.3
    assert best == {"h_merge": 1, "h_flops_per_atomic": 0, "density_pblocks": 3, "persistent": 0}
    assert len(calls) == 16 and len(log) == 16
    # the density pass is never timed with an h_merge knob and vice versa
    assert all("h_merge" not in c for k, c in calls if k == "density")
    assert all("density_pblocks" not in c for k, c in calls if k == "h")


def test_search_restricted_candidates_and_empty():
    best, _ = search(lambda k, c: 1.0, density_pblocks=[4], h_merge=[2], persistent=[1], h_ratio=[])
    assert best == {"h_merge": 2, "h_flops_per_atomic": 0, "density_pblocks": 4, "persistent": 1}
    with pytest.raises(ValueError):
        search(lambda k, c: 1.0, persistent=[])


def test_search_cost_model_partition():
    # the cost-model partition with ratio 256 beats every fixed level; the density knobs are
    # timed without any H knob
    def cost(kind, cfg):
        if kind == "density":
            assert set(cfg) == {"density_pblocks", "persistent"}
            return 5.0
        if cfg["h_flops_per_atomic"]:
            assert cfg["h_merge"] == 0
            return {64: 7.0, 256: 5.5, 1024: 6.0, 4096: 8.0}[cfg["h_flops_per_atomic"]]
        return 6.5 + cfg["h_merge"]
    best, log = search(cost)
    assert best["h_flops_per_atomic"] == 256 and best["h_merge"] == 0
    assert len(log) == 2 * (4 + 4 + 4)


def test_workload_key_buckets():
    k1 = workload_key("gfx950", "fp64", 1, 1_122_621, 1_122_621 * 410.0 ** 2)
    k2 = workload_key("gfx950", "fp64", 1, 1_100_000, 1_100_000 * 405.0 ** 2)
    assert k1 == k2 == "gfx950|fp64|sys1|pts1048576|nb416"
    assert workload_key("gfx950", "fp32", 1, 1_122_621, 1.0) != k1
    assert "sys256" in workload_key("gfx950", "fp64", 256, 10_000_000, 1e12)
    assert "sys256" in workload_key("gfx950", "fp64", 200, 10_000_000, 1e12)


def test_cache_roundtrip(tmp_path):
    p = str(tmp_path / "sub" / "tuning.json")
    assert load_cache(p) == {}
    store_cache(p, "a", {"h_merge": 1, "density_pblocks": 3, "persistent": 0})
    store_cache(p, "b", {"h_merge": 2, "density_pblocks": 5, "persistent": 1})
    data = load_cache(p)
    assert data["a"]["density_pblocks"] == 3 and data["b"]["persistent"] == 1
    with open(p, "w") as f:
        f.write("{not json")
    assert load_cache(p) == {}
    with open(p, "w") as f:
        json.dump([1, 2], f)
    assert load_cache(p) == {}


def test_refine_buckets_per_bucket_choices():
    """Coordinate descent over the tile-shape buckets: each bucket with work gets the shape that
    makes its pass faster; buckets without work are never timed; small gains are ignored."""
    from paper_2208_12335_amd.autotune import refine_buckets
    dfl = [0.0, 5.0, 0.0, 9.0, 0.0, 0.0, 0.0, 1.0]
    hfl = [0.0] * 16
    hfl[2], hfl[5], hfl[9] = 4.0, 7.0, 1.0

    def cost(kind, cfg):
        if kind == "density":
            bp = cfg["density_bucket_pblocks"]
            pb = lambda b: bp[b] or cfg["density_pblocks"]
            t = 10.0
            t -= 1.0 if pb(3) == 4 else 0.0        # bucket 3 likes 4 point blocks
            t -= 0.5 if pb(1) == 5 else 0.0        # bucket 1 likes 5
            t -= 0.01 if pb(7) == 3 else 0.0       # below the 0.5% threshold
            return t
        m = cfg["h_tile32_mask"]
        return 20.0 - (2.0 if m >> 5 & 1 else 0.0) + (1.0 if m >> 2 & 1 else 0.0)

    timed = []
    base = {"h_merge": 1, "h_flops_per_atomic": 0, "density_pblocks": 2, "persistent": 1}
    best, log = refine_buckets(lambda k, c: (timed.append((k, c)), cost(k, c))[1], base, dfl, hfl)
    assert best["density_bucket_pblocks"] == [0, 5, 0, 4, 0, 0, 0, 0]
    assert best["h_tile32_mask"] == 1 << 5
    assert all(k in best for k in base)
    # empty buckets are never tried
    assert not any("bucket 0 " in k or "bucket 2 p" in k for k in log)
    assert not any("h bucket 0 " in k for k in log)
    # FP64 / FP32 only for the 32 x 32 H tiles
    best2, _ = refine_buckets(cost, base, dfl, hfl, allow_h32=False)
    assert best2["h_tile32_mask"] == 0
