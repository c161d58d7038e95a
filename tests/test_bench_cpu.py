"""Host-side logic of bench.py, on the CPU: the roofline of the dominant kernel credits
algorithmic flops only (a merged H partition's surplus is stated, not credited), every form
carries its own roofline, and a stored traffic record is used only for the exact kernel and
partitioning sources, workload, batching, form, family and tuning it was measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

TUNING = {"h_merge": 1, "density_pblocks": 2, "persistent": 1, "h_flops_per_atomic": 0}


def _kern(density_ms, hs_ms, steps=10, alg=182.7e9, executed=200.0e9):
    return {"density": {"work_flop": 2 * steps * alg, "ms_per_step": density_ms,
                        "launches": 2 * steps, "avg_launch_ms": density_ms / 2},
            "hs": {"work_flop": 2 * steps * executed, "ms_per_step": hs_ms,
                   "launches": 2 * steps, "avg_launch_ms": hs_ms / 2}}


def test_dominant_kernel_and_algorithmic_credit():
    r = bench._roofline(_kern(7.9, 8.6), "fp64", 10)
    assert r["kernel"] == "hs"
    # credited: the density partition's flops over the H kernel's time
    assert r["work_flop_per_launch"] == pytest.approx(182.7e9)
    assert r["executed_flop_per_launch"] == pytest.approx(200.0e9)
    assert r["achieved"] == pytest.approx(2 * 182.7e9 / 8.6e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6)
    r = bench._roofline(_kern(9.0, 8.6), "fp64", 10)
    assert r["kernel"] == "density" and r["executed_flop_per_launch"] == r["work_flop_per_launch"]


def test_bf16x3_states_the_mfma_fraction():
    r = bench._roofline(_kern(5.6, 3.8), "bf16x3", 10)
    assert r["peak"] == 2500.0 and r["mfma_flop_per_flop"] == 3
    assert r["mfma_frac"] == pytest.approx(3 * r["frac"])
    assert "mfma_frac" not in bench._roofline(_kern(7.9, 8.6), "fp32", 10)


def test_traffic_record_matching(tmp_path, monkeypatch):
    srcs = [tmp_path / "k.hip", tmp_path / "i.hip", tmp_path / "t.h"]
    for i, f in enumerate(srcs):
        f.write_text(f"kernel source {i}")
    import hashlib
    sha = hashlib.sha256(b"".join(f.read_bytes() for f in srcs)).hexdigest()
    rec = {"workload": "c2", "form": "fp64", "family": "hs", "tuning": TUNING,
           "fetch_bytes_per_launch": 5, "write_bytes_per_launch": 2, "sources_sha256": sha,
           "flop_per_step": 7.3e11}
    other = dict(rec, family="density", fetch_bytes_per_launch=100)
    f = tmp_path / "t.md"
    f.write_text("# summary\n\n" + json.dumps(other) + "\n" + json.dumps(rec) + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    monkeypatch.setattr(bench, "KERNEL_SRCS", [str(x) for x in srcs])
    assert bench._measured_traffic("c2", "fp64", "hs", TUNING, 7.3e11) == 7
    assert bench._measured_traffic("c2", "fp64", "density", TUNING, 7.3e11) == 102
    # any mismatch: no traffic
    assert bench._measured_traffic("c2", "fp64", "hs", TUNING, 7.4e11) is None      # batching
    assert bench._measured_traffic("c3", "fp64", "hs", TUNING, 7.3e11) is None      # workload
    assert bench._measured_traffic("c2", "fp32", "hs", TUNING, 7.3e11) is None      # form
    assert bench._measured_traffic("c2", "fp64", "hs", dict(TUNING, h_merge=2), 7.3e11) is None
    # a tuning field of the other family does not matter, one of its own does
    assert bench._measured_traffic("c2", "fp64", "hs", dict(TUNING, density_pblocks=5), 7.3e11) == 7
    assert bench._measured_traffic("c2", "fp64", "density", dict(TUNING, density_pblocks=5), 7.3e11) is None
    for x in srcs:                                   # any of the kernel sources changed
        old = x.read_text()
        x.write_text("changed")
        assert bench._measured_traffic("c2", "fp64", "hs", TUNING, 7.3e11) is None
        x.write_text(old)
    assert bench._measured_traffic("c2", "fp64", "hs", TUNING, 7.3e11) == 7


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr) or "1 GPU" in (p.stdout + p.stderr)
