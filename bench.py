#!/usr/bin/env python3
"""Throughput of one s.c.f. step of NAO real-space grid integration on one MI355X.

A step is one density update (n = sum_ij P_ij phi_i phi_j with the N, E_V, E_T sums) followed
by one Hamiltonian integration (H_ij = sum_p w_p phi_i (v phi_j + t phi_j)), on the 64-atom
random cluster (l <= 3 basis, 75 x 302 grid, batches <= 256 points) with inputs resident in
HBM.  Both the plain FP64 form and the mixed form are timed; ``value`` is the mixed form's
GFLOP/s with F = 4 sum_b n_p n_b^2 (the per-batch contractions, counted once), and its energy
error against the FP64 form is reported next to it.  One JSON line on stdout.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--mixed fp32|bf16x3]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}   # MI355X dense MFMA peaks
HBM_GBS = 8000.0


def _cpu_baseline(inst, F, n_chunks, seed=0):
    """The FP64 oracle as it stands, on a bounded random sample of point chunks of the same
    workload, extrapolated to the whole step by the point count."""
    from oracle import GridOracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    o = GridOracle(inst)
    rng = np.random.default_rng(seed)
    nch = (inst.n_points + o.chunk - 1) // o.chunk
    pick = np.sort(rng.choice(nch, size=min(n_chunks, nch), replace=False))
    idx = np.concatenate([np.arange(c * o.chunk, min(inst.n_points, (c + 1) * o.chunk)) for c in pick])
    t0 = time.perf_counter()
    o.density(inst.P, inst.v, points=idx)
    o.integrate_h(inst.v, want_S=False, points=idx)
    dt = time.perf_counter() - t0
    t_full = dt * inst.n_points / idx.size
    return {"value": F / t_full / 1e9, "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "s_per_step": t_full,
            "sample": f"{len(pick)} random chunks of {o.chunk} points ({idx.size} of "
                      f"{inst.n_points} points, {dt:.1f} s), extrapolated by point count"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mixed", default="fp32", choices=["fp32", "bf16x3"])
    ap.add_argument("--cpu-chunks", type=int, default=10,
                    help="point chunks of the oracle's CPU baseline sample (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the batches would shard across GPUs with one FP64 reduction of H; see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2208_12335_amd import AimsGrid

    dev = torch.device("cuda", 0)
    t0 = time.time()
    inst = synth.make_instance("c2", seed=0)
    print(f"[bench] instance: {inst.n_points} points, {inst.n_basis} functions "
          f"({time.time() - t0:.1f} s)", file=sys.stderr, flush=True)
    t0 = time.time()
    g = AimsGrid(inst, device=0)
    ws = g.work_stats()
    F = ws["flops_per_step"]
    print(f"[bench] setup {time.time() - t0:.1f} s, {ws['n_batches']} batches, "
          f"F = {F:.3e} flop/step", file=sys.stderr, flush=True)
    P = torch.from_numpy(inst.P).to(dev).reshape(-1)
    v = torch.from_numpy(inst.v).to(dev)
    n = torch.empty(g.n_points, dtype=torch.float64, device=dev)
    sums = torch.empty(1, 3, dtype=torch.float64, device=dev)
    H = torch.empty(g.mat_elems, dtype=torch.float64, device=dev)
    stream = g.stream

    def step(prec):
        g.update_density(P, v, prec=prec, n_out=n, sums_out=sums)
        g.integrate_h(v, prec=prec, H_out=H)

    res = {}
    for prec in ("fp64", args.mixed):
        for _ in range(args.warmup):
            step(prec)
        torch.cuda.synchronize()
        g.profile(True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record(stream)
        for _ in range(args.steps):
            step(prec)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - w0) / args.steps * 1e3
        ms = e0.elapsed_time(e1) / args.steps
        kern = {}
        for k in ("phi_eval", "density", "hs", "finish"):
            cnt, kms, work = g.profile_read(k)
            kern[k] = {"launches": cnt, "ms_per_step": kms / args.steps,
                       "avg_launch_ms": kms / cnt if cnt else 0.0, "work_flop": work}
        g.profile(False)
        s = sums.cpu().numpy()[0]
        res[prec] = {"ms_per_step": ms, "wall_ms_per_step": wall, "gflops": F / (ms * 1e-3) / 1e9,
                     "N": float(s[0]), "E": float(s[1] + s[2]), "kernels": kern,
                     "H_fro": float(torch.linalg.norm(H).item())}
        print(f"[bench] {prec}: {ms:.3f} ms/step, {res[prec]['gflops']:.1f} GFLOP/s", file=sys.stderr,
              flush=True)

    mixed = res[args.mixed]
    dE = abs(mixed["E"] - res["fp64"]["E"])
    # dominant kernel of the mixed form: the MFMA kernel with the most time per step
    dom = max(("density", "hs"), key=lambda k: mixed["kernels"][k]["ms_per_step"])
    kd = mixed["kernels"][dom]
    achieved = kd["work_flop"] / (kd["ms_per_step"] * args.steps * 1e-3) / 1e12 if kd["ms_per_step"] else 0.0
    roof = {"kernel": dom, "bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[args.mixed],
            "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[args.mixed], "traffic": None,
            "avg_launch_ms": kd["avg_launch_ms"], "launches_per_step": kd["launches"] / args.steps}
    line = {
        "metric": "H+density integration GFLOP/s (mixed precision, FP32 MFMA per batch, FP64 reduce)",
        "value": mixed["gflops"], "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": mixed["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if args.mixed == "fp32" else "bf16x3",
        "data": "synthetic",
        "config": {"workload": "64-atom random cluster (Z in {1,6,8}, box 20 bohr), l<=3 NAO basis "
                               f"({inst.n_basis} functions), 75x302 grid ({inst.n_points} points), "
                               "batches <= 256 points; one step = density update + H integration",
                   "n_points": inst.n_points, "n_basis": inst.n_basis,
                   "n_batches": ws["n_batches"], "flop_per_step": F, "parallelism": "single GPU"},
        "fp64": {"ms_per_step": res["fp64"]["ms_per_step"], "gflops": res["fp64"]["gflops"],
                 "frac_of_fp64_peak": res["fp64"]["gflops"] / 1e3 / PEAK_TFLOPS["fp64"]},
        "mixed_vs_fp64": {"speedup": res["fp64"]["ms_per_step"] / mixed["ms_per_step"],
                          "abs_dE_Ha": dE, "E_fp64": res["fp64"]["E"], "E_mixed": mixed["E"],
                          "meets_1e-6_Ha": bool(dE <= 1e-6),
                          "rel_dN": abs(mixed["N"] - res["fp64"]["N"]) / abs(res["fp64"]["N"]),
                          "rel_dH_fro": abs(mixed["H_fro"] - res["fp64"]["H_fro"]) / res["fp64"]["H_fro"]},
        "kernels": {p: r["kernels"] for p, r in res.items()},
        "roofline": roof,
    }
    if args.cpu_chunks > 0:
        print("[bench] CPU baseline (oracle sample)...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = _cpu_baseline(inst, F, args.cpu_chunks)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
