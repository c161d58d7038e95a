#!/usr/bin/env python3
"""Throughput of one s.c.f. step of NAO real-space grid integration on one MI355X.

A step is one density update (n = sum_ij P_ij phi_i phi_j with the N, E_V, E_T sums) followed
by one Hamiltonian integration (H_ij = sum_p w_p phi_i (v phi_j + t phi_j)), with inputs
resident in HBM.  GFLOP/s use F = 4 sum_b n_p n_b^2 (the per-batch contractions, counted once,
also for BF16x3).  The FP64 form and the mixed forms are timed; the headline ``value`` is the
fastest form whose total energy stays within 1e-6 Ha of the FP64 form.  Every form carries its
own roofline (dominant kernel, algorithmic flops against the MFMA peak of its type; BF16x3
also states the fraction at three bf16 MFMA flops per algorithmic flop).  One JSON line on
stdout.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--workload c2|c3|c4|c5]

Workloads: c2 (default) the 64-atom random cluster, 75 x 302 grid, batches <= 256 (its line
also carries c3, c4 and c5 under "scale_c3", "grouped_c4" and "backward_c5", unless --extras ''
or --step-only);
c3 the 512-atom water cluster; c4 256 independent molecules in one grouped handle (timed as a
graph replay, as eager calls and as 256 per-molecule launch sets); c5 the 128-atom cluster,
forward + backward (dE/dP, dE/dv, dE/dR) per step, F = 8 sum_b n_p n_b^2.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "int8x7": 5000.0}   # MI355X dense MFMA peaks (int8: TOP/s)
MFMA_PER_FLOP_INT8 = {"density": 34, "hs": 28}   # int8 digit products per product
SINGLE_SCRATCH_MB = 512     # scratch budget of each per-molecule baseline handle (c4)
HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(HERE, "profiles", "tiled_kernels_c2_all_forms_counters.md")
KERNEL_SRCS = [os.path.join(HERE, "paper_2208_12335_amd", "csrc", f)
               for f in ("kernels.hip", "int8.hip", "tiles.h")]
# the tuning fields that shape each family's launches
FAMILY_TUNING = {"density": ("density_pblocks", "density_bucket_pblocks", "persistent"),
                 "hs": ("h_merge", "h_flops_per_atomic", "h_tile32_mask", "persistent")}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "int8x7": "int8x7"}
FAMILIES = ("phi_eval", "density", "hs", "backward", "finish", "operands")

WORKLOADS = {
    "c2": "64-atom random cluster (Z in {1,6,8}, box 20 bohr), l<=3 NAO basis, 75x302 grid, "
          "batches <= 256 points; one step = density update + H integration",
    "c3": "512-atom water cluster (170 H2O + OH, 1 g/cm^3), l<=3 NAO basis, 75x302 grid, "
          "batches <= 300 points; one step = density update + H integration",
    "c4": "256 independent molecules (3-40 atoms, Z in {1,6,7,8}) in one grouped handle, "
          "l<=2 NAO basis, 50x110 grid, batches <= 200 points; one step = density update + "
          "H integration of every molecule",
    "c5": "128-atom random cluster (box 25.2 bohr), l<=3 NAO basis, 75x302 grid, batches <= "
          "256; one step = density update + backward (dE/dP, dE/dv, dE/dR)",
}


def _threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count() or 1


def _cpu_baseline(inst, F, n_chunks, seed=0):
    """The FP64 oracle as it stands, on a bounded random sample of point chunks of the same
    workload, extrapolated to the whole step by the point count."""
    from oracle import GridOracle
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
    return {"value": F / t_full / 1e9, "unit": "GFLOP/s", "cores": int(_threads()), "kind": "oracle",
            "s_per_step": t_full,
            "sample": f"{len(pick)} random chunks of {o.chunk} points ({idx.size} of "
                      f"{inst.n_points} points, {dt:.1f} s), extrapolated by point count"}


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class Timer:
    """HIP events on the library stream around K steps (the kernels run on that stream)."""

    def __init__(self, torch, stream):
        self.torch, self.stream = torch, stream

    def run(self, fn, steps, warmup):
        """Mean ms per step over the K steps (events around all of them), wall-clock ms per
        step; per-step event pairs give the median and minimum in ``self.last``."""
        torch = self.torch
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        w0 = time.perf_counter()
        ev[0].record(self.stream)
        for i in range(steps):
            fn()
            ev[i + 1].record(self.stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - w0) / steps * 1e3
        per = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
        self.last = {"median": per[len(per) // 2], "min": per[0]}
        return ev[0].elapsed_time(ev[-1]) / steps, wall


def _kernels(g, steps):
    out = {}
    for k in FAMILIES:
        cnt, kms, work = g.profile_read(k)
        if cnt:
            out[k] = {"launches": cnt, "ms_per_step": kms / steps, "avg_launch_ms": kms / cnt,
                      "work_flop": work}
    return out


def _measured_traffic(workload, form, family, tuning, flop_per_step=None):
    """HBM bytes per launch of the dominant kernel from the committed profiler summary (two
    rocprofv3 --pmc passes, FETCH_SIZE and WRITE_SIZE, scaled by a plain copy kernel), used only
    when that summary was taken on the same kernel sources, workload (and batching: the same
    algorithmic flops per step), form and tuning fields of that kernel family."""
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
        recs = [json.loads(l) for l in text.splitlines() if l.startswith("{")]
        sha = hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SRCS)).hexdigest()
    except (OSError, ValueError):
        return None
    keys = FAMILY_TUNING.get(family, ())
    for rec in recs:
        if (rec.get("sources_sha256") == sha and rec.get("workload") == workload and
                rec.get("form") == form and rec.get("family") == family and
                rec.get("flop_per_step") == flop_per_step and tuning is not None and
                all(rec.get("tuning", {}).get(k) == tuning.get(k) for k in keys)):
            return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    return None


def _roofline(kern, head, steps, workload=None, tuning=None, flop_per_step=None):
    dom = max(("density", "hs"), key=lambda k: kern.get(k, {}).get("ms_per_step", 0.0))
    kd = kern[dom]
    # algorithmic flops: 2 sum n_p n_b^2 over the density partition.  A merged H partition
    # executes more (each merged batch screens the union of its halves' atoms); that surplus is
    # stated beside the roofline, not credited.
    work = kd["work_flop"]
    executed = work
    if dom == "hs" and "density" in kern:
        work = min(work, kern["density"]["work_flop"])
    achieved = work / (kd["ms_per_step"] * steps * 1e-3) / 1e12
    return {"kernel": dom, "bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[head],
            "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[head],
            "traffic": _measured_traffic(workload, head, dom, tuning, flop_per_step),
            "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "avg_launch_ms": kd["avg_launch_ms"], "launches_per_step": kd["launches"] / steps,
            "work_flop_per_launch": work / kd["launches"],
            "executed_flop_per_launch": executed / kd["launches"],
            **({"mfma_flop_per_flop": 3, "mfma_frac": 3.0 * achieved / PEAK_TFLOPS[head]}
               if head == "bf16x3" else {}),
            # int8 digit products per algorithmic multiply-add pair: 34 (density), 28 (H)
            **({"mfma_flop_per_flop": MFMA_PER_FLOP_INT8[dom],
                "mfma_frac": MFMA_PER_FLOP_INT8[dom] * achieved / PEAK_TFLOPS[head]}
               if head == "int8x7" else {})}


def _forms_summary(res):
    ref = res["fp64"]
    for prec, r in res.items():
        r["abs_dE_Ha_vs_fp64"] = abs(r["E"] - ref["E"])
        r["rel_dN_vs_fp64"] = abs(r["N"] - ref["N"]) / abs(ref["N"])
        r["meets_1e-6_Ha"] = bool(r["abs_dE_Ha_vs_fp64"] <= 1e-6)
    ok = [p for p in res if res[p]["meets_1e-6_Ha"]]
    head = min(ok, key=lambda p: res[p]["ms_per_step"])
    fastest = min(res, key=lambda p: res[p]["ms_per_step"])
    return head, fastest


def _make(workload, torch):
    import synth
    if workload == "c2":
        return synth.make_instance("c2", seed=0)
    with synth.generator_device(torch.device("cuda", 0)):
        if workload == "c4":
            return synth.make_molecule_set(n_mol=256, seed=0)
        return synth.make_instance(workload, seed=0)


def _time_forms(args, torch, g, P, v, F, forms, fixed, backward, steps, warmup, timer, n, sums,
                H, gE, reps=2):
    """Every precision form on one handle: autotuned (or fixed) tuning, then K timed steps."""
    from paper_2208_12335_amd.autotune import autotune
    res = {}
    for prec in forms:
        if prec in fixed:
            g.set_tuning(prec=prec, **fixed[prec])
        elif not args.no_autotune:
            t0 = time.time()
            r = autotune(g, P, v, prec=prec, reps=reps, cache="")   # measured here, never cached
            _log(f"{prec}: autotuned {dict((k, r[k]) for k in ('h_merge', 'density_pblocks', 'persistent', 'h_flops_per_atomic', 'h_tile32_mask', 'density_bucket_pblocks') if k in r)}"
                 f" ({time.time() - t0:.1f} s)")

        if backward:
            def step():
                g.update_density(P, v, prec=prec, n_out=n, sums_out=sums)
                g.backward(P, v, gE, prec=prec)
        else:
            def step():
                g.update_density(P, v, prec=prec, n_out=n, sums_out=sums)
                g.integrate_h(v, prec=prec, H_out=H)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        g.profile(True)
        ms, wall = timer.run(step, steps, 0)
        kern = _kernels(g, steps)
        g.profile(False)
        s = sums.cpu().numpy()[0]
        res[prec] = {"ms_per_step": ms, "wall_ms_per_step": wall, "gflops": F / (ms * 1e-3) / 1e9,
                     "ms_per_step_median": timer.last["median"], "ms_per_step_min": timer.last["min"],
                     "N": float(s[0]), "E": float(s[1] + s[2]), "kernels": kern,
                     "tuning": g.get_tuning(prec)}
        _log(f"{prec}: {ms:.3f} ms/step, {res[prec]['gflops']:.1f} GFLOP/s")
    return res


def bench_scale_c3(args, torch, forms):
    """The 512-atom water cluster beside the headline workload: every form autotuned (one
    repetition per candidate) and timed over a few steps; the same per-form record as the
    headline's, without the measurements outside the step."""
    import synth
    from paper_2208_12335_amd import AimsGrid
    dev = torch.device("cuda", 0)
    t0 = time.time()
    with synth.generator_device(dev):
        inst = synth.make_instance("c3", seed=0)
    t_inst = time.time() - t0
    t0 = time.time()
    g = AimsGrid(inst, device=0)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    ws = g.work_stats()
    F = ws["flops_per_step"]
    _log(f"c3: instance {t_inst:.1f} s, setup {setup_s:.1f} s, {ws['n_batches']} batches, F = {F:.3e}")
    P = torch.from_numpy(inst.P).to(dev).reshape(-1)
    v = torch.from_numpy(inst.v).to(dev)
    n = torch.empty(g.n_points, dtype=torch.float64, device=dev)
    sums = torch.empty(1, 3, dtype=torch.float64, device=dev)
    H = torch.empty(g.mat_elems, dtype=torch.float64, device=dev)
    timer = Timer(torch, g.stream)
    steps, warmup = 3, 1
    res = _time_forms(args, torch, g, P, v, F, forms, {}, False, steps, warmup, timer, n, sums, H,
                      None, reps=1)
    head, fastest = _forms_summary(res)
    dm = _density_matrix_at_scale(torch, g, inst, v, H, timer, res, n, sums)
    out = {"config": {"workload": WORKLOADS["c3"], "n_points": inst.n_points,
                      "n_basis": inst.n_basis, "n_batches": ws["n_batches"], "flop_per_step": F,
                      "sum_np_nb2": ws["sum_np_nb2"], "setup_s": setup_s, "instance_s": t_inst},
           "steps": steps, "warmup": warmup, "headline_form": head,
           "value": res[head]["gflops"], "unit": "GFLOP/s", "ms_per_step": res[head]["ms_per_step"],
           "forms": {p: {k: r[k] for k in ("ms_per_step", "ms_per_step_median", "ms_per_step_min",
                                            "gflops", "abs_dE_Ha_vs_fp64", "meets_1e-6_Ha",
                                            "rel_dN_vs_fp64", "tuning", "E", "N")}
                        | {"roofline": _roofline(r["kernels"], p, steps, "c3", r["tuning"], F)}
                     for p, r in res.items()},
           "fastest_form": {"form": fastest, "ms_per_step": res[fastest]["ms_per_step"]},
           "kernels": {p: r["kernels"] for p, r in res.items()},
           "density_matrix_fp64": dm}
    del g
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def _density_matrix_at_scale(torch, g, inst, v, H, timer, res, n, sums):
    """The step after H on a large system: the occupied-subspace density matrix by the
    eigensolver and by purification (times and their agreement), and every form's density
    pass on that occupied-orbital P next to two FP64 routes to its energy (the density pass,
    and tr(P H) from the H pass)."""
    dev = H.device
    nb = inst.n_basis
    S = torch.empty_like(H)
    g.set_tuning(prec="fp64", **res["fp64"]["tuning"])
    g.integrate_h(v, prec="fp64", H_out=H, S_out=S, want_S=True)
    n_e = float(np.sum(inst.atom_Z))
    n_e -= n_e % 2
    P_eig = torch.empty_like(H)
    P_pur = torch.empty_like(H)
    out = {"n_electrons": n_e, "n_basis": nb}
    ms, _ = timer.run(lambda: g.density_matrix(H, S, n_e, method="eigen", P_out=P_eig,
                                               want_eps=False), 2, 1)
    out["eigen"] = {"ms": ms}
    try:
        ms, _ = timer.run(lambda: g.density_matrix(H, S, n_e, method="purify", P_out=P_pur,
                                                   want_eps=False), 3, 1)
        k = g.last_purify_products()
        S_alt = (S * (1.0 + 2.0 ** -40)).contiguous()
        flip = [S_alt, S]

        def solve_factor():
            flip.reverse()
            g.density_matrix(H, flip[0], n_e, method="purify", P_out=P_pur, want_eps=False)
        ms_f, _ = timer.run(solve_factor, 2, 0)
        g.density_matrix(H, S, n_e, method="purify", P_out=P_pur, want_eps=False)
        out["purify"] = {"ms": ms, "ms_with_factorisation": ms_f, "products": k,
                         "symmetric_product_tflops": k * float(nb) ** 3 / (ms * 1e-3) / 1e12,
                         "max_abs_dP_vs_eigen_rel": float((P_pur - P_eig).abs().max() /
                                                          P_eig.abs().max()),
                         "tr_PS_minus_n_e": float((P_pur * S).sum()) - n_e,
                         "speedup_vs_eigen": out["eigen"]["ms"] / ms}
        _log(f"c3 density matrix: eigen {out['eigen']['ms']:.1f} ms, purify {ms:.1f} ms "
             f"({k} products)")
    except Exception as e:                      # e.g. no gap for the purification
        out["purify"] = {"error": str(e)}
    out["eigen"]["tr_PS_minus_n_e"] = float((P_eig * S).sum()) - n_e
    out["max_abs_P"] = float(P_eig.abs().max())
    del S, P_pur
    occ = {}
    for prec in res:
        g.set_tuning(prec=prec, **res[prec]["tuning"])
        g.update_density(P_eig, v, prec=prec, n_out=n, sums_out=sums)
        s_ = sums.cpu().numpy()[0]
        occ[prec] = {"E": float(s_[1] + s_[2]), "N": float(s_[0])}
    e64 = occ["fp64"]["E"]
    for prec, r in occ.items():
        if prec != "fp64":
            r["abs_dE_Ha_vs_fp64"] = abs(r["E"] - e64)
            r["meets_1e-6_Ha"] = r["abs_dE_Ha_vs_fp64"] <= 1e-6
    g.integrate_h(v, prec="fp64", H_out=H)
    occ["fp64_trPH_minus_density_route_Ha"] = float((P_eig * H).sum()) - e64
    out["forms_on_occupied_P"] = occ
    _log(f"c3 forms on the occupied P: {json.dumps(occ)}")
    del P_eig
    torch.cuda.empty_cache()
    return out


def bench_extra_c4(args, torch):
    """The grouped workload beside the headline: the c4 record (3 timed steps)."""
    import copy
    a = copy.copy(args)
    a.steps, a.warmup, a.workload = 3, 1, "c4"
    t0 = time.time()
    mols = _make("c4", torch)
    _log(f"c4: instance {time.time() - t0:.1f} s")
    rec = bench_grouped(a, torch, mols)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    for k in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data"):
        rec.pop(k, None)
    return rec


def bench_extra_c5(args, torch, forms):
    """The backward workload beside the headline: every form, density + backward per step
    (3 timed steps, autotuned with one repetition), without the total-force measurements."""
    import copy
    a = copy.copy(args)
    a.steps, a.warmup, a.workload, a.step_only, a.cpu_chunks, a.extras, a.tuning = 3, 1, "c5", True, 0, "", ""
    a.forms = ",".join(f for f in forms if f != "int8x7")     # the sliced form has no backward
    t0 = time.time()
    inst = _make("c5", torch)
    _log(f"c5: instance {time.time() - t0:.1f} s")
    rec = bench_single(a, torch, inst, backward=True, reps=1)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    keep = ("value", "unit", "ms_per_step", "headline_form", "config", "forms", "fastest_form",
            "kernels", "roofline")
    return {k: rec[k] for k in keep if k in rec} | {"steps": a.steps, "warmup": a.warmup}


def bench_single(args, torch, inst, backward=False, reps=2):
    """c2 / c3 / c5: one handle, every precision form, optionally with the backward."""
    from paper_2208_12335_amd import AimsGrid

    dev = torch.device("cuda", 0)
    t0 = time.time()
    g = AimsGrid(inst, device=0)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    ws = g.work_stats()
    F = ws["flops_per_step"] * (2.0 if backward else 1.0)
    _log(f"setup {time.time() - t0:.1f} s, {ws['n_batches']} batches, F = {F:.3e} flop/step")
    P = torch.from_numpy(inst.P).to(dev).reshape(-1)
    v = torch.from_numpy(inst.v).to(dev)
    n = torch.empty(g.n_points, dtype=torch.float64, device=dev)
    sums = torch.empty(1, 3, dtype=torch.float64, device=dev)
    H = torch.empty(g.mat_elems, dtype=torch.float64, device=dev)
    gE = torch.ones(1, dtype=torch.float64, device=dev)
    timer = Timer(torch, g.stream)

    forms = ["fp64"] + [f for f in args.forms.split(",") if f and f != "fp64"]
    fixed = json.loads(args.tuning) if args.tuning else {}
    res = _time_forms(args, torch, g, P, v, F, forms, fixed, backward, args.steps, args.warmup,
                      timer, n, sums, H, gE, reps=reps)
    head, fastest = _forms_summary(res)
    hr = res[head]
    # outside the step: the overlap matrix (computed once per geometry)
    S = torch.empty(g.mat_elems, dtype=torch.float64, device=dev)
    g.set_tuning(prec="fp64", **res["fp64"]["tuning"])
    ms_S, _ = timer.run(lambda: g.integrate_h(v, prec="fp64", H_out=H, S_out=S, want_S=True), 3, 1)
    outside = {"setup_s": setup_s, "ms_integrate_h_with_S_fp64": ms_S}
    if not backward and not args.step_only:
        # the step after H: the occupied-subspace density matrix (closed shell), and a whole
        # s.c.f. iteration (density + H + density matrix) with the density-matrix share of it
        n_e = float(np.sum(inst.atom_Z))
        n_e -= n_e % 2
        P_new = torch.empty(g.mat_elems, dtype=torch.float64, device=dev)
        dm = {"n_electrons": n_e, "n_basis": inst.n_basis}
        for meth in ("eigen", "purify"):
            def solve():
                g.density_matrix(H, S, n_e, method=meth, P_out=P_new, want_eps=False)
            try:
                ms_dm, _ = timer.run(solve, 3, 1)
            except Exception as e:                 # e.g. no gap for the purification
                dm[meth] = {"error": str(e)}
                continue
            r = {"ms": ms_dm}
            if meth == "purify":
                k = g.last_purify_products()
                r["products"] = k
                # the inverse factor of S is kept while S is unchanged (every s.c.f. iteration
                # after the first); alternating two overlap matrices times the call that also
                # factorises S
                S_alt = (S * (1.0 + 2.0 ** -40)).contiguous()
                flip = [S_alt, S]
                def solve_factor():
                    flip.reverse()
                    g.density_matrix(H, flip[0], n_e, method=meth, P_out=P_new, want_eps=False)
                r["ms_with_factorisation"], _ = timer.run(solve_factor, 4, 0)
                r["symmetric_product_tflops"] = k * float(inst.n_basis) ** 3 / (ms_dm * 1e-3) / 1e12
            ms_it = res["fp64"]["ms_per_step"] + ms_dm
            r["scf_iteration_ms"] = ms_it
            r["density_matrix_share"] = ms_dm / ms_it
            dm[meth] = r
            _log(f"density matrix ({meth}): {ms_dm:.2f} ms")
        outside["density_matrix_fp64"] = dm
        # the potential step of a semilocal s.c.f. iteration on the occupied density: n and
        # grad n, LDA and PBE, H with the gradient term; with the density matrix, a whole GGA
        # iteration (density + gradient, PBE, H, density matrix)
        if "ms" in dm.get("eigen", {}):
            g.density_matrix(H, S, n_e, method="eigen", P_out=P_new, want_eps=False)
            nn = torch.empty(g.n_points, dtype=torch.float64, device=dev)
            gr = torch.empty(g.n_points, 3, dtype=torch.float64, device=dev)
            H2 = torch.empty(g.mat_elems, dtype=torch.float64, device=dev)
            xc = {}
            xc["ms_density_and_gradient"], _ = timer.run(
                lambda: g.density_gradient(P_new, n_out=nn, grad_out=gr), 3, 1)
            xc["ms_lda"], _ = timer.run(lambda: g.xc(nn), 3, 1)
            vn, u, _ = g.xc_gga(nn, gr)
            xc["ms_pbe"], _ = timer.run(lambda: g.xc_gga(nn, gr), 3, 1)
            vt = v + vn
            xc["ms_h_with_gradient_term"], _ = timer.run(
                lambda: g.integrate_h_gga(vt, u, H_out=H2), 3, 1)
            best_dm = min((r["ms"] for r in dm.values() if isinstance(r, dict) and "ms" in r))
            xc["gga_iteration_ms"] = (xc["ms_density_and_gradient"] + xc["ms_pbe"] +
                                      xc["ms_h_with_gradient_term"] + best_dm)
            outside["xc_fp64"] = xc
            _log(f"xc: {json.dumps({k: round(x, 3) for k, x in xc.items()})}")
            # the mixed forms' energy error on the occupied-orbital density matrix (physical P,
            # n >= 0) next to the random-sign P of the workload
            occ = {}
            e64 = None
            for prec in ("fp64", "fp32", "bf16x3", "int8x7"):
                g.update_density(P_new, v, prec=prec, n_out=nn, sums_out=sums)
                s_ = sums.cpu().numpy()[0]
                e = float(s_[1] + s_[2])
                if prec == "fp64":
                    e64 = e
                else:
                    occ[prec] = {"abs_dE_Ha_vs_fp64": abs(e - e64), "meets_1e-6_Ha": abs(e - e64) <= 1e-6}
            occ["E_fp64"] = e64
            outside["mixed_forms_on_occupied_P"] = occ
            _log(f"mixed forms on occupied P: {json.dumps(occ)}")
            # the electrostatic step and one whole LDA s.c.f. iteration (density, Hartree,
            # exchange-correlation, H, density matrix)
            import synth
            g.set_hartree_grid([synth.radial_shells(inst)], l_max=6)
            vh = torch.empty(g.n_points, dtype=torch.float64, device=dev)
            EH = torch.empty(1, dtype=torch.float64, device=dev)
            g.hartree(nn, v_out=vh, E_out=EH)                       # first call builds tables
            it = {"l_max": 6}
            it["ms_hartree"], _ = timer.run(lambda: g.hartree(nn, v_out=vh, E_out=EH), 3, 1)
            vx = torch.empty(g.n_points, dtype=torch.float64, device=dev)

            def scf_iteration():
                g.update_density(P_new, v, prec="fp64", n_out=nn, sums_out=sums)
                g.hartree(nn, v_out=vh, E_out=EH)
                g.xc(nn, v_out=vx)
                torch.add(vh, vx, out=vt)
                vt.add_(v)
                g.integrate_h(vt, prec="fp64", H_out=H2)
                g.density_matrix(H2, S, n_e, method="purify", P_out=P_new, want_eps=False)
            g.density_matrix(H, S, n_e, method="eigen", P_out=P_new, want_eps=False)
            it["ms_lda_scf_iteration"], _ = timer.run(scf_iteration, 3, 1)
            it["E_H"] = float(EH.item())
            outside["hartree_fp64"] = it
            _log(f"hartree: {json.dumps({k: round(x, 3) for k, x in it.items()})}")
    if backward and inst.pt_wgrid is not None and not args.step_only:
        # total (moving-grid) forces: Pulay + partition-weight + nuclear-potential + point motion
        g.set_moving_grid()
        dR = torch.empty(inst.n_atoms, 3, dtype=torch.float64, device=dev)
        fsums = torch.empty(1, 3, dtype=torch.float64, device=dev)

        def forces():
            nonlocal dR
            dR, _ = g.total_forces(P, gE, prec="fp64", sums_out=fsums)
        outside["ms_total_forces_fp64"], _ = timer.run(forces, 3, 1)
        outside["total_forces_translation_residual"] = float(
            dR.sum(dim=0).abs().max() / dR.abs().max())
    line = {
        "metric": "H+density integration GFLOP/s and ms per SCF step (fastest form within 1e-6 Ha "
                  "of FP64; mixed forms reported beside it)" if not backward else
                  "density + backward (dE/dP, dE/dv, dE/dR) GFLOP/s and ms per step",
        "value": hr["gflops"], "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": hr["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[head],
        "data": "synthetic", "headline_form": head,
        "config": {"workload": WORKLOADS[args.workload], "n_points": inst.n_points,
                   "n_basis": inst.n_basis, "n_batches": ws["n_batches"], "flop_per_step": F,
                   "sum_np_nb2": ws["sum_np_nb2"], "parallelism": "single GPU"},
        "forms": {p: {k: r[k] for k in ("ms_per_step", "ms_per_step_median", "ms_per_step_min",
                                         "wall_ms_per_step", "gflops",
                                         "abs_dE_Ha_vs_fp64", "meets_1e-6_Ha", "rel_dN_vs_fp64",
                                         "tuning", "E", "N")}
                     | {"roofline": _roofline(r["kernels"], p, args.steps, args.workload, r["tuning"], F)}
                  for p, r in res.items()},
        "fastest_form": {"form": fastest, "ms_per_step": res[fastest]["ms_per_step"],
                         "gflops": res[fastest]["gflops"],
                         "speedup_vs_fp64": res["fp64"]["ms_per_step"] / res[fastest]["ms_per_step"]},
        "kernels": {p: r["kernels"] for p, r in res.items()},
        "autotuned": {p: (p not in fixed and not args.no_autotune) for p in forms},
        "outside_step": outside,
        "roofline": _roofline(hr["kernels"], head, args.steps, args.workload, hr["tuning"], F),
    }
    extras = [] if args.workload != "c2" or args.step_only else [x for x in args.extras.split(",") if x]
    if "c3" in extras:
        line["scale_c3"] = bench_scale_c3(args, torch, forms)
    if "c4" in extras:
        line["grouped_c4"] = bench_extra_c4(args, torch)
    if "c5" in extras:
        line["backward_c5"] = bench_extra_c5(args, torch, forms)
    if args.cpu_chunks > 0:
        _log("CPU baseline (oracle sample)...")
        cb = _cpu_baseline(inst, ws["flops_per_step"], args.cpu_chunks)
        if backward:
            cb["sample"] += " (forward step only)"
        line["cpu_baseline"] = cb
    return line


def bench_grouped(args, torch, mols):
    """c4: one grouped handle over every molecule, timed as a captured step graph and as eager
    calls, against 256 per-molecule handles (one launch set per molecule)."""
    from paper_2208_12335_amd import AimsGrid
    from paper_2208_12335_amd.autotune import autotune

    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(dev)
    t0 = time.time()
    g = AimsGrid(mols, device=0, stream=stream)
    ws = g.work_stats()
    F = ws["flops_per_step"]
    _log(f"grouped setup {time.time() - t0:.1f} s, {ws['n_batches']} batches, F = {F:.3e}")
    P = torch.cat([torch.from_numpy(m.P).reshape(-1) for m in mols]).to(dev)
    v = torch.cat([torch.from_numpy(m.v) for m in mols]).to(dev)
    n = torch.empty(g.n_points, dtype=torch.float64, device=dev)
    sums = torch.empty(len(mols), 3, dtype=torch.float64, device=dev)
    H = torch.empty(g.mat_elems, dtype=torch.float64, device=dev)
    timer = Timer(torch, stream)
    prec = "fp64"
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        if not args.no_autotune:
            r = autotune(g, P, v, prec=prec, reps=2, cache="")
            _log(f"autotuned {dict((k, r[k]) for k in ('h_merge', 'density_pblocks', 'persistent', 'h_flops_per_atomic', 'h_tile32_mask', 'density_bucket_pblocks'))}")

        def eager():
            g.update_density(P, v, prec=prec, n_out=n, sums_out=sums)
            g.integrate_h(v, prec=prec, H_out=H)

        ms_eager, wall_eager = timer.run(eager, args.steps, args.warmup)
        g.profile(True)
        timer.run(eager, args.steps, 0)
        kern = _kernels(g, args.steps)
        g.profile(False)
        E_eager = sums.cpu().numpy().copy()
        graph = g.step_graph(P, v, n, sums, H, prec=prec)
        ms_graph, wall_graph = timer.run(graph.launch, args.steps, args.warmup)
        E_graph = sums.cpu().numpy().copy()
    _log(f"grouped eager {ms_eager:.3f} ms, graph {ms_graph:.3f} ms")

    # per-molecule baseline: one handle and one launch set per molecule on the same stream.
    # Each handle sizes its own scratch to its molecule, and 256 such scratches at the default
    # budget would not fit HBM together, so the baseline handles take a bounded budget.
    singles = []
    tg = g.get_tuning(prec)
    scratch_env = os.environ.get("AIMS_SCRATCH_MB")
    os.environ["AIMS_SCRATCH_MB"] = str(SINGLE_SCRATCH_MB)
    for m in mols:
        gm = AimsGrid(m, device=0, stream=stream)
        gm.set_tuning(h_merge=tg["h_merge"], density_pblocks=tg["density_pblocks"], prec=prec,
                      h_flops_per_atomic=tg["h_flops_per_atomic"], h_tile32_mask=tg["h_tile32_mask"],
                      density_bucket_pblocks=tg["density_bucket_pblocks"])
        Pm = torch.from_numpy(m.P).to(dev).reshape(-1)
        vm = torch.from_numpy(m.v).to(dev)
        nm = torch.empty(gm.n_points, dtype=torch.float64, device=dev)
        sm = torch.empty(1, 3, dtype=torch.float64, device=dev)
        Hm = torch.empty(gm.mat_elems, dtype=torch.float64, device=dev)
        singles.append((gm, Pm, vm, nm, sm, Hm))
    torch.cuda.synchronize()

    def per_molecule():
        for gm, Pm, vm, nm, sm, Hm in singles:
            gm.update_density(Pm, vm, prec=prec, n_out=nm, sums_out=sm)
            gm.integrate_h(vm, prec=prec, H_out=Hm)

    with torch.cuda.stream(stream):
        ms_single, wall_single = timer.run(per_molecule, args.steps, args.warmup)
    if scratch_env is None:
        del os.environ["AIMS_SCRATCH_MB"]
    else:
        os.environ["AIMS_SCRATCH_MB"] = scratch_env
    E_single = np.stack([s[4].cpu().numpy()[0] for s in singles])
    _log(f"per-molecule {ms_single:.3f} ms (wall {wall_single:.3f} ms)")
    dE = float(np.max(np.abs((E_graph[:, 1] + E_graph[:, 2]) - (E_single[:, 1] + E_single[:, 2]))))
    nmol = len(mols)
    return {
        "metric": "grouped s.c.f. step throughput over 256 molecules (graph replay), molecules/s",
        "value": nmol / (ms_graph * 1e-3), "unit": "molecules/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_graph,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["c4"], "n_molecules": nmol, "n_points": g.n_points,
                   "n_basis_total": g.n_basis, "n_batches": ws["n_batches"], "flop_per_step": F,
                   "parallelism": "single GPU"},
        "gflops_graph": F / (ms_graph * 1e-3) / 1e9,
        "modes": {"graph": {"ms_per_step": ms_graph, "wall_ms_per_step": wall_graph},
                  "eager_grouped": {"ms_per_step": ms_eager, "wall_ms_per_step": wall_eager},
                  "per_molecule": {"ms_per_step": ms_single, "wall_ms_per_step": wall_single,
                                   "scratch_mb_per_handle": SINGLE_SCRATCH_MB,
                                   "molecules_per_s": nmol / (ms_single * 1e-3)}},
        "speedup_graph_vs_per_molecule": ms_single / ms_graph,
        "max_abs_dE_Ha_grouped_vs_per_molecule": dE,
        "max_abs_dE_Ha_graph_vs_eager": float(np.max(np.abs(E_graph - E_eager))),
        "tuning": tg, "kernels": {"fp64": kern},
        "roofline": _roofline(kern, "fp64", args.steps),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--forms", default="fp64,fp32,bf16x3,int8x7",
                    help="precision forms to time (fp64 is always included)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the library's default tuning instead of the autotuner's choice")
    ap.add_argument("--tuning", default="",
                    help='fixed tuning per form instead of the autotuner, as JSON, e.g. '
                         '\'{"fp64": {"h_merge": 1, "density_pblocks": 2, "persistent": 1}}\'')
    ap.add_argument("--cpu-chunks", type=int, default=120,
                    help="point chunks of the oracle's CPU baseline sample (0 = skip)")
    ap.add_argument("--step-only", action="store_true",
                    help="time the step alone: skip the measurements outside it (density matrix, "
                         "exchange-correlation, Hartree, total forces), e.g. for profiler runs")
    ap.add_argument("--extras", default="c3,c4,c5",
                    help="the other workloads the default (c2) line carries beside the headline: "
                         "c3 every form, c4 the grouped step (graph, eager, per molecule), c5 "
                         "every form with the backward; '' skips them")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 launches): the reference "
                         "kernel that scales the HBM byte counters of a profiler run")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the batches would shard across GPUs with one FP64 reduction of H)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 8, "copy_calibration_bytes_written": n * 8,
                          "launches": 3}), flush=True)
        return
    t0 = time.time()
    inst = _make(args.workload, torch)
    _log(f"instance {args.workload} ({time.time() - t0:.1f} s)")
    if args.workload == "c4":
        line = bench_grouped(args, torch, inst)
    else:
        line = bench_single(args, torch, inst, backward=(args.workload == "c5"))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
