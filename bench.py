"""Benchmark of the reciprocal-space SKP-PME path on one MI355X.

One step = one full reciprocal evaluation (bin + spread -> Kronecker operator
with correction -> gather of potentials and forces -> FP64 energies), inputs
resident in HBM, plan built beforehand (its creation time is reported
separately).  Default workload: the 1e6-atom water box (N = 1,000,002,
128^3 grid, p = 6, beta = 0.34, R from the 1e-6 Frobenius rule), the
configuration the precision metric is quoted on.

The mixed-precision path (FP16X3 by default) is timed, its error against the
FP64 GPU path at equal R is measured outside the timed region, the FP64 GPU
path is timed the same way for the speedup, and the BF16X3 split is measured
beside it (error and time).  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "reciprocal PME evals/sec & ns/particle at 1e-5 rel energy err: mixed-prec vs FP64"
PEAK_TFLOPS = {"fp16x3": 2500.0, "bf16x3": 2500.0, "fp32": 157.3, "fp64": 78.6}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default=None, choices=["fp16x3", "bf16x3", "fp32"],
                    help="mixed path: FP16X3 for the single-system workloads, the BF16 "
                         "split for the 64-system batch (the precision each is quoted in)")
    ap.add_argument("--workload", default="water_1m",
                    choices=["water_100k", "water_1m", "water_200k_noncubic", "lagrange_m10",
                             "batch64"])
    ap.add_argument("--skp-form", default="circulant", choices=["circulant", "rect"],
                    help="operator form: circulant factors on the matrix cores, or the "
                         "rectangular real cos/sin factors (FP64/FP32)")
    ap.add_argument("--skp-method", default="nested_svd", choices=["nested_svd", "sinc"],
                    help="Kronecker-term construction: nested SVD (Frobenius tail rule) or "
                         "the sinc quadrature (max-norm symbol tolerance)")
    ap.add_argument("--quad-tol", type=float, default=1e-6,
                    help="sinc quadrature: relative max-norm symbol tolerance")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-repeats", type=int, default=3,
                    help="repeats of the bounded CPU-oracle sample (median reported)")
    ap.add_argument("--no-bf16", action="store_true", help="skip the BF16X3 side measurement")
    ap.add_argument("--mixed-only", action="store_true",
                    help="time only the mixed path (short profiler runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run 5 device copies of MIB MiB and exit (byte-counter calibration)")
    ap.add_argument("--gemm-calibration", type=int, default=0, metavar="N",
                    help="time the vendor library's dense N x N x N FP16 and BF16 GEMM "
                         "(torch.matmul) and exit (the practical matrix-core rate)")
    a = ap.parse_args()
    if a.precision is None:
        a.precision = "bf16x3" if a.workload == "batch64" else "fp16x3"
    return a


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# what the split-precision stage-2 kernel is built from: its source text in
# skp_kernels.hip (from the section comment to the FP32/FP64 kernel's), the
# header that picks its instance (tiles, streams) and the device helpers it
# calls (fragments, splits, MFMA wrappers)
CSRC = os.path.join(ROOT, "paper_2601_18838_amd", "csrc")
STAGE2_SECTION = ("// Stage 2, split precision.", "// Stage 2, FP32 / FP64 with the 16x16x4 MFMAs.")
KERNELS_HPP_GRID_SECTION = "// Grid kernels: binning, spread and gather."
HBM_PEAK_GBS = 8000.0


def stage2_source_sha():
    """SHA-256 of the stage-2 kernel's source text and the headers it uses."""
    import hashlib
    text = open(os.path.join(CSRC, "skp_kernels.hip"), encoding="utf-8").read()
    a = text.index(STAGE2_SECTION[0])
    b = text.index(STAGE2_SECTION[1], a)
    h = hashlib.sha256(text[a:b].encode())
    # the SKP part of the launch header (its argument struct and LDS layout)
    hdr = open(os.path.join(CSRC, "kernels.hpp"), encoding="utf-8").read()
    h.update(hdr[:hdr.index(KERNELS_HPP_GRID_SECTION)].encode())
    h.update(open(os.path.join(CSRC, "device_common.hpp"), "rb").read())
    return h.hexdigest()


def committed_traffic(workload, precision, parts):
    """HBM bytes per stage-2 launch from the committed rocprofv3 counter summary
    for this workload (FETCH_SIZE and WRITE_SIZE, scaled by the copy-kernel
    calibration), or None when there is none, it is for another configuration,
    or the kernel's source has changed since the counters were taken."""
    summary = os.path.join(ROOT, "profiles", f"stage2_x3_{workload}_traffic.md")
    try:
        fields = {}
        for line in open(summary):
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].strip().split(": ", 1)
                fields[k] = v.strip("` ")
        sha = stage2_source_sha()
        if (fields.get("source_sha256") != sha or fields.get("workload") != workload
                or fields.get("precision") != precision or int(fields.get("stage2_parts", -1)) != parts):
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def copy_calibration(mib):
    """Five plain device-to-device copies of a known size, for scaling HBM byte counters."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 4, "bytes_written": n * 4,
                      "dispatches": 5}), flush=True)


def gemm_calibration(n, reps=20):
    """Dense square GEMMs through torch.matmul (the vendor BLAS) in FP16 and
    BF16: achieved TFLOP/s against the dense matrix-core peak, the rate a
    library GEMM sustains on this device."""
    import torch
    out = {"gemm_calibration_n": n, "peak_tflops": 2500.0}
    for name, dt in (("fp16", torch.float16), ("bf16", torch.bfloat16)):
        g = torch.Generator(device="cuda").manual_seed(0)
        a = torch.randn(n, n, device="cuda", dtype=dt, generator=g)
        b = torch.randn(n, n, device="cuda", dtype=dt, generator=g)
        for _ in range(3):
            c = a @ b
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            c = a @ b
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        tf = 2.0 * n ** 3 / us / 1e6
        out[name] = {"us": us, "tflops": tf, "frac": tf / 2500.0}
        del a, b, c
    print(json.dumps(out), flush=True)


def time_steps(plan, P, Q, out, steps, warmup):
    """Wall time per evaluation over `steps` back-to-back evaluations (no
    per-stage events in this region), then the per-stage breakdown from a
    second, event-instrumented pass of the same length."""
    import torch
    for _ in range(warmup):
        plan.evaluate(P, Q, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.evaluate(P, Q, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.profile(True)
    plan.profile_read()
    for _ in range(steps):
        plan.evaluate(P, Q, out=out)
    torch.cuda.synchronize()
    stages = plan.profile_read()
    plan.profile(False)
    return dt / steps, stages


def bench_batch(args):
    """64 independent +-1 systems in one replayed graph vs a per-system FP64 loop."""
    import torch
    from paper_2601_18838_amd import kpme, systems
    batch = systems.batch_systems(count=64)
    wls = [b[0] for b in batch]
    n = [w.n for w in wls]
    mixed = args.precision
    res = {}
    for prec in (mixed, "fp64"):
        dt = torch.float64 if prec == "fp64" else torch.float32
        pos = torch.tensor(np.concatenate([b[1] for b in batch]), dtype=dt, device="cuda")
        q = torch.tensor(np.concatenate([b[2] for b in batch]), dtype=dt, device="cuda")
        t0 = time.perf_counter()
        if prec == mixed:
            bp = kpme.BatchPlan([w.box for w in wls], [w.grid for w in wls],
                                [w.order for w in wls], [w.beta for w in wls],
                                [w.rank for w in wls], precision=prec, max_particles=n)
            # fixed output buffers: the graph is recorded once and replayed
            outs_b = (torch.empty((64, 4), dtype=torch.float64, device="cuda"),
                      torch.empty(sum(n), dtype=dt, device="cuda"),
                      torch.empty((sum(n), 3), dtype=dt, device="cuda"))
            run = lambda: bp.evaluate(n, pos, q, energy=outs_b[0], pot=outs_b[1],
                                      force=outs_b[2])
        else:
            plans = [kpme.Plan(w.box, w.grid, w.order, w.beta, rank=w.rank, precision=prec,
                               max_particles=w.n) for w in wls]
            offs = np.concatenate([[0], np.cumsum(n)])
            views = [(pos[offs[k]:offs[k + 1]], q[offs[k]:offs[k + 1]]) for k in range(64)]

            def run():
                return [pl.evaluate(*v) for pl, v in zip(plans, views)]
        t_plan = time.perf_counter() - t0
        for _ in range(args.warmup):
            out = run()
        torch.cuda.synchronize()
        steps = args.steps if prec == mixed else max(3, args.steps // 10)
        t0 = time.perf_counter()
        for _ in range(steps):
            out = run()
        torch.cuda.synchronize()
        res[prec] = ((time.perf_counter() - t0) / steps, t_plan, out)
    form, launches = bp.info()
    # the same batch recorded as every system's own launch sequence on
    # parallel graph branches (the library's other form), for comparison
    prev = os.environ.get("KPME_BATCH_FUSED")
    os.environ["KPME_BATCH_FUSED"] = "0"
    try:
        bp2 = kpme.BatchPlan([w.box for w in wls], [w.grid for w in wls], [w.order for w in wls],
                             [w.beta for w in wls], [w.rank for w in wls], precision=mixed,
                             max_particles=n)
    finally:
        if prev is None:
            del os.environ["KPME_BATCH_FUSED"]
        else:
            os.environ["KPME_BATCH_FUSED"] = prev
    dt = torch.float32
    pos = torch.tensor(np.concatenate([b[1] for b in batch]), dtype=dt, device="cuda")
    q = torch.tensor(np.concatenate([b[2] for b in batch]), dtype=dt, device="cuda")
    for _ in range(args.warmup):
        bp2.evaluate(n, pos, q, energy=outs_b[0], pot=outs_b[1], force=outs_b[2])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bp2.evaluate(n, pos, q, energy=outs_b[0], pot=outs_b[1], force=outs_b[2])
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / args.steps
    form2, launches2 = bp2.info()
    del bp2
    e_mixed = res[mixed][2][0][:, 0].cpu().numpy()
    e_ref = np.array([o[0][0].item() for o in res["fp64"][2]])
    rel = np.abs(e_mixed - e_ref) / np.abs(e_ref)
    t = res[mixed][0]
    # stage-2 flops of every system (issued: three products per split
    # product) over the whole batch time: a lower bound on the matrix cores'
    # use across the batch
    flops = sum(3.0 * 2.0 * (w.grid[0] * w.grid[1] * w.grid[2]) * w.rank * (w.grid[0] + w.grid[1])
                for w in wls)
    out = {"metric": "batched reciprocal PME: systems/s for 64 independent systems in one graph",
           "value": 64.0 / t, "unit": "systems/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": t * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": mixed, "data": "synthetic",
           "config": {"workload": "batch64_pm1", "systems": 64, "N_total": int(sum(n)),
                      "grids": sorted({str(w.grid) for w in wls}), "ranks": [6, 24]},
           "ns_per_particle": t * 1e9 / sum(n),
           "fp64_loop_ms": res["fp64"][0] * 1e3,
           "speedup_vs_fp64_loop": res["fp64"][0] / t,
           "max_rel_energy_err": float(rel.max()),
           "batched_form": {"form": {1: "one launch per stage and kernel instance",
                                     2: "persistent launches over a work queue"}.get(
                                         form, "per-system graph branches"),
                            "launches_per_batch": launches},
           "per_system_graph": {"ms_per_step": t_graph * 1e3, "launches_per_batch": launches2,
                                "form": form2},
           "speedup_vs_per_system_graph": t_graph / t,
           "roofline": {"bound": "mfma", "kernel": "all stage-2 flops over the batch time",
                        "achieved": flops / t / 1e12, "peak": PEAK_TFLOPS[mixed],
                        "unit": "TFLOP/s", "frac": flops / t / 1e12 / PEAK_TFLOPS[mixed],
                        "traffic": None, "flops_per_batch": flops},
           "plan_seconds": {mixed: res[mixed][1], "fp64": res["fp64"][1]}}
    print(json.dumps(out), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, pos, q, repeats):
    """The FP64 oracle on the host cores, on a bounded sample of the workload:
    the Kronecker operator applied once to a full grid, and spread + gather of
    a contiguous 1/32 of the particles (whole molecules), each repeated and
    the median taken; evals/s = 1 / (t_apply + 32 t_spread_gather)."""
    import statistics
    from oracle import skp, spme
    if wl.extra.get("interpolation") == "lagrange":
        from oracle import lagrange as lg
        cells = (wl.extra["cells"],) * 3
        pl = lg.Plan(wl.box, cells, wl.order, wl.extra["mode_cutoff"], wl.beta, tol=wl.tol)
        sp = lambda p_, q_: lg.spread(p_, q_, wl.box, cells, wl.order)
        ga = lambda p_, q_, g_: lg.gather(p_, q_, wl.box, cells, wl.order, g_)
    else:
        pl = skp.Plan(wl.box, wl.grid, wl.order, wl.beta, tol=wl.tol)
        sp = lambda p_, q_: spme.spread(p_, q_, wl.box, wl.grid, wl.order)
        ga = lambda p_, q_, g_: spme.gather(p_, q_, wl.box, wl.grid, wl.order, g_)
    frac = 32
    ns = (len(q) // frac) // 3 * 3
    t_sg, t_ap = [], []
    for _ in range(repeats):
        t0 = time.perf_counter()
        Qg = sp(pos[:ns], q[:ns])
        t1 = time.perf_counter()
        Phi = pl.apply(Qg)
        t2 = time.perf_counter()
        ga(pos[:ns], q[:ns], Phi)
        t3 = time.perf_counter()
        t_sg.append((t1 - t0) + (t3 - t2))
        t_ap.append(t2 - t1)
    per_eval = statistics.median(t_ap) + statistics.median(t_sg) * len(q) / ns
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / per_eval, "unit": "evals/s",
            "cores": min(threads, os.cpu_count() or 1), "kind": "oracle",
            "cpu_model": cpu_model(), "seconds_per_eval": per_eval,
            "sample": f"FP64 oracle on {wl.name} (R={pl.rank}): median of {repeats} runs of "
                      f"one Kronecker-operator application on the full grid plus spread and "
                      f"gather of {ns} of {len(q)} particles, the latter scaled by "
                      f"{len(q) / ns:.3f} (spread and gather are per-particle work)"}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the reciprocal path is a single-device "
              "library; multi-GPU sharding is a design note, not a run.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2601_18838_amd import kpme, systems
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gemm_calibration:
        gemm_calibration(args.gemm_calibration)
        return
    if args.workload == "batch64":
        bench_batch(args)
        return

    wl = {"water_100k": systems.WATER_100K, "water_1m": systems.WATER_1M,
          "water_200k_noncubic": systems.WATER_200K_NONCUBIC,
          "lagrange_m10": systems.LAGRANGE_M10}[args.workload]
    interp = dict(interpolation=wl.extra.get("interpolation", "bspline"),
                  mode_cutoff=wl.extra.get("mode_cutoff", 0), form=args.skp_form)
    pos, q = wl.particles()
    n = len(q)
    mixed, ref = args.precision, "fp64"
    side = [] if (args.no_bf16 or args.mixed_only or mixed == "bf16x3"
                  or args.skp_form == "rect") else ["bf16x3"]
    plans, tensors, outs, plan_s, tune_s = {}, {}, {}, {}, {}
    for prec in [mixed, ref] + side:
        dt = torch.float64 if prec == "fp64" else torch.float32
        t0 = time.perf_counter()
        if args.skp_method == "sinc":
            plans[prec] = kpme.Plan(wl.box, wl.grid, wl.order, wl.beta, rank=0,
                                    tol=args.quad_tol, precision=prec, max_particles=n,
                                    method="sinc", **interp)
        else:
            plans[prec] = kpme.Plan(wl.box, wl.grid, wl.order, wl.beta, rank=wl.rank,
                                    tol=wl.tol, precision=prec, max_particles=n, **interp)
        plan_s[prec] = time.perf_counter() - t0
        t0 = time.perf_counter()
        plans[prec].autotune()          # the library's work-split tuner
        tune_s[prec] = time.perf_counter() - t0
        log(f"{prec} plan {plan_s[prec]:.1f} s, autotune {tune_s[prec]:.1f} s")
        tensors[prec] = (torch.tensor(pos, dtype=dt, device="cuda"),
                         torch.tensor(q, dtype=dt, device="cuda"))
        outs[prec] = (torch.empty(4, dtype=torch.float64, device="cuda"),
                      torch.empty(n, dtype=dt, device="cuda"),
                      torch.empty((n, 3), dtype=dt, device="cuda"))
    info = plans[mixed].info
    # accuracy of the mixed paths against the FP64 GPU path at equal R
    res = {}
    for prec in [mixed, ref] + side:
        e4, pot, frc = plans[prec].evaluate(*tensors[prec], out=outs[prec])
        torch.cuda.synchronize()
        res[prec] = (e4.cpu().numpy().copy(), pot.double().cpu().numpy(),
                     frc.double().cpu().numpy())
    rms = lambda a, b: float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))

    def errors(prec):
        return (abs(res[prec][0][0] - res[ref][0][0]) / abs(res[ref][0][0]),
                rms(res[prec][1], res[ref][1]), rms(res[prec][2], res[ref][2]))

    rel_e, rms_phi, rms_f = errors(mixed)

    log(f"{mixed} relE {rel_e:.2e} rmsF {rms_f:.2e}; timing")
    t_mixed, st_mixed = time_steps(plans[mixed], *tensors[mixed], outs[mixed], args.steps,
                                   args.warmup)
    log(f"{mixed} {1.0 / t_mixed:.1f} evals/s")
    if args.mixed_only:
        t_ref, st_ref = float("nan"), {k: (float("nan"), 1) for k in st_mixed}
    else:
        t_ref, st_ref = time_steps(plans[ref], *tensors[ref], outs[ref],
                                   max(5, args.steps // 5), min(args.warmup, 2))
    side_out = {}
    for prec in side:
        t_s, _ = time_steps(plans[prec], *tensors[prec], outs[prec], max(5, args.steps // 5),
                            min(args.warmup, 2))
        e_s, p_s, f_s = errors(prec)
        side_out[prec] = {"evals_per_s": 1.0 / t_s, "ns_per_particle": t_s * 1e9 / n,
                          "rel_energy_err": e_s, "rel_rms_potential_err": p_s,
                          "rel_rms_force_err": f_s,
                          "accuracy_target_met": bool(e_s <= 1e-5 and f_s <= 1e-4)}

    K1, K2, K3 = wl.grid
    G = K1 * K2 * K3
    R = info["rank"]
    if args.skp_form == "rect":
        # rectangular form: three thin products into the real mode basis and
        # three back (the "stage 2" timer covers all six and the scaling);
        # n_j = min(2 M_j + 1, K_j) rows, M_j the mode cutoff (K_j / 2 for
        # the full B-spline symbol)
        cut = wl.extra.get("mode_cutoff", 0)
        nr = [min(2 * (cut if cut else k // 2) + 1, k) for k in wl.grid]
        flops_s2 = 2.0 * 2.0 * (nr[2] * K1 * K2 * K3 + nr[1] * nr[2] * K1 * K2
                                + nr[0] * nr[1] * nr[2] * K1)
    else:
        flops_s2 = 2.0 * G * R * (K1 + K2)              # grouped stage-2, one product
    issued = 3.0 * flops_s2 if mixed.endswith("x3") else flops_s2
    ms_s2, cnt_s2 = st_mixed["skp_stage2"]
    avg_s2 = ms_s2 / max(cnt_s2, 1) * 1e-3
    achieved = issued / avg_s2 / 1e12
    peak = PEAK_TFLOPS[mixed]
    stage_us = {k: (v[0] / max(v[1], 1) * 1e3) for k, v in st_mixed.items()}
    stage_us_fp64 = {k: (v[0] / max(v[1], 1) * 1e3) for k, v in st_ref.items()}

    # HBM rooflines of the particle-grid stages from their algorithmic bytes
    # (FP32 values): the spread (binning included) reads positions and charges
    # (16 B per particle) and writes the grid once (4 B per point); the gather
    # reads positions, charges and the grid once and writes potential and
    # force (16 B per particle)
    def hbm(bytes_, us):
        gbs = bytes_ / (us * 1e-6) / 1e9
        return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "algorithmic_bytes": bytes_, "us": us}
    spread_bytes = 16.0 * n + 4.0 * G
    gather_bytes = 16.0 * n + 4.0 * G + 16.0 * n

    out = {
        "metric": METRIC,
        "value": 1.0 / t_mixed,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mixed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": mixed,
        "data": "synthetic",
        "config": {"workload": wl.name, "N": n, "grid": list(wl.grid), "order": wl.order,
                   "beta": wl.beta, "box": list(wl.box), "rank": R, "r0": info["r0"],
                   "skp_method": args.skp_method, "skp_form": args.skp_form,
                   "interpolation": interp["interpolation"],
                   "mode_cutoff": interp["mode_cutoff"],
                   "rank_rule": (f"relative Frobenius tail <= {wl.tol:g}"
                                 if args.skp_method == "nested_svd" else
                                 f"sinc rule N={info['quad_N']}, h={info['quad_h']:.6g}: "
                                 f"max-norm symbol error {info['sym_err']:.3g} <= "
                                 f"{args.quad_tol:g}"),
                   "precision": mixed, "reference": "fp64 GPU path at equal R",
                   "stage2_parts": plans[mixed].stage2_parts(),
                   "stage1_split": plans[mixed].stage1_split(),
                   "stage2_streams": plans[mixed].stage2_streams()},
        "ns_per_particle": t_mixed * 1e9 / n,
        "fp64_evals_per_s": 1.0 / t_ref,
        "fp64_ns_per_particle": t_ref * 1e9 / n,
        "speedup_vs_fp64": t_ref / t_mixed,
        "rel_energy_err": rel_e,
        "rel_rms_potential_err": rms_phi,
        "rel_rms_force_err": rms_f,
        "accuracy_target_met": bool(rel_e <= 1e-5 and rms_f <= 1e-4),
        "E_rec": float(res[ref][0][0]),
        "plan_seconds": plan_s,
        "autotune_seconds": tune_s,
        "stage_us": stage_us,
        "stage_us_fp64": stage_us_fp64,
        "roofline": {"bound": "mfma",
                     "kernel": "skp_stage2" if args.skp_form != "rect" else "rect_apply",
                     "achieved": achieved,
                     "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": committed_traffic(wl.name, mixed, plans[mixed].stage2_parts()),
                     "flops_per_launch": issued,
                     "effective_single_product_tflops": flops_s2 / avg_s2 / 1e12},
        "roofline_spread": hbm(spread_bytes, stage_us["spread"]),
        "roofline_gather": hbm(gather_bytes, stage_us["gather"]),
    }
    for prec, v in side_out.items():
        out[prec] = v
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(wl, pos, q, args.cpu_repeats)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
