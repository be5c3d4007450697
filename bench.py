#!/usr/bin/env python3
"""Benchmark of the disconnected-loop trace estimator on one MI355X.

Workload (default): 16^3 x 32 lattice, link spread eps = 0.5, m0 = 0.02,
antiperiodic in time; distance-2 torus colouring of the 4D lattice (16
colours, sigma = (1,2,3,4)) x time dilution on t0 = 0 x 12-fold spin-colour
dilution x 4 Rademacher seeds.  One step = one colour batch of 48 right-hand
sides through the whole hot path: source generation, batched solve to a true
relative residual of 1e-10 (FP16-storage / FP32-arithmetic BiCGStab inside
FP64 defect correction), and the gamma5 contraction on t0.  Inputs are
synthetic and resident in HBM before timing starts.

Reported (one JSON line):
  value     algorithmic HBM GB/s of the Wilson-Dirac operator kernels over the
            timed steps (bytes: each input spinor read once, each output
            written once, links once per launch; time: HIP events on the
            library's stream around every launch);
  roofline  the same for the dominant operator kernel against 8 TB/s;
  seconds per trace (all colour batches) for the mixed path and for the
  FP64 path on the same lattice, and the oracle timed on this host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0

# HBM bytes per operator dispatch on this workload, from two rocprofv3 counter
# runs (FETCH_SIZE, then WRITE_SIZE, averaged over the dispatches of each
# precision); FETCH_SIZE is scaled by 2 and WRITE_SIZE by 1, the factors that
# turn the counters of a device copy of known size into its true byte count.
# They describe the sources they were taken on and are reported only while
# those sources are unchanged.
OPERATOR_SOURCES = ["kernels.h", "device.h", "dslash.hip", "solver.hip", "internal.h"]
MEASURED_TRAFFIC = {"sources": "213ac8bfed7bcde1",
                    "dslash_eo_fp16": 1047.0e6, "dslash_hop_fp16": 841.7e6}


def operator_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in OPERATOR_SOURCES:
        with open(os.path.join(ROOT, "paper_2607_05157_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def stream_copy_gbps(nbytes, reps=10):
    """Device-to-device copy of nbytes (read + write counted): what a plain
    streaming kernel reaches on this GPU."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    return 2 * a.numel() * 4 / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9


def cpu_baseline(U, m0, dims, b_host, n_rhs):
    """The oracle's operator (scipy CSR assembled from the definition, then a
    sparse product) applied to the whole batch, timed on this host."""
    import numpy as np
    from oracle import dirac
    t = time.perf_counter()
    dirac.apply_D(U, m0, b_host, dims, -1)
    dt = time.perf_counter() - t
    V = int(np.prod(dims))
    alg = V * (n_rhs * 2 * 192 + 4 * 144)
    return dict(value=alg / dt / 1e9, unit="GB/s", cores=1, kind="oracle",
                sample=f"one application of the oracle's D (CSR assembly + product) to the "
                       f"{n_rhs}-RHS FP64 batch on {dims}, {dt:.1f} s; scipy's sparse product "
                       f"runs on one thread (host has {len(os.sched_getaffinity(0))} cores)")


def batched_leg(log, n_per_shape=32):
    """The uneven workload: 8^4, 8^3x16 and 12^3x24 instances (n_per_shape
    each) with seeded eps, m0 and 16..48 Rademacher RHS, FP64 to 1e-10, solved
    as one graph-replayed batch (after a short plan tuning) and as one solve
    per system."""
    import torch
    from synth.gauge import gauge_field
    from synth.workloads import batched_instances
    from paper_2607_05157_amd import wdt
    inst = batched_instances(n_per_shape=n_per_shape)
    systems = []
    for i in inst:
        lat = wdt.Lattice(i["dims"], -1)
        g = wdt.Gauge(lat, gauge_field(i["dims"], i["eps"], i["gauge_seed"]))
        b = lat.new_batch(i["n_rhs"])
        wdt.sources(lat, wdt.source_descs([i["noise_seed_base"] + k for k in range(i["n_rhs"])]), b)
        systems.append(dict(lat=lat, g=g, b=b, x=lat.new_batch(i["n_rhs"]), m0=i["m0"], N=i["n_rhs"]))
    log("batched leg:", len(systems), "systems")
    B = wdt.Batch([s["g"] for s in systems], [s["m0"] for s in systems], [s["N"] for s in systems])
    untuned = B.info()
    ms_it = B.tune(iters=3)
    plan = B.info()
    B.solve([s["b"] for s in systems], [s["x"] for s in systems], tol=1e-10)   # warm
    torch.cuda.synchronize()
    t = time.perf_counter()
    rc, st = B.solve([s["b"] for s in systems], [s["x"] for s in systems], tol=1e-10)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t
    del B
    for s in systems[:3]:
        wdt.solve(s["g"], s["m0"], s["b"], s["x"], s["N"], tol=1e-10)      # warm
    torch.cuda.synchronize()
    t = time.perf_counter()
    st1 = []
    for s in systems:
        _, stt = wdt.solve(s["g"], s["m0"], s["b"], s["x"], s["N"], tol=1e-10)
        st1.extend(stt)
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t
    return {"systems": len(systems), "total_rhs": sum(s["N"] for s in systems),
            "seconds_batched_graph": round(t_batched, 4),
            "seconds_one_solve_per_system": round(t_single, 4),
            "speedup": round(t_single / t_batched, 3),
            "tuned_plan": plan, "untuned_plan": untuned, "tuned_ms_per_iteration": round(ms_it, 4),
            "max_true_residual_batched": max(x["true_residual"] for x in st),
            "max_true_residual_single": max(x["true_residual"] for x in st1),
            "iterations_max": max(x["iterations"] for x in st),
            "iterations_mean_single": round(sum(x["iterations"] for x in st1) / len(st1), 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--bf16-steps", type=int, default=2)
    ap.add_argument("--clover-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--inner-tol", type=float, default=0.003)
    ap.add_argument("--no-batched", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the trace estimate "
              "shards by colour batch with no communication", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from synth.gauge import gauge_field
    from synth.workloads import workload
    from paper_2607_05157_amd import wdt

    cfg = workload("loop_16c32_d2")
    dims, m0, N, t0 = cfg["dims"], cfg["m0"], cfg["n_rhs"], cfg["t0"]
    seeds = cfg["noise_seeds"]
    wdt.init(0)
    log("gauge field", dims)
    U = gauge_field(dims, cfg["eps"], cfg["gauge_seed"])
    lat = wdt.Lattice(dims, cfg["bc_t"])
    g = wdt.Gauge(lat, U)
    n_c, sigma = wdt.colouring_search(dims, cfg["colouring_d"])
    # colours present on the source slice t0 (time dilution keeps only those)
    Lx, Ly, Lz = dims[:3]
    xs = np.indices((Lx, Ly, Lz)).reshape(3, -1)
    present = sorted(set(int(v) for v in (np.array(sigma[:3]) @ xs + sigma[3] * t0) % n_c))
    G5 = np.diag([1, 1, -1, -1]).astype(complex)

    def descs(j):
        sd = [s for s in seeds for _ in range(12)]
        comp = [k for _ in seeds for k in range(12)]
        return wdt.source_descs(sd, n_c=n_c, colour=j, sigma=sigma, component=comp, t0=t0)

    b = lat.new_batch(N)
    x = lat.new_batch(N)

    def step(j, prec):
        wdt.sources(lat, descs(j), b)
        rc, st = wdt.solve(g, m0, b, x, N, tol=cfg["tol"], prec=prec, inner_tol=args.inner_tol,
                           max_iter=20000, max_outer=60, check_every=10)
        loop = wdt.contract(lat, b, x, N, spin=G5)[:, t0]
        return st, loop

    log("warmup", args.warmup)
    for w in range(args.warmup):
        step(present[w % len(present)], wdt.FP16)
    torch.cuda.synchronize()

    log("timed mixed steps", args.steps)
    wdt.profile(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    stats = []
    step_ms = []
    for k in range(args.steps):
        ts = time.perf_counter()
        st, loop = step(present[k % len(present)], wdt.FP16)   # ends with a host read-back
        step_ms.append((time.perf_counter() - ts) * 1e3)
        stats.append(st)
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t_start) / args.steps
    prof = wdt.profile_read()
    wdt.profile(False)

    # the same steps with BF16 storage (inner tolerance 0.05: BF16 keeps 8
    # mantissa bits), for the record
    t_bf16 = None
    if args.bf16_steps > 0:
        log("bf16 steps", args.bf16_steps, "after one warm-up step")
        for k in range(args.bf16_steps + 1):
            if k == 1:
                torch.cuda.synchronize()
                t0_ = time.perf_counter()
            wdt.sources(lat, descs(present[k % len(present)]), b)
            wdt.solve(g, m0, b, x, N, tol=cfg["tol"], prec=wdt.BF16, inner_tol=0.05,
                      max_iter=20000, max_outer=60)
            wdt.contract(lat, b, x, N, spin=G5)
        torch.cuda.synchronize()
        t_bf16 = (time.perf_counter() - t0_) / args.bf16_steps

    # the same steps with the clover term (c_sw = 1, its tree-level value) on
    # the operator, for the record
    t_clov, clov = None, None
    if args.clover_steps > 0:
        log("clover steps", args.clover_steps, "after one warm-up step")
        gc = wdt.Gauge(lat, U)
        gc.set_clover(1.0)
        its = []
        for k in range(args.clover_steps + 1):
            if k == 1:
                torch.cuda.synchronize()
                wdt.profile(True)
                t0_ = time.perf_counter()
            wdt.sources(lat, descs(present[k % len(present)]), b)
            rc_, st_ = wdt.solve(gc, m0, b, x, N, tol=cfg["tol"], prec=wdt.FP16,
                                 inner_tol=args.inner_tol, max_iter=20000, max_outer=60)
            wdt.contract(lat, b, x, N, spin=G5)
            if k >= 1:
                its += [s_["iterations"] for s_ in st_]
        torch.cuda.synchronize()
        t_clov = (time.perf_counter() - t0_) / args.clover_steps
        pc = wdt.profile_read()
        wdt.profile(False)
        del gc
        clov = {"csw": 1.0, "iterations_max": max(its),
                "kernels": {k: {"calls": v["calls"], "ms": round(v["ms"], 3),
                                "gbps": round(v["gbps"], 1)}
                            for k, v in pc.items() if k.startswith("dslash")}}

    log("fp64 steps", args.fp64_steps)
    torch.cuda.synchronize()
    t0_ = time.perf_counter()
    wdt.profile(True)
    st64 = []
    for k in range(args.fp64_steps):
        st, _ = step(present[k % len(present)], wdt.FP64)
        st64.append(st)
    torch.cuda.synchronize()
    t_fp64 = (time.perf_counter() - t0_) / max(1, args.fp64_steps)
    prof64 = wdt.profile_read()
    wdt.profile(False)

    dsl = {k: v for k, v in prof.items() if k.startswith("dslash")}
    tot_b = sum(v["bytes"] for v in dsl.values())
    tot_ms = sum(v["ms"] for v in dsl.values())
    value = tot_b / (tot_ms * 1e-3) / 1e9
    dom = max(dsl, key=lambda k: dsl[k]["ms"])
    d = dsl[dom]
    per_launch_b = d["bytes"] / d["calls"]
    per_launch_ms = d["ms"] / d["calls"]
    achieved = per_launch_b / (per_launch_ms * 1e-3) / 1e9
    traffic = (MEASURED_TRAFFIC.get(dom)
               if operator_sources_hash() == MEASURED_TRAFFIC["sources"] else None)
    d64 = None
    dsl64 = [v for k, v in prof64.items() if k.startswith("dslash")]
    if dsl64:
        d64 = {"gbps": sum(v["bytes"] for v in dsl64) / (sum(v["ms"] for v in dsl64) * 1e-3) / 1e9}
    max_res = max(s["true_residual"] for st in stats for s in st)
    iters = [s["iterations"] for st in stats for s in st]
    outer = [s["outer"] for st in stats for s in st]

    stream = stream_copy_gbps(b.numel() * b.element_size())
    batched = None
    if not args.no_batched:
        batched = batched_leg(log)

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(U, m0, dims, b.cpu().numpy(), N)

    out = {
        "metric": "Dslash HBM GB/s (% peak); mixed vs FP64 GPU seconds per trace at 1e-10 residual",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_mixed * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16-storage/f32-arith operator inside f64 refinement",
        "data": "synthetic",
        "config": {"workload": "disconnected loop tr[gamma5 D^-1(t0,t0)], 16^3x32, eps=0.5, "
                               "m0=0.02, 4D torus colouring d=2 x time dilution x Dil12 x 4 seeds",
                   "dims": list(dims), "n_rhs_per_batch": N, "n_colours": n_c,
                   "sigma": list(sigma), "colour_batches_per_trace": len(present),
                   "tol": cfg["tol"], "inner_tol": args.inner_tol},
        "pct_of_hbm_peak": round(100 * value / HBM_PEAK_GBPS, 1),
        "stream_copy_gbps": round(stream, 1),
        "pct_of_stream": round(100 * value / stream, 1),
        "step_ms": [round(v, 2) for v in step_ms],
        "median_step_ms": round(sorted(step_ms)[len(step_ms) // 2], 3),
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "bytes_per_launch": per_launch_b, "avg_launch_ms": per_launch_ms,
                     "traffic": traffic,
                     "traffic_over_algorithmic": round(traffic / per_launch_b, 3) if traffic else None},
        "seconds_per_trace": {"mixed": round(t_mixed * len(present), 3),
                              "mixed_bf16_storage": (round(t_bf16 * len(present), 3)
                                                     if t_bf16 else None),
                              "mixed_clover": (round(t_clov * len(present), 3)
                                               if t_clov else None),
                              "fp64": round(t_fp64 * len(present), 3) if st64 else None,
                              "speedup_mixed_vs_fp64": round(t_fp64 / t_mixed, 3) if st64 else None},
        "fp64_dslash_gbps": round(d64["gbps"], 1) if d64 else None,
        "clover_operator": clov,
        "kernels_mixed": {k: {"calls": v["calls"], "ms": round(v["ms"], 3),
                              "gbps": round(v["gbps"], 1)} for k, v in prof.items()},
        "kernels_fp64": {k: {"calls": v["calls"], "ms": round(v["ms"], 3),
                             "gbps": round(v["gbps"], 1)} for k, v in prof64.items()},
        "solver": {"max_true_residual": max_res, "iterations_max": max(iters),
                   "outer_max": max(outer),
                   "fp64_iterations_max": max((s["iterations"] for st in st64 for s in st),
                                              default=None)},
        "batched_uneven_workload": batched,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
