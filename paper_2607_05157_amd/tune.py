"""Launch-shape tuner for the multi-RHS operator kernel.

Times wdt_apply_D over a grid of launch shapes (RHS tile, sites per block,
blocks per tile, z-slab, tile order, t-march chunk, brick order, one site per
wavefront) for one lattice, batch size and precision, and reports the
algorithmic bandwidth of each (bytes: every input spinor read once, every
output written once, the links once per launch).  Also times a plain device
copy of the same size as a bandwidth reference.

    python -m paper_2607_05157_amd.tune --dims 16 16 16 32 --nrhs 48 --prec fp64 fp16 \
        --out tune.json
"""
import argparse
import itertools
import json
import sys

import numpy as np

if __name__ == "__main__":
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

SITE_BYTES = {0: 192, 1: 96, 2: 52, 3: 48}
LINK_BYTES = {0: 144, 1: 72, 2: 72, 3: 72}  # FP32 links (also BF16); FP16: two packed halves


def alg_bytes(V, N, prec):
    return V * (N * 2 * SITE_BYTES[prec] + 4 * LINK_BYTES[prec])


def time_apply(W, g, lat, x, y, N, prec, reps, torch):
    # warm-up: the first launches of a shape run on a cold GPU (clocks, caches)
    for _ in range(max(3, reps // 2)):
        W.apply_D(g, 0.02, x, y, N, prec)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        W.apply_D(g, 0.02, x, y, N, prec)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def copy_gbps(nbytes, torch, reps=10):
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return 2 * a.numel() * 4 / (ms * 1e-3) / 1e9


def main(argv=None):
    import torch
    from synth.gauge import gauge_field
    from paper_2607_05157_amd import wdt as W

    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", type=int, nargs=4, default=[16, 16, 16, 32])
    ap.add_argument("--nrhs", type=int, default=48)
    ap.add_argument("--prec", nargs="+", default=["fp64", "fp16"])
    ap.add_argument("--tiles", type=int, nargs="+", default=[0, 8, 16, 24, 48])
    ap.add_argument("--sb", type=int, nargs="+", default=[0])
    ap.add_argument("--gmax", type=int, nargs="+", default=[0, 1024, 4096])
    ap.add_argument("--bz", type=int, nargs="+", default=[0])
    ap.add_argument("--serial", type=int, nargs="+", default=[-1],
                    help="operator blocks sweep RHS tiles in turn: 1 on, 0 off, -1 automatic")
    ap.add_argument("--tchunk", type=int, nargs="+", default=[-1],
                    help="operator marches along t in chunks of this many slices (0 off)")
    ap.add_argument("--wps", type=int, nargs="+", default=[-1],
                    help="operator: one site per wavefront (1 on, 0 off, -1 automatic)")
    ap.add_argument("--brick", nargs="+", default=["auto"],
                    help="site-sweep brick order: x,y,z extents, 'auto' or 'off'")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)

    W.init(0)
    dims, N = tuple(a.dims), a.nrhs
    V = int(np.prod(dims))
    U = gauge_field(dims, 0.5, seed=2)
    lat = W.Lattice(dims, -1)
    g = W.Gauge(lat, U)
    results = []
    ref = copy_gbps(lat.spinor_bytes(N, W.FP64), torch)
    print(json.dumps({"copy_gbps": round(ref, 1), "bytes": lat.spinor_bytes(N, W.FP64)}), flush=True)
    for pname in a.prec:
        prec = W.PREC[pname]
        x = torch.zeros(lat.spinor_bytes(N, prec), dtype=torch.uint8, device="cuda")
        if prec == W.FP64:
            x = torch.randn((V, 12, N), dtype=torch.complex128, device="cuda")
        elif prec == W.FP32:
            x = torch.randn((V, 12, N), dtype=torch.complex64, device="cuda")
        else:
            # FP16 batch: random halves in [-1, 1] and unit scales
            h = torch.rand(V * 12 * N * 2, device="cuda", dtype=torch.float32) * 2 - 1
            s = torch.ones(V * N, device="cuda", dtype=torch.float32)
            x = torch.cat([h.half().view(torch.uint8), s.view(torch.uint8)])
        y = torch.zeros_like(x)
        bricks = [(0, 0, 0) if b == "auto" else (-1, -1, -1) if b == "off"
                  else tuple(int(v) for v in b.split(",")) for b in a.brick]
        for nt, sb, gm, bz, se, tc, br, wp in itertools.product(
                a.tiles, a.sb, a.gmax, a.bz, a.serial, a.tchunk, bricks, a.wps):
            W.set_launch_shape(nt, sb, gm, bz, se, tc, br, wp)
            ms = time_apply(W, g, lat, x, y, N, prec, a.reps, torch)
            gbps = alg_bytes(V, N, prec) / (ms * 1e-3) / 1e9
            r = dict(prec=pname, rhs_tile=nt, sites_per_block=sb, max_blocks=gm, z_slab=bz,
                     serial=se, tchunk=tc, brick=list(br), wps=wp, ms=round(ms, 4),
                     gbps=round(gbps, 1))
            results.append(r)
            print(json.dumps(r), flush=True)
        W.set_launch_shape()
    best = {}
    for r in results:
        if r["prec"] not in best or r["gbps"] > best[r["prec"]]["gbps"]:
            best[r["prec"]] = r
    summary = dict(dims=list(dims), nrhs=N, copy_gbps=ref, best=best, results=results)
    print(json.dumps({"best": best}), flush=True)
    if a.out:
        json.dump(summary, open(a.out, "w"), indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
