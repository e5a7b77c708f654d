"""Benchmark: zone-cycles/s of the full RK3-IMEX GRRMHD step on one MI355X.

Workload: 3-D Kerr-Schild accretion-shaped grid, spin 0.9375, 128x64x32
interior cells (log r in [1.2, 40], theta in (0, pi), phi periodic), FP64,
LAXF fluxes, MC reconstruction, flux-CT, implicit 4-force per cell; inputs
are synthetic and seeded (paper_1312_6127_amd.inputs.accretion_disk).

Prints one JSON line.  value = interior cells x steps / wall time of the K
timed steps (HIP events on the step's stream, inputs resident in HBM).
roofline: the dominant kernel (the per-cell implicit solve), its average
launch time measured with HIP events on its stream.  cpu_baseline: the FP64
oracle stepping the same workload on the host cores (bounded sample).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector peak
HBM_PEAK_GBS = 8000.0        # MI355X HBM3E peak
# Algorithmic state bytes of one zone-cycle of the FP64 step: stage 1 reads
# P^n, U^n and writes U^(1), P^(1); stages 2 and 3 also read U^n (12 doubles
# each array): (4 + 5 + 5) x 96 B.
STEP_BYTES_PER_ZONE = 1344

# Counter figures of the implicit kernel on this workload, from rocprofv3
# --pmc runs of this script (profiles/k_implicit_disk128x64x32_counters.md):
# FP64 flops per lane slot of a Newton trip (64 x (ADD + MUL + TRANS +
# 2 FMA) wave instructions over the lane slots), and HBM bytes per launch
# (FETCH_SIZE x 2 + WRITE_SIZE x 1, the scales from a copy of known size).
# They hold for the kernel sources whose digest is KERNEL_DIGEST; otherwise
# traffic is reported as null and the flop figure as stale.
FLOPS_PER_TRIP = 3009.0
HBM_BYTES_PER_LAUNCH = 121.7e6
KERNEL_DIGEST = "310e16509b82f1b2"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, nargs=3, default=[128, 64, 32])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also copy a buffer of this many MiB (counter calibration)")
    ap.add_argument("--batch-cells", type=int, default=0,
                    help="also time the batched implicit solve on this many independent cells "
                         "in each execution form (16777216 for the 16.7M-cell batch)")
    ap.add_argument("--batch-only", action="store_true",
                    help="time only the batched implicit solve")
    return ap.parse_args()


def kernel_digest():
    """sha256 over the HIP sources of the implicit kernel."""
    import hashlib

    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1312_6127_amd", "csrc")
    for f in ("dual.h", "common.h", "physics.h", "invert.h", "implicit.h", "kernels.h"):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _factor3(n):
    """A near-cubic (nx, ny, nz) with nx*ny*nz == n (powers of two split evenly)."""
    best = (n, 1, 1)
    for nz in range(1, int(round(n ** (1 / 3))) + 2):
        if n % nz:
            continue
        m = n // nz
        for ny in range(nz, int(m ** 0.5) + 2):
            if m % ny == 0 and m // ny >= ny and max(m // ny, ny, nz) < max(best):
                best = (m // ny, ny, nz)
    return best


def batch_inputs(G, I, torch, dev, n, seed=11):
    """Seeded batch (inputs.implicit_batch) with its explicit state: the
    primitives' conserved form from the library's own prim_to_cons on a flat
    grid holding the cells, the radiation energy raised 30% and the gas
    energy lowered to match, so every cell starts out of equilibrium."""
    pd, P, dt, ca, ce = I.implicit_batch(n, seed=seed)
    shape = _factor3(n)
    gd = dict(pd, n=shape)
    g = G.Grid(gd)
    na = I.nalloc(gd)
    Pf = torch.zeros((12, g.N), dtype=torch.float64, device=dev)
    inner = I.interior(gd)
    Pv = Pf.view(12, *na[::-1])
    Pt = torch.tensor(P, device=dev)
    Pv[(slice(None),) + inner] = Pt.view(12, *shape[::-1])
    Uf = g.prim_to_cons(Pf)
    U = Uf.view(12, *na[::-1])[(slice(None),) + inner].reshape(12, n).contiguous()
    g.close()
    del Pf, Uf
    Ui = U.clone()
    Ui[8] *= 1.3
    Ui[1] -= 0.3 * U[8]
    return pd, [Ui, Pt, torch.tensor(dt, device=dev), torch.tensor(ca, device=dev),
                torch.tensor(ce, device=dev)]


def bench_batch(G, I, torch, dev, n, reps=3):
    """Cell-solves/s of the batched implicit solve in each execution form,
    with the active-lane fraction of the first PMHD attempts."""
    pd, args = batch_inputs(G, I, torch, dev, n)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    tune, allt, outs = G.autotune_implicit_source(pd, *args)
    st = outs[3].cpu().numpy()
    its = outs[2].cpu().numpy()
    res = {"cells": n, "tol_pmhd": pd["tol_pmhd"],
           "failed_frac": float(((st & G.ST_FAIL) != 0).mean()),
           "urad_frac": float(((st & G.ST_URAD) != 0).mean()),
           "mean_iters": float(its.mean()), "max_iters": int(its.max()),
           "autotune": [{"form": G.FORM_NAMES[a.mode], "block": a.block,
                         "waves_per_cu": a.waves_per_cu, "ms": a.ms} for a in allt],
           "autotuned": {"form": G.FORM_NAMES[tune.mode], "block": tune.block,
                         "waves_per_cu": tune.waves_per_cu}, "forms": {}}
    pers = min((a for a in allt if a.mode == G.PERSISTENT), key=lambda a: a.ms)
    forms = [("per_cell", G.PER_CELL, 64, 1), ("per_iteration", G.PER_ITERATION, 64, 1),
             ("persistent", G.PERSISTENT, pers.block, pers.waves_per_cu)]
    for name, mode, block, wpc in forms:
        ws = G.batch_workspace(n, mode)
        out = G._batch_out(args[0], args[1])
        G.implicit_source_ex(pd, *args, mode, block, wpc, out=out, ws=ws)
        e0.record(stream)
        for _ in range(reps):
            G.implicit_source_ex(pd, *args, mode, block, wpc, out=out, ws=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        trips, slots, ncas = G.batch_stats(ws)
        same = all(torch.equal(a, b) for a, b in zip(out[1:], outs))
        res["forms"][name] = {"ms": ms, "cell_solves_per_s": n / (ms * 1e-3), "block": block,
                              "waves_per_cu": wpc if mode == G.PERSISTENT else None,
                              "first_attempt_trips": trips, "lane_slots": slots,
                              "active_lane_frac": trips / max(slots, 1), "cascade_cells": ncas,
                              "identical_results": same}
        del ws, out
        print(f"batch form {name}: {ms:.3f} ms", file=sys.stderr, flush=True)
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the step runs on a single MI355X; multi-GPU sharding is not part of this build)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1312_6127_amd import grrmhd as G
    from paper_1312_6127_amd import inputs as I

    dev = torch.device("cuda:0")
    if args.batch_only:
        print(json.dumps({"implicit_batch": bench_batch(G, I, torch, dev, args.batch_cells or (1 << 24))}))
        return
    n = tuple(args.n)
    pd, P, ca, ce = I.accretion_disk(n=n, seed=3)
    stream = torch.cuda.current_stream()
    g = G.Grid(pd)
    Pt = torch.tensor(P, device=dev)
    Ut = g.prim_to_cons(Pt)
    cat = torch.tensor(ca, device=dev)
    cet = torch.tensor(ce, device=dev)
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    st = torch.zeros(g.N, dtype=torch.int32, device=dev)
    it = torch.zeros(g.N, dtype=torch.int32, device=dev)
    P0, U0 = Pt.clone(), Ut.clone()
    if args.copy_probe_mb:
        src = torch.ones(args.copy_probe_mb * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        g.step(Pt, Ut, cat, cet, dt, status=st, iters=it)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    g.time_implicit(True)
    e0.record(stream)
    for _ in range(args.steps):
        g.step(Pt, Ut, cat, cet, dt, status=st, iters=it)
    e1.record(stream)
    torch.cuda.synchronize()
    g.time_implicit(False)
    ms = e0.elapsed_time(e1)
    ms_step = ms / args.steps
    zones = n[0] * n[1] * n[2]
    value = zones * args.steps / (ms * 1e-3)
    interior = I.interior(pd)
    na = I.nalloc(pd)
    stv = st.cpu().numpy().reshape(na[::-1])[interior]
    itv = it.cpu().numpy().reshape(na[::-1])[interior]
    nfail = int(((stv & G.ST_FAIL) != 0).sum())

    # dominant kernel: the implicit kernel of each stage, timed with HIP events
    # on its stream inside the timed region
    imp_total_ms, imp_launches = g.implicit_time()
    trips, slots, _ = g.implicit_stats()
    imp_ms = imp_total_ms / max(imp_launches, 1)
    fresh = KERNEL_DIGEST is not None and KERNEL_DIGEST == kernel_digest()
    roof = {"kernel": "k_implicit", "bound": "alu", "unit": "TFLOP/s", "peak": FP64_PEAK_TFLOPS,
            "avg_launch_ms": imp_ms, "launches": imp_launches,
            "newton_trips_per_launch": trips / max(imp_launches, 1),
            "lane_slots_per_launch": slots / max(imp_launches, 1),
            "active_lane_frac": trips / max(slots, 1),
            "flops_per_trip": FLOPS_PER_TRIP, "counters_current": fresh,
            "achieved": None, "frac": None, "traffic": None}
    if FLOPS_PER_TRIP:
        ach = FLOPS_PER_TRIP * trips / (imp_total_ms * 1e-3) / 1e12
        roof["achieved"] = ach
        roof["frac"] = ach / FP64_PEAK_TFLOPS
        roof["issued_frac"] = FLOPS_PER_TRIP * slots / (imp_total_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS
    if fresh and HBM_BYTES_PER_LAUNCH:
        roof["traffic"] = HBM_BYTES_PER_LAUNCH
        roof["traffic_GBs"] = HBM_BYTES_PER_LAUNCH / (imp_ms * 1e-3) / 1e9

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        oracle.build()
        Ph = P0.cpu().numpy()
        Uh = U0.cpu().numpy()
        t0 = time.perf_counter()
        for _ in range(args.cpu_steps):
            Ph, Uh, dth, sth, ith, nb = oracle.step(pd, Ph, Uh, ca, ce)
        tc = time.perf_counter() - t0
        cpu = {"value": zones * args.cpu_steps / tc, "unit": "zone-cycles/s",
               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
               "kind": "oracle",
               "sample": f"{args.cpu_steps} full steps of the same {n[0]}x{n[1]}x{n[2]} workload"}

    out = {
        "metric": "zone-cycles/s per GRRMHD step (FP32-mixed vs FP64) at stated rel. error; % HBM peak",
        "value": value,
        "unit": "zone-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3-D Kerr-Schild a=0.9375 accretion-shaped grid {n[0]}x{n[1]}x{n[2]}, "
                               "FP64 RK3-IMEX step, LAXF, MC, flux-CT, implicit G^mu",
                   "grid": list(n), "precision": "fp64", "parity_vs_oracle": "1e-11 per field (tests)"},
        "implicit": {"mean_newton_iters_per_cell_step": float(itv.mean()), "failed_cells": nfail},
        "step_hbm": {"algorithmic_bytes_per_zone_cycle": STEP_BYTES_PER_ZONE,
                     "achieved_GBs": value * STEP_BYTES_PER_ZONE / 1e9,
                     "frac": value * STEP_BYTES_PER_ZONE / 1e9 / HBM_PEAK_GBS},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if args.batch_cells:
        out["implicit_batch"] = bench_batch(G, I, torch, dev, args.batch_cells)
    print(json.dumps(out))
    g.close()


if __name__ == "__main__":
    main()
