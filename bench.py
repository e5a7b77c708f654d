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

# FP64 instructions per PMHD/URAD Newton iteration and per cell of the
# implicit kernel, from a rocprofv3 counter run (see the profiles folder);
# used to turn the live launch time into achieved FP64 throughput.
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


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
    return ap.parse_args()


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

    n = tuple(args.n)
    pd, P, ca, ce = I.accretion_disk(n=n, seed=3)
    dev = torch.device("cuda:0")
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
    e0.record(stream)
    for _ in range(args.steps):
        g.step(Pt, Ut, cat, cet, dt, status=st, iters=it)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ms_step = ms / args.steps
    zones = n[0] * n[1] * n[2]
    value = zones * args.steps / (ms * 1e-3)
    interior = I.interior(pd)
    na = I.nalloc(pd)
    stv = st.cpu().numpy().reshape(na[::-1])[interior]
    itv = it.cpu().numpy().reshape(na[::-1])[interior]
    nfail = int(((stv & G.ST_FAIL) != 0).sum())

    # dominant kernel: the implicit solve of stage 1 on the current state,
    # launched alone through the C ABI and timed with events on its stream
    Pb = g.apply_bc(Pt.clone())
    F, emf, vch = g.fluxes(Pb, cat, cet)
    dts = g.timestep(vch)
    Ue = g.explicit_update(1.0, 0.0, 1.0, dts, Pb, Ut, Ut, F, emf)
    reps = 5
    k0 = torch.cuda.Event(enable_timing=True)
    k1 = torch.cuda.Event(enable_timing=True)
    g.implicit(Ue, Pb, 1.0, dts, cat, cet)
    torch.cuda.synchronize()
    k0.record(stream)
    for _ in range(reps):
        res = g.implicit(Ue, Pb, 1.0, dts, cat, cet)
    k1.record(stream)
    torch.cuda.synchronize()
    imp_ms = k0.elapsed_time(k1) / reps
    imp_iters = res[2].cpu().numpy().reshape(na[::-1])[interior]
    # per-launch algorithmic FP64 flops: Newton iterations of the launch times
    # the flops one iteration costs (see DESIGN: per-iteration count)
    flops_per_iter = float(os.environ.get("GRRMHD_FLOPS_PER_ITER", "0")) or None
    roof = {"kernel": "k_implicit", "bound": "alu", "unit": "TFLOP/s", "peak": FP64_PEAK_TFLOPS,
            "avg_launch_ms": imp_ms, "newton_iters_per_launch": int(imp_iters.sum()),
            "achieved": None, "frac": None, "traffic": None}
    if flops_per_iter:
        ach = flops_per_iter * imp_iters.sum() / (imp_ms * 1e-3) / 1e12
        roof["achieved"] = ach
        roof["frac"] = ach / FP64_PEAK_TFLOPS

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
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    g.close()


if __name__ == "__main__":
    main()
