"""Benchmark: zone-cycles/s of the full RK3-IMEX GRRMHD step on one MI355X.

Workload: 3-D Kerr-Schild accretion-shaped grid, spin 0.9375, 128x64x32
interior cells (log r in [1.2, 40], theta in (0, pi), phi periodic), FP64,
LAXF fluxes, MC reconstruction, flux-CT, implicit 4-force per cell; inputs
are synthetic and seeded (paper_1312_6127_amd.inputs.accretion_disk).

Prints one JSON line.  value = interior cells x steps / wall time of the K
timed FP64 steps (HIP events on the step's stream, inputs resident in HBM).
mixed_precision: the same run with FP32 reconstruction, face states,
Riemann fluxes and EMFs, and the per-field error of both precisions against
the FP64 oracle after the oracle's steps.  imex3: the same workload stepped
with the IMEX3 scheme (eq. IMEX3; four implicit stages), its time per step
and its error against the oracle's IMEX3 steps.  ppm: the same disk recipe
with PPM reconstruction and the shock flattener (ghost width 4), its time
per step and its error against the oracle's PPM steps.  roofline: the dominant kernel
(the implicit kernel's first PMHD attempt), its average launch time from HIP
events on its stream inside the timed region.  cpu_baseline: the FP64 oracle
stepping the same workload on the host cores (bounded sample).
adjoint: the adjoint of one FP64 step of the 96x48x24 Kerr-Schild disk
(dt held fixed), its time per call next to the forward step's, and a
directional-derivative check of it on the GPU; the same for IMEX3 and for
PPM reconstruction.  implicit_batch
(--batch-cells): the batched implicit solve in each execution form.
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
FLOPS_PER_TRIP = 1732.0
HBM_BYTES_PER_LAUNCH = 161.4e6
KERNEL_DIGEST = "a496eb5245363797"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, nargs=3, default=[128, 64, 32])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint leg")
    ap.add_argument("--adjoint-only", action="store_true", help="run only the adjoint leg")
    ap.add_argument("--imex-err-steps", type=int, default=3,
                    help="IMEX3 and PPM steps compared with the oracle's")
    ap.add_argument("--cpu-steps", type=int, default=20,
                    help="oracle steps (the CPU baseline sample and the error reference)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also copy a buffer of this many MiB (counter calibration)")
    ap.add_argument("--batch-cells", type=int, default=0,
                    help="also time the batched implicit solve on this many independent cells "
                         "in each execution form (16777216 for the 16.7M-cell batch)")
    ap.add_argument("--batch-only", action="store_true",
                    help="time only the batched implicit solve")
    ap.add_argument("--no-fiducial", action="store_true",
                    help="skip the 256x128x64 leg (the paper's fiducial disk shape)")
    ap.add_argument("--cpu1-steps", type=int, default=1,
                    help="oracle steps on one host thread (single-core baseline; 0 skips)")
    return ap.parse_args()


def kernel_digest():
    """sha256 over the HIP sources of the implicit kernel: the headers it
    includes and the part of kernels.h from the implicit-solve section
    (make_phys, make_opts, Work, the tile order, k_implicit) up to the
    listed-cell kernel, plus xcd_block."""
    import hashlib

    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1312_6127_amd", "csrc")
    for f in ("dual.h", "common.h", "physics.h", "invert.h", "implicit.h"):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(d, "kernels.h"), encoding="utf-8") as fh:
        k = fh.read()
    a = k.index("// steps 11-12: implicit solve per interior cell")
    b = k.index("// Rest of the cascade over the work list")
    x = k.index("DEV long xcd_block")
    h.update(k[x:k.index("}", x) + 1].encode())
    h.update(k[a:b].encode())
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
           "cold_frac": float(((st & G.ST_COLD) != 0).mean()),
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
        ctrips, cslots = G.batch_cascade_stats(ws)
        same = all(torch.equal(a, b) for a, b in zip(out[1:], outs))
        res["forms"][name] = {"ms": ms, "cell_solves_per_s": n / (ms * 1e-3), "block": block,
                              "waves_per_cu": wpc if mode == G.PERSISTENT else None,
                              "first_attempt_trips": trips, "lane_slots": slots,
                              "active_lane_frac": trips / max(slots, 1), "cascade_cells": ncas,
                              "cascade_trips": ctrips, "cascade_lane_slots": cslots,
                              "cascade_active_lane_frac": ctrips / max(cslots, 1),
                              "identical_results": same}
        del ws, out
        print(f"batch form {name}: {ms:.3f} ms", file=sys.stderr, flush=True)
    return res


GROUPS = [(0,), (1,), (2, 3, 4), (5, 6, 7), (8,), (9, 10, 11)]
FIELDS = ["rho", "u_g", "u1", "u2", "u3", "B1", "B2", "B3", "Ebar", "ur1", "ur2", "ur3"]


def bench_adjoint(G, I, torch, dev, reps=5, warmup=2, h=1e-7, scheme="rk3", recon="mc"):
    """Adjoint of one FP64 step (RK3, or the scheme named; MC, or PPM with
    four ghost cells) of the 96x48x24 Kerr-Schild disk, dt held
    fixed (the forward step recomputed with its stage checkpoints, then the
    reverse sweep): ms per call and the forward step's ms, both from HIP
    events on the library's stream; and <gP, v> against the central
    difference (L(P + h v) - L(P - h v)) / 2h of the GPU step, with
    L = sum(gU . U^{n+1}), gU seeded normals on the interior cells and v
    seeded normals on 256 of them, each component scaled by its own cell's
    magnitude; h = 1e-7 (at 1e-6 the difference crosses limiter kinks of a
    few cells, below 1e-8 rounding dominates)."""
    import numpy as np

    n = (96, 48, 24)
    kw = dict(ng=4, recon="ppm") if recon == "ppm" else {}
    pd, P, ca, ce = I.accretion_disk(n=n, seed=3, **kw)
    pd = dict(pd, scheme=scheme)
    P = I.jitter(P, 11)
    g = G.Grid(pd)

    def T(x):
        return torch.tensor(np.ascontiguousarray(x), device=dev)

    Pt, cat, cet = T(P), T(ca), T(ce)
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    Pw = Pt.clone()
    Uw = g.prim_to_cons(Pw)
    g.step(Pw, Uw, cat, cet, dt)
    mask = np.zeros(I.nalloc(pd)[::-1], bool)
    mask[I.interior(pd)] = True
    mask = mask.reshape(-1)
    r = np.random.default_rng(7)
    w = np.zeros_like(P)
    w[:, mask] = r.standard_normal((12, int(mask.sum())))
    # direction: 256 random interior cells, each component scaled by its own
    # cell's magnitude (vector components floored at 1e-3 of their vector's
    # norm in the cell), so that h v is a small relative change of every
    # quantity (rho0, u_g and Ebar span decades across the disk)
    cells = r.choice(np.flatnonzero(mask), 256, replace=False)
    sc = np.abs(P[:, cells])
    for a, b in ((2, 5), (5, 8), (9, 12)):
        nv = np.sqrt((P[a:b, cells] ** 2).sum(axis=0))
        sc[a:b] = np.maximum(sc[a:b], 1e-3 * nv + 1e-300)
    v = np.zeros_like(P)
    v[:, cells] = r.standard_normal((12, 256)) * sc
    wt, vt = T(w), T(v)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(fn):
        for _ in range(warmup):
            fn()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_adj = timed(lambda: g.step_adjoint(Pt, cat, cet, dt, wt))
    ms_adj_chi = timed(lambda: g.step_adjoint(Pt, cat, cet, dt, wt, want_chi=True))
    ms_fwd = timed(lambda: g.step(Pw, Uw, cat, cet, dt, dt_fixed=True))
    # the two halves autograd uses: forward with checkpoints, then the reverse sweep alone
    ws = g.new_adjoint_workspace()
    ms_ckpt = timed(lambda: g.step_checkpointed(Pt, cat, cet, dt, ws))
    ms_rev = timed(lambda: g.step_adjoint_saved(ws, cat, cet, dt, wt))
    del ws

    def L(Pin):
        Pq = Pin.clone()
        Uq = g.prim_to_cons(Pq)
        g.step(Pq, Uq, cat, cet, dt, dt_fixed=True)
        return float((wt * Uq).sum())

    gP = g.step_adjoint(Pt, cat, cet, dt, wt)
    ad = float((gP * vt).sum())
    fd = (L(Pt + h * vt) - L(Pt - h * vt)) / (2 * h)
    g.close()
    return {"grid": list(n), "scheme": scheme, "recon": recon, "ms_per_adjoint": ms_adj, "ms_per_adjoint_with_opacity_grad": ms_adj_chi,
            "ms_forward_step": ms_fwd, "time_vs_forward": ms_adj / ms_fwd,
            "ms_forward_with_checkpoints": ms_ckpt, "ms_reverse_from_checkpoints": ms_rev,
            "directional_check": {"adjoint": ad, "central_difference": fd, "h": h,
                                  "rel_diff": abs(ad - fd) / abs(fd)}}


def field_errors(a, b):
    """Per-field max|a - b| over interior cells, relative to max|b| over the
    field (over the three components for vectors)."""
    import numpy as np

    out = {}
    for grp in GROUPS:
        s = max(np.abs(b[q]).max() for q in grp)
        for q in grp:
            d = np.abs(a[q] - b[q]).max()
            out[FIELDS[q]] = float(d / s) if s > 0 else float(d)
    return out


def time_steps(G, torch, dev, pd, P, ca, ce, steps, warmup, kernel_timing):
    """Warm up, then time `steps` RK3-IMEX steps with HIP events on the
    step's stream (inputs resident in HBM)."""
    stream = torch.cuda.current_stream()
    g = G.Grid(pd)
    Pt = torch.tensor(P, device=dev)
    Ut = g.prim_to_cons(Pt)
    cat = torch.tensor(ca, device=dev)
    cet = torch.tensor(ce, device=dev)
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    st = torch.zeros(g.N, dtype=torch.int32, device=dev)
    it = torch.zeros(g.N, dtype=torch.int32, device=dev)
    for _ in range(warmup):
        g.step(Pt, Ut, cat, cet, dt, status=st, iters=it)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    if kernel_timing:
        g.time_implicit(True)
    e0.record(stream)
    for _ in range(steps):
        g.step(Pt, Ut, cat, cet, dt, status=st, iters=it)
    e1.record(stream)
    torch.cuda.synchronize()
    res = {"ms": e0.elapsed_time(e1), "st": st.cpu().numpy(), "it": it.cpu().numpy()}
    if kernel_timing:
        g.time_implicit(False)
        res["imp_total_ms"], res["imp_launches"] = g.implicit_time()
        res["trips"], res["slots"], _ = g.implicit_stats()
    g.close()
    return res


def time_steps_stag(G, torch, dev, pd, P, Bf, ca, ce, steps, warmup):
    """time_steps for a staggered-field grid (grrmhd_step_staggered), the
    faces' ghost fill and face-to-centre field set up first."""
    stream = torch.cuda.current_stream()
    g = G.Grid(pd)
    Pt = torch.tensor(P, device=dev)
    Bt = torch.tensor(Bf, device=dev)
    g.apply_bc_faces(Bt)
    g.face_to_center(Bt, Pt, None)
    g.apply_bc(Pt)
    Ut = g.prim_to_cons(Pt)
    cat = torch.tensor(ca, device=dev)
    cet = torch.tensor(ce, device=dev)
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    for _ in range(warmup):
        g.step_staggered(Pt, Ut, Bt, cat, cet, dt)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        g.step_staggered(Pt, Ut, Bt, cat, cet, dt)
    e1.record(stream)
    torch.cuda.synchronize()
    res = {"ms": e0.elapsed_time(e1)}
    g.close()
    return res


def bench_batch_cascade(G, I, torch, dev, n, reps=3):
    """The batched solve (per-cell form) with the normal and the full
    cascade: ms per batch and the fraction of cells per outcome."""
    pd, args = batch_inputs(G, I, torch, dev, n)
    stream = torch.cuda.current_stream()
    out = {"cells": n}
    for cas in (0, 1):
        pdc = dict(pd, cascade=cas)
        ws = G.batch_workspace(n, G.PER_CELL)
        o = G._batch_out(args[0], args[1])
        G.implicit_source_ex(pdc, *args, G.PER_CELL, 64, 1, out=o, ws=ws)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            G.implicit_source_ex(pdc, *args, G.PER_CELL, 64, 1, out=o, ws=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        st = o[4].cpu().numpy()   # (n, P, U, iters, status, err)
        frac = lambda b: float(((st & b) != 0).mean())
        out["full" if cas else "normal"] = {
            "ms": e0.elapsed_time(e1) / reps, "failed_frac": frac(G.ST_FAIL),
            "cold_frac": frac(G.ST_COLD), "urad_frac": frac(G.ST_URAD), "prad_frac": frac(G.ST_PRAD),
            "entropy_frac": frac(G.ST_ENTROPY), "staged_frac": frac(G.ST_STAGED)}
        del ws, o
    print(f"batch cascades: failed {out['normal']['failed_frac']:.4f} -> {out['full']['failed_frac']:.4f}",
          file=sys.stderr, flush=True)
    return out


def gpu_run(G, torch, dev, pd, P, ca, ce, steps):
    """Interior P, U after `steps` steps from the initial state (untimed)."""
    g = G.Grid(pd)
    Pt = torch.tensor(P, device=dev)
    Ut = g.prim_to_cons(Pt)
    cat, cet = torch.tensor(ca, device=dev), torch.tensor(ce, device=dev)
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    for _ in range(steps):
        g.step(Pt, Ut, cat, cet, dt)
    out = Pt.cpu().numpy(), Ut.cpu().numpy()
    g.close()
    return out


def oracle_one_core(n, steps):
    """Zone-cycles/s of the oracle stepping the workload on one host thread,
    in a child process (OpenMP's thread count is fixed when it starts)."""
    import subprocess

    code = ("import sys, time; sys.path.insert(0, %r)\n"
            "import oracle\n"
            "from paper_1312_6127_amd import inputs as I\n"
            "pd, P, ca, ce = I.accretion_disk(n=%r, seed=3)\n"
            "U = oracle.prim_to_cons(pd, P)\n"
            "t0 = time.perf_counter()\n"
            "for _ in range(%d):\n"
            "    P, U, *_ = oracle.step(pd, P, U, ca, ce)\n"
            "print(time.perf_counter() - t0)\n") % (ROOT, tuple(n), steps)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       check=True)
    tc = float(r.stdout.strip().splitlines()[-1])
    return {"value": n[0] * n[1] * n[2] * steps / tc, "unit": "zone-cycles/s", "cores": 1,
            "kind": "oracle", "sample": f"{steps} full step(s) of the same workload on one thread"}


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
    if args.adjoint_only:
        print(json.dumps({"adjoint": bench_adjoint(G, I, torch, dev),
                          "adjoint_imex3": bench_adjoint(G, I, torch, dev, scheme="imex3"),
                          "adjoint_ppm": bench_adjoint(G, I, torch, dev, recon="ppm")}))
        return
    if args.copy_probe_mb:
        src = torch.ones(args.copy_probe_mb * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n = tuple(args.n)
    zones = n[0] * n[1] * n[2]
    pd, P, ca, ce = I.accretion_disk(n=n, seed=3)
    interior = I.interior(pd)
    na = I.nalloc(pd)

    r64 = time_steps(G, torch, dev, pd, P, ca, ce, args.steps, args.warmup, kernel_timing=True)
    print(f"fp64 steps: {r64['ms'] / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
    ms_step = r64["ms"] / args.steps
    value = zones * args.steps / (r64["ms"] * 1e-3)
    stv = r64["st"].reshape(na[::-1])[interior]
    itv = r64["it"].reshape(na[::-1])[interior]
    nfail = int(((stv & G.ST_FAIL) != 0).sum())
    pdm = dict(pd, precision="mixed")
    rmx = time_steps(G, torch, dev, pdm, P, ca, ce, args.steps, args.warmup, kernel_timing=False)
    print(f"mixed steps: {rmx['ms'] / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
    pdi = dict(pd, scheme="imex3")
    rim = time_steps(G, torch, dev, pdi, P, ca, ce, args.steps, args.warmup, kernel_timing=False)
    print(f"imex3 steps: {rim['ms'] / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
    imex = {"value": zones * args.steps / (rim["ms"] * 1e-3), "ms_per_step": rim["ms"] / args.steps,
            "time_vs_rk3": rim["ms"] / r64["ms"]}
    pdp, Pp, cap, cep = I.accretion_disk(n=n, seed=3, ng=4, recon="ppm")
    rpp = time_steps(G, torch, dev, pdp, Pp, cap, cep, args.steps, args.warmup, kernel_timing=False)
    print(f"ppm steps: {rpp['ms'] / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
    ppm = {"value": zones * args.steps / (rpp["ms"] * 1e-3), "ms_per_step": rpp["ms"] / args.steps,
           "time_vs_mc": rpp["ms"] / r64["ms"]}

    # the paper's own stopping rule for the implicit solve (roundoff = 0)
    pdr = dict(pd, roundoff=0)
    rpm = time_steps(G, torch, dev, pdr, P, ca, ce, args.steps, args.warmup, kernel_timing=False)
    print(f"paper-rule steps: {rpm['ms'] / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
    itp = rpm["it"].reshape(na[::-1])[interior]
    paper = {"value": zones * args.steps / (rpm["ms"] * 1e-3), "ms_per_step": rpm["ms"] / args.steps,
             "time_vs_roundoff_mode": rpm["ms"] / r64["ms"],
             "mean_newton_iters_per_cell_step": float(itp.mean()),
             "mean_newton_iters_per_cell_step_roundoff_mode": float(itv.mean())}
    # the staggered face-centred field with four-state corner EMFs
    pds, Ps, cas, ces, Bfs = I.accretion_disk(n=n, seed=3, faces=True, ct="staggered")
    rst = time_steps_stag(G, torch, dev, pds, Ps, Bfs, cas, ces, args.steps, args.warmup)
    print(f"staggered steps: {rst['ms'] / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
    stag = {"value": zones * args.steps / (rst["ms"] * 1e-3), "ms_per_step": rst["ms"] / args.steps,
            "time_vs_flux_ct": rst["ms"] / r64["ms"]}
    # the full implicit cascade (PRAD, staged, entropy methods) on the disk
    pdc = dict(pd, cascade=1)
    rca = time_steps(G, torch, dev, pdc, P, ca, ce, args.steps, args.warmup, kernel_timing=False)
    print(f"full-cascade steps: {rca['ms'] / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
    casc = {"value": zones * args.steps / (rca["ms"] * 1e-3), "ms_per_step": rca["ms"] / args.steps,
            "time_vs_normal_cascade": rca["ms"] / r64["ms"],
            "batch": bench_batch_cascade(G, I, torch, dev, 1 << 20)}
    fid = None
    if not args.no_fiducial:
        nf = (256, 128, 64)
        pdf, Pf, caf, cef = I.accretion_disk(n=nf, seed=3)
        rf = time_steps(G, torch, dev, pdf, Pf, caf, cef, max(args.steps // 2, 1), 2, kernel_timing=True)
        nfs = max(args.steps // 2, 1)
        vf = nf[0] * nf[1] * nf[2] * nfs / (rf["ms"] * 1e-3)
        fid = {"grid": list(nf), "steps": nfs, "ms_per_step": rf["ms"] / nfs, "value": vf,
               "unit": "zone-cycles/s",
               "step_hbm_frac": vf * STEP_BYTES_PER_ZONE / 1e9 / HBM_PEAK_GBS,
               "implicit_avg_launch_ms": rf["imp_total_ms"] / max(rf["imp_launches"], 1),
               "implicit_active_lane_frac": rf["trips"] / max(rf["slots"], 1)}
        if FLOPS_PER_TRIP:
            fid["implicit_frac_fp64"] = FLOPS_PER_TRIP * rf["trips"] / (rf["imp_total_ms"] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS
        print(f"fiducial 256x128x64: {fid['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
        del Pf, caf, cef

    adj = None if args.no_adjoint else bench_adjoint(G, I, torch, dev)
    adj3 = None if args.no_adjoint else bench_adjoint(G, I, torch, dev, scheme="imex3")
    adjp = None if args.no_adjoint else bench_adjoint(G, I, torch, dev, recon="ppm")
    if adj:
        print(f"adjoint: {adj['ms_per_adjoint']:.3f} ms/call (IMEX3 {adj3['ms_per_adjoint']:.3f}, "
              f"PPM {adjp['ms_per_adjoint']:.3f})", file=sys.stderr, flush=True)

    # dominant kernel: the implicit kernel of each stage, timed with HIP events
    # on its stream inside the timed region
    trips, slots = r64["trips"], r64["slots"]
    imp_total_ms, imp_launches = r64["imp_total_ms"], r64["imp_launches"]
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

    mixed = {"value": zones * args.steps / (rmx["ms"] * 1e-3), "ms_per_step": rmx["ms"] / args.steps,
             "speedup_vs_fp64": r64["ms"] / rmx["ms"], "r_fp64": pdm["r_fp64"]}
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle steps the same workload from the same initial state; its
        # result is also the reference of both GPU precisions' error
        import oracle

        oracle.build()
        Uh = oracle.prim_to_cons(pd, P)
        Ph = P
        t0 = time.perf_counter()
        for _ in range(args.cpu_steps):
            Ph, Uh, dth, sth, ith, nb = oracle.step(pd, Ph, Uh, ca, ce)
        tc = time.perf_counter() - t0
        cpu = {"value": zones * args.cpu_steps / tc, "unit": "zone-cycles/s",
               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
               "kind": "oracle",
               "sample": f"{args.cpu_steps} full steps of the same {n[0]}x{n[1]}x{n[2]} workload "
                         "from its initial state"}
        ref = [x.reshape((12,) + na[::-1])[(slice(None),) + interior].reshape(12, -1) for x in (Ph, Uh)]
        errs = {}
        for name, pdx in (("fp64", pd), ("mixed", pdm)):
            Pg, Ug = gpu_run(G, torch, dev, pdx, P, ca, ce, args.cpu_steps)
            got = [x.reshape((12,) + na[::-1])[(slice(None),) + interior].reshape(12, -1) for x in (Pg, Ug)]
            errs[name] = {"P": field_errors(got[0], ref[0]), "U": field_errors(got[1], ref[1])}
            errs[name]["max"] = max(max(errs[name]["P"].values()), max(errs[name]["U"].values()))
        mixed["err_vs_oracle"] = errs["mixed"]
        mixed["fp64_err_vs_oracle_max"] = errs["fp64"]["max"]
        mixed["err_steps"] = args.cpu_steps
        # IMEX3 against the oracle's IMEX3 (a few steps: the oracle is slow)
        Ph, Uh = P, oracle.prim_to_cons(pdi, P)
        for _ in range(args.imex_err_steps):
            Ph, Uh, dth, sth, ith, nb = oracle.step(pdi, Ph, Uh, ca, ce)
        ref = [x.reshape((12,) + na[::-1])[(slice(None),) + interior].reshape(12, -1) for x in (Ph, Uh)]
        Pg, Ug = gpu_run(G, torch, dev, pdi, P, ca, ce, args.imex_err_steps)
        got = [x.reshape((12,) + na[::-1])[(slice(None),) + interior].reshape(12, -1) for x in (Pg, Ug)]
        e = [field_errors(got[0], ref[0]), field_errors(got[1], ref[1])]
        imex["err_vs_oracle_max"] = max(max(e[0].values()), max(e[1].values()))
        imex["err_steps"] = args.imex_err_steps
        # PPM against the oracle's PPM (same few steps)
        nap, intp = I.nalloc(pdp), I.interior(pdp)
        Ph, Uh = Pp, oracle.prim_to_cons(pdp, Pp)
        for _ in range(args.imex_err_steps):
            Ph, Uh, dth, sth, ith, nb = oracle.step(pdp, Ph, Uh, cap, cep)
        ref = [x.reshape((12,) + nap[::-1])[(slice(None),) + intp].reshape(12, -1) for x in (Ph, Uh)]
        Pg, Ug = gpu_run(G, torch, dev, pdp, Pp, cap, cep, args.imex_err_steps)
        got = [x.reshape((12,) + nap[::-1])[(slice(None),) + intp].reshape(12, -1) for x in (Pg, Ug)]
        e = [field_errors(got[0], ref[0]), field_errors(got[1], ref[1])]
        ppm["err_vs_oracle_max"] = max(max(e[0].values()), max(e[1].values()))
        ppm["err_steps"] = args.imex_err_steps
        # the paper's stopping rule against the oracle's (same few steps)
        Ph, Uh = P, oracle.prim_to_cons(pdr, P)
        for _ in range(args.imex_err_steps):
            Ph, Uh, dth, sth, ith, nb = oracle.step(pdr, Ph, Uh, ca, ce)
        ref = [x.reshape((12,) + na[::-1])[(slice(None),) + interior].reshape(12, -1) for x in (Ph, Uh)]
        Pg, Ug = gpu_run(G, torch, dev, pdr, P, ca, ce, args.imex_err_steps)
        got = [x.reshape((12,) + na[::-1])[(slice(None),) + interior].reshape(12, -1) for x in (Pg, Ug)]
        e = [field_errors(got[0], ref[0]), field_errors(got[1], ref[1])]
        paper["err_vs_oracle_max"] = max(max(e[0].values()), max(e[1].values()))
        paper["err_steps"] = args.imex_err_steps
        # the staggered field against the oracle's (same few steps)
        Bh = oracle.bc_face(pds, Bfs)
        Ph, Uh = oracle.face_to_center(pds, Bh, Ps, np.zeros_like(Ps))
        Ph = oracle.bc(pds, Ph)
        Uh = oracle.prim_to_cons(pds, Ph)
        P0, U0, B0 = Ph, Uh, Bh
        for _ in range(args.imex_err_steps):
            Ph, Uh, Bh, dth, sth, ith, nb = oracle.step_stag(pds, Ph, Uh, Bh, cas, ces)
        gs = G.Grid(pds)
        Pt, Ut, Bt = (torch.tensor(x, device=dev) for x in (P0, U0, B0))
        cat, cet = torch.tensor(cas, device=dev), torch.tensor(ces, device=dev)
        dtt = torch.zeros(1, dtype=torch.float64, device=dev)
        for _ in range(args.imex_err_steps):
            gs.step_staggered(Pt, Ut, Bt, cat, cet, dtt)
        Pg, Ug, Bg = Pt.cpu().numpy(), Ut.cpu().numpy(), Bt.cpu().numpy()
        gs.close()
        ref = [x.reshape((12,) + na[::-1])[(slice(None),) + interior].reshape(12, -1) for x in (Ph, Uh)]
        got = [x.reshape((12,) + na[::-1])[(slice(None),) + interior].reshape(12, -1) for x in (Pg, Ug)]
        e = [field_errors(got[0], ref[0]), field_errors(got[1], ref[1])]
        stag["err_vs_oracle_max"] = max(max(e[0].values()), max(e[1].values()))
        stag["err_steps"] = args.imex_err_steps
        if args.cpu1_steps:
            cpu["one_core"] = oracle_one_core(n, args.cpu1_steps)

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
                   "grid": list(n), "precision": "fp64", "parity_vs_oracle": "1e-12 per step per field (tests)"},
        "implicit": {"mean_newton_iters_per_cell_step": float(itv.mean()), "failed_cells": nfail},
        "step_hbm": {"algorithmic_bytes_per_zone_cycle": STEP_BYTES_PER_ZONE,
                     "achieved_GBs": value * STEP_BYTES_PER_ZONE / 1e9,
                     "frac": value * STEP_BYTES_PER_ZONE / 1e9 / HBM_PEAK_GBS},
        "mixed_precision": mixed,
        "imex3": imex,
        "ppm": ppm,
        "paper_stopping_rule": paper,
        "staggered_field": stag,
        "full_cascade": casc,
        "fiducial_256x128x64": fid,
        "adjoint": adj,
        "adjoint_imex3": adj3,
        "adjoint_ppm": adjp,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if args.batch_cells:
        out["implicit_batch"] = bench_batch(G, I, torch, dev, args.batch_cells)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
