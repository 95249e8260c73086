#!/usr/bin/env python3
"""Throughput of the block-iterative CT solver on one MI355X.

A step is one epoch of Alg. 6 on the 2D fan-beam workload: 512 x 512 image at
0.5 mm, 720 views over 360 degrees, 768-bin curved detector (1e-3 rad), source
500 mm / detector 1000 mm from the source, 12-ellipse seeded phantom, 1%
Gaussian noise; 8 view groups x 8 image tiles, row blocks drawn with
probability proportional to nnz(A_I^J), alpha = 0.5, group size 1.  Each epoch
runs, per column block, the gather back-projection, the fused forward
projection, the step, and the finalize/residual kernels.

Printed as one JSON line.  value = ray-voxel updates per second over the
timed epochs (2 nnz(A_{I_G}^J) per group update, from the exact density
table), inputs resident in HBM.  The roofline figure is the dominant kernel's
algorithmic work over its average launch time, measured with a HIP event pair
around every kernel in a replay of as many epochs right after the timed ones
(the events themselves add gaps, so they stay out of the timed epochs).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# roofline constants (MI355X)
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TFLOPS = 78.6          # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz, no packed FP32
FLOPS_PER_UPDATE = 5.0           # select next crossing, segment length, advance, multiply-add
GATHER_BYTES_PER_UPDATE = 4.0    # what an explicit-A SpMV would stream per nonzero


def workload(name):
    from paper_1709_00953_amd import inputs
    if name == "fan2d_512":
        return inputs.config_c2(), dict(alpha=0.5, gamma=1.0, s=1, b=1.0, seed=2000, noise=0.01)
    if name == "par2d_64":
        return inputs.config_c1(), dict(alpha=0.5, gamma=1.0, s=1, b=0.5, seed=1000, noise=0.01)
    raise SystemExit(f"unknown workload {name}")


def updates_per_epoch(ex, nnz):
    out = []
    for e in range(len(ex["epoch_col_ptr"]) - 1):
        u = 0
        for c in range(ex["epoch_col_ptr"][e], ex["epoch_col_ptr"][e + 1]):
            J = ex["cols"][c]
            lo = ex["group_rb_ptr"][ex["col_group_ptr"][c]]
            hi = ex["group_rb_ptr"][ex["col_group_ptr"][c + 1]]
            u += 2 * int(nnz[ex["rbs"][lo:hi], J].sum())
        out.append(u)
    return out


def cpu_baseline(g, y, ex, budget_s=15.0):
    """The FP64 oracle, as it is, on a bounded sample of the same workload:
    whole epochs of the same schedule and y (wrapping around the schedule)
    until about ``budget_s`` seconds of oracle time, with the explicit A built
    first (its build time is reported, not timed)."""
    from oracle import csgd, siddon
    t0 = time.perf_counter()
    A = siddon.system_matrix(g)
    S = csgd.BlockSystem(A, g)
    for I in range(g.m):                     # sub-block extraction is setup, like A
        for J in range(g.n):
            S.block(I, J)
    t_build = time.perf_counter() - t0

    class Sched:
        def __init__(self, ex):
            self.ex = ex

        def steps(self, e):
            ex = self.ex
            for c in range(ex["epoch_col_ptr"][e], ex["epoch_col_ptr"][e + 1]):
                groups = []
                for G in range(ex["col_group_ptr"][c], ex["col_group_ptr"][c + 1]):
                    rbs = ex["rbs"][ex["group_rb_ptr"][G]:ex["group_rb_ptr"][G + 1]]
                    groups.append(([int(t) for t in rbs], float(ex["beta"][G])))
                yield int(ex["cols"][c]), groups

    sched = Sched(ex)
    E = len(ex["epoch_col_ptr"]) - 1
    st = csgd.State(S, np.asarray(y, dtype=np.float64))
    t_run, epochs = 0.0, 0
    while t_run < budget_s and epochs < 1000:
        t = time.perf_counter()
        csgd.epoch(st, sched, epochs % E)
        t_run += time.perf_counter() - t
        epochs += 1
    return {"value": st.updates / t_run, "unit": "ray-voxel updates/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"{epochs} epochs (schedule wrapped every {E}) of the same workload, "
                       f"schedule and y: {st.updates} updates in {t_run:.2f} s, scipy CSR "
                       f"matvecs on 1 thread; explicit FP64 A ({A.nnz} nnz) and its {g.m}x{g.n} "
                       f"sub-blocks built beforehand in {t_build:.1f} s, untimed"),
            "seconds": t_run}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="fan2d_512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {max(args.gpus, world)}); "
              "sharding the column blocks across GPUs is not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1709_00953_amd import ct, inputs

    torch.cuda.set_device(0)
    g, cfg = workload(args.workload)
    t_setup = time.perf_counter()
    G = ct.ct_geom_create(g)
    tau = 1e-5 * min(g.vx, g.vy)
    x_true = inputs.phantom_for(g, cfg["seed"])
    xt = torch.as_tensor(x_true.astype(np.float32), device="cuda")
    p = torch.zeros(G.M, device="cuda")
    for J in range(G.n):                       # y = A x_true with the validated projector
        ct.ct_block_fwd(G, list(range(G.m)), J, xt, p, flags=ct.CT_ACCUMULATE if J else 0)
    y_np = inputs.gaussian_noise(p.cpu().numpy().astype(np.float64), cfg["noise"], cfg["seed"])
    y = torch.as_tensor(y_np, device="cuda")
    nnz = ct.ct_geom_block_nnz(G, tau)
    E = args.warmup + args.steps
    # epochs [0, W) warm up, [W, E) are timed, [E, E + K) are replayed with a
    # HIP event pair around every kernel for the per-kernel durations (the
    # events add gaps, so they stay out of the timed epochs)
    params = ct.sched_params(E + args.steps, cfg["alpha"], cfg["gamma"], cfg["s"], cfg["b"],
                             seed=cfg["seed"])
    sched = ct.ct_schedule_create(G, params, nnz)
    ex = ct.ct_schedule_export(sched)
    upd = updates_per_epoch(ex, nnz)
    sol = ct.ct_solver_create(G)
    x = torch.zeros(G.N, device="cuda")
    ct.ct_solver_reset(sol, y)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup

    for e in range(args.warmup):
        ct.ct_block_epoch(sol, sched, e, y, x)
    torch.cuda.synchronize()

    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for e in range(args.warmup, E):
        ct.ct_block_epoch(sol, sched, e, y, x)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    rel = ct.ct_true_residual(sol, y, x)

    ct.ct_solver_profile(sol, True)
    for e in range(E, E + args.steps):
        ct.ct_block_epoch(sol, sched, e, y, x)
    kt = ct.ct_solver_profile_read(sol)
    ct.ct_solver_profile(sol, False)
    prof_updates = sum(upd[E:E + args.steps])

    timed_updates = sum(upd[args.warmup:E])
    value = timed_updates / (ms * 1e-3)

    # dominant kernel and its roofline
    dom = max(kt, key=lambda k: kt[k][0])
    dom_ms, dom_n = kt[dom]
    avg_ms = dom_ms / max(dom_n, 1)
    if dom in ("back", "fwd"):
        units = prof_updates / 2                # ray-voxel pairs handled by one projector
        per_launch = units / dom_n
        achieved = per_launch * FLOPS_PER_UPDATE / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 4), "peak": VALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / VALU_PEAK_TFLOPS, 5),
                "traffic": None, "kernel": dom, "avg_launch_ms": round(avg_ms, 5),
                "launches": dom_n, "units_per_launch": per_launch,
                "flops_per_unit": FLOPS_PER_UPDATE}
        gbytes = per_launch * GATHER_BYTES_PER_UPDATE / (avg_ms * 1e-3) / 1e9
        gather = {"achieved": round(gbytes, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(gbytes / HBM_PEAK_GBS, 5)}
    else:
        roof = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": None, "traffic": None, "kernel": dom}
        gather = None

    out = {
        "metric": "ray-voxel updates/s (fwd+back)",
        "value": value,
        "unit": "ray-voxel updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ("fan2d_curved 512x512 0.5mm, 720 views/360deg, 768 bins "
                                "1e-3 rad, SID 500 SDD 1000, 8x8 blocks, P~nnz, alpha 0.5, s 1"
                                if args.workload == "fan2d_512" else args.workload),
                   "epoch_updates": upd[args.warmup], "b": cfg["b"],
                   "rel_residual_after": rel, "setup_s": round(t_setup, 3)},
        "roofline": roof,
        "gather_equivalent_hbm": gather,
        "kernels_ms": {k: round(v[0], 4) for k, v in kt.items()},
        "kernels_note": "per-kernel HIP-event times from the same number of epochs run right after the timed ones",
        "kernels_launches": {k: v[1] for k, v in kt.items()},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, y_np, ex, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
