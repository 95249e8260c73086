#!/usr/bin/env python3
"""Throughput of the block-iterative CT solver on one MI355X.

Default workload (cone3d_256, the largest single-GPU case): a step is one
epoch of Alg. 6 on the 3D cone-beam case: 256^3 volume at 0.5 mm, 360 views
of 384 x 384 bins at 1 mm over 360 degrees on a circular orbit, source 500 mm
/ detector 1000 mm from the source, 20-ellipsoid seeded phantom, Poisson
noise at 1e5 photons per ray; 12 view groups x 8 z-slabs, alpha = 1, groups
of s = 3 row blocks (4 groups per column block).  Each epoch runs, per column
block, the gather back-projection, the fused forward projection, the step,
and the finalize/residual kernels.

Other workloads (--workload): fan2d_512 (2D fan beam, 512^2, 720 views, 768
curved bins, 8 x 8 blocks), par2d_64 (the small parallel-beam case),
batch64 (64 fan slices of uneven sizes, all jobs advanced by shared
launches, against the same jobs solved one at a time), serve40 (a Poisson
stream of mixed fan and cone jobs served by the continuous-batching server,
against the same stream served one job at a time).

Printed as one JSON line.  value = ray-voxel updates per second over the
timed epochs (2 nnz(A_{I_G}^J) per group update, from the exact density
table), inputs resident in HBM.  The roofline object is the dominant
kernel's gather-equivalent byte rate: 4 B per ray-voxel pair plus 4 B per
output element per launch (what a matrix-stored projector would stream),
over its average launch time measured with a HIP event pair around every
kernel in a replay of as many epochs right after the timed ones (the events
add gaps, so they stay out of the timed epochs), against the 8 TB/s HBM
peak.  Measured DRAM bytes and VALU instructions from rocprofv3 counters of
the same kernel version are given beside it.
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
GATHER_BYTES = 4.0               # per ray-voxel pair and per output element
N_SIMD, CLOCK_HZ = 1024, 2.4e9   # 256 CUs x 4 SIMDs; a wave64 VALU instruction issues over 4 cycles
BATCH_SIZES = (128, 256, 384, 512, 768, 1024)
# Counters of the dominant kernels, per dispatch, from rocprofv3 runs of the
# kernel version they name (FETCH_SIZE and WRITE_SIZE in KiB, each from its
# own pass, scaled by what the same counters read for a plain 256 MiB device
# copy: fetch x 2.0, write x 1.0; SQ_INSTS_VALU in wave instructions).  An
# entry holds only for the kernel version it was taken on.
PMC_FETCH_SCALE, PMC_WRITE_SCALE = 2.0, 1.0
COUNTERS = {
    ("fan2d_512", "back"): {"fetch": 21810.0, "write": 2112.0, "valu": 1.179e7,
                            "profile": "profiles/fan2d_512_back_projection_hbm_traffic.md"},
    ("cone3d_256", "back"): {"fetch": 187089.4, "write": 132013.0, "valu": 7.841e8,
                             "profile": "profiles/cone3d_256_counters.md"},
}
SERVE_FAN = (256, 384, 512, 768, 1024)
SERVE_CONE = (64, 96, 128, 160, 192)


def single_workload(name):
    from paper_1709_00953_amd import inputs
    if name == "fan2d_512":
        return (inputs.config_c2(), dict(alpha=0.5, gamma=1.0, s=1, b=1.0, seed=2000, noise=0.01),
                "fan2d_curved 512x512 0.5mm, 720 views/360deg, 768 bins 1e-3 rad, SID 500 SDD 1000, "
                "8x8 blocks, P~nnz, alpha 0.5, s 1")
    if name == "par2d_64":
        return (inputs.config_c1(), dict(alpha=0.5, gamma=1.0, s=1, b=0.5, seed=1000, noise=0.01),
                "par2d 64x64 1mm, 90 views/180deg, 96 bins 1mm, 4x4 blocks, P~nnz, alpha 0.5, s 1")
    if name == "cone3d_256":
        return (inputs.config_c3(), dict(alpha=1.0, gamma=1.0, s=3, b=1.0, seed=3000, photons=1e5),
                "cone3d 256^3 0.5mm, 360 views/360deg of 384x384 1mm, SID 500 SDD 1000, 12 view "
                "groups x 8 z-slabs, alpha 1, s 3 (4 groups), Poisson 1e5 photons")
    if name == "fan2d_512_parallel":
        return (inputs.config_c2(), dict(alpha=0.5, gamma=0.5, s=1, b=1.0, seed=2000, noise=0.01,
                                         sync="epoch"),
                "fan2d_curved 512x512 as fan2d_512, fully parallel reading: r refreshed once per "
                "epoch, half of the column blocks per epoch (gamma 0.5), alpha 0.5, s 1")
    if name == "paper2d_64":
        return (inputs.config_paper2d(), dict(alpha=0.5, gamma=1.0, s=100, b=2.0, seed=6000,
                                              noise=0.01),
                "paper 2D setting: fan2d_flat 64x64 1mm, 360 views/360deg, 187 bins 1mm, SID 115 "
                "SDD 230, 720 row blocks (view x detector half) x 4 quadrants, alpha 0.5, s 100, b 2")
    if name == "paper3d_128":
        return (inputs.config_paper3d(), dict(alpha=0.5, gamma=1.0, s=90, b=1.0, seed=6200,
                                              noise=0.01),
                "paper 3D setting: cone3d_flat 128^3 over 32^3, 720 random views on a sphere of "
                "radius 66, 202^2 bins over 101^2, SDD 132, 720 row blocks (views) x 8 blocks, "
                "alpha 0.5, s 90, b 1")
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


def cpu_baseline(g, y, ex, budget_s=15.0, note=""):
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
            "sample": (f"{note}{epochs} epochs (schedule wrapped every {E}) of the same workload, "
                       f"schedule and y: {st.updates} updates in {t_run:.2f} s, scipy CSR "
                       f"matvecs on 1 thread; explicit FP64 A ({A.nnz} nnz) and its {g.m}x{g.n} "
                       f"sub-blocks built beforehand in {t_build:.1f} s, untimed"),
            "seconds": t_run}


def projector_outputs(ex, g, epochs):
    """Output elements written by the projector launches of the given epochs:
    the back-projection writes g_J once per group of a column step (|J| per
    group), the fused forward A x and A g for every ray of a group's row
    blocks."""
    vox = [int((b[1] - b[0]) * (b[3] - b[2]) * (b[5] - b[4])) for b in g.col_blocks]
    rays = [int(sum((t[2] - t[1]) * (t[4] - t[3]) for t in rb)) for rb in g.row_blocks]
    back = fwd = 0
    for e in epochs:
        for c in range(ex["epoch_col_ptr"][e], ex["epoch_col_ptr"][e + 1]):
            J = ex["cols"][c]
            for G in range(ex["col_group_ptr"][c], ex["col_group_ptr"][c + 1]):
                back += vox[J]
                for k in range(ex["group_rb_ptr"][G], ex["group_rb_ptr"][G + 1]):
                    fwd += 2 * rays[ex["rbs"][k]]
    return {"back": back, "fwd": fwd}


def cpu_baseline_matrix_free(g, y_np, ex, budget_s=15.0):
    """The FP64 oracle's matrix-free group step (rows of A regenerated by its
    Siddon row generator for every product, as a whole A of this size does
    not fit in memory), as it is, on a bounded sample of the same workload:
    the first group update of the schedule (J, its first group, beta; epoch
    start x = 0, r = y) on the rays of the group's first V views, V chosen so
    the run takes about ``budget_s``.  Run on the row generator's OpenMP
    threads (OMP_NUM_THREADS, else the affinity mask), then on one thread for
    one view."""
    from oracle import csgd, siddon
    c = ex["epoch_col_ptr"][0]
    J = int(ex["cols"][c])
    G0 = ex["col_group_ptr"][c]
    rbs = [int(t) for t in ex["rbs"][ex["group_rb_ptr"][G0]:ex["group_rb_ptr"][G0 + 1]]]
    beta = float(ex["beta"][G0])
    rows = np.concatenate([g.row_block_rays(I) for I in rbs])
    per_view = g.nu * g.nv
    x0 = np.zeros(g.n_vox)
    y64 = np.asarray(y_np, dtype=np.float64)
    aff = len(os.sched_getaffinity(0))
    want = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or aff

    def timed(nv, threads):
        used = siddon.set_threads(threads)
        t = time.perf_counter()
        _, _, _, nnz = csgd.step_group_matrix_free(g, rows[:nv * per_view], J, x0, y64, beta)
        return time.perf_counter() - t, nnz, used

    t1, _, _ = timed(1, want)                       # calibration: one view
    nv = int(max(1, min(len(rows) // per_view, budget_s / max(t1, 1e-3))))
    t_all, nnz_all, used = timed(nv, want)
    t_one, nnz_one, _ = timed(1, 1)
    siddon.set_threads(want)
    return {"value": 2 * nnz_all / t_all, "unit": "ray-voxel updates/s", "cores": used,
            "kind": "oracle",
            "sample": (f"matrix-free FP64 oracle group step on the same geometry, y and schedule: "
                       f"column block {J}, its first group (row blocks {rbs}, beta {beta:.4g}), "
                       f"x = 0, r = y, restricted to the rays of the group's first {nv} of "
                       f"{len(rows) // per_view} views ({nv * per_view} rays, {nnz_all} pairs in J); "
                       f"A's rows regenerated by the C Siddon generator for g = A^T r and again "
                       f"for A g and A x_J; {2 * nnz_all} updates in {t_all:.2f} s on {used} "
                       f"OpenMP threads (affinity mask: {aff} CPUs)"),
            "seconds": t_all,
            "one_thread": {"value": 2 * nnz_one / t_one, "cores": 1, "seconds": t_one,
                           "sample": f"the same step on the group's first view ({per_view} rays, "
                                     f"{nnz_one} pairs in J) on one thread"}}


def roofline_of(kt, prof_updates, outputs, workload=None):
    """Roofline object of the dominant kernel from per-class (ms, launches).

    Projectors: algorithmic bytes per launch = 4 B x (ray-voxel pairs +
    output elements), the stream an explicit-A sparse product of the same
    block would need; achieved = those bytes / the average launch time."""
    dom = max(kt, key=lambda k: kt[k][0])
    dom_ms, dom_n = kt[dom]
    avg_ms = dom_ms / max(dom_n, 1)
    if dom not in ("back", "fwd"):
        return {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": None, "traffic": None, "kernel": dom}
    pairs = prof_updates / 2 / dom_n            # ray-voxel pairs handled by one launch
    outs = outputs[dom] / dom_n
    alg = GATHER_BYTES * (pairs + outs)
    gbs = alg / (avg_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": None, "kernel": dom,
            "avg_launch_ms": round(avg_ms, 5), "launches": dom_n,
            "pairs_per_launch": pairs, "outputs_per_launch": outs,
            "algorithmic_bytes_per_launch": alg,
            "model": "4 B per ray-voxel pair + 4 B per output element (gather-equivalent)"}
    c = COUNTERS.get((workload, dom))
    if c is not None:
        roof["traffic"] = (c["fetch"] * PMC_FETCH_SCALE + c["write"] * PMC_WRITE_SCALE) * 1024.0
        roof["traffic_note"] = (f"measured HBM bytes per launch (FETCH_SIZE x {PMC_FETCH_SCALE} + "
                                f"WRITE_SIZE x {PMC_WRITE_SCALE}), {c['profile']}")
        if c.get("valu"):
            roof["valu"] = {"wave_instructions_per_launch": c["valu"],
                            "lane_instructions_per_pair": round(c["valu"] * 64 / pairs, 2),
                            "busy_frac": round(c["valu"] * 4 / (N_SIMD * CLOCK_HZ) /
                                               (avg_ms * 1e-3), 4),
                            "note": "SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x 2.4 GHz) over the "
                                    "launch time: the fraction of the VALU issue ceiling used"}
    return roof


def make_y(ct, inputs, G, g, cfg, seed):
    """y from the validated GPU projector: A x_true plus the workload's noise."""
    import torch
    # the small parallel-beam workload names 10 ellipses; the other 2D cases 12
    n_ell = 10 if g.kind == inputs.PAR2D else None
    xt = torch.as_tensor(inputs.phantom_for(g, seed, n_ell=n_ell).astype(np.float32), device="cuda")
    p = torch.zeros(G.M, device="cuda")
    for J in range(G.n):
        ct.ct_block_fwd(G, list(range(G.m)), J, xt, p, flags=ct.CT_ACCUMULATE if J else 0)
    pn = p.cpu().numpy().astype(np.float64)
    del p, xt
    if "photons" in cfg:
        y_np = inputs.poisson_noise(pn, cfg["photons"], seed)
    else:
        y_np = inputs.gaussian_noise(pn, cfg["noise"], seed)
    return y_np, torch.as_tensor(y_np, device="cuda")


def base_record(args, metric_value, ms_total, steps, dtype="f32"):
    return {
        "metric": "ray-voxel updates/s (fwd+back)",
        "value": metric_value,
        "unit": "ray-voxel updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_total / max(steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
    }


def run_single(args):
    import torch
    from paper_1709_00953_amd import ct, inputs

    g, cfg, desc = single_workload(args.workload)
    t_setup = time.perf_counter()
    G = ct.ct_geom_create(g)
    tau = 1e-5 * min(g.vx, g.vy)
    y_np, y = make_y(ct, inputs, G, g, cfg, cfg["seed"])
    nnz = ct.ct_geom_block_nnz(G, tau)
    E = args.warmup + args.steps
    # epochs [0, W) warm up, [W, E) are timed, [E, E + K) are replayed with a
    # HIP event pair around every kernel for the per-kernel durations
    params = ct.sched_params(E + args.steps, cfg["alpha"], cfg["gamma"], cfg["s"], cfg["b"],
                             seed=cfg["seed"])
    sched = ct.ct_schedule_create(G, params, nnz)
    ex = ct.ct_schedule_export(sched)
    upd = updates_per_epoch(ex, nnz)
    # launch shapes of the projectors, timed once per size class (set-up)
    t_tune = time.perf_counter()
    shape = ct.ct_geom_tune(G, sched)
    t_tune = time.perf_counter() - t_tune
    sol = ct.ct_solver_create(G, ct.CT_SYNC_EPOCH if cfg.get("sync") == "epoch" else ct.CT_SYNC_COLUMN)
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
    out = base_record(args, timed_updates / (ms * 1e-3), ms, args.steps)
    roof = roofline_of(kt, prof_updates, projector_outputs(ex, g, range(E, E + args.steps)),
                       args.workload)
    out["config"] = {"workload": desc, "epoch_updates": upd[args.warmup], "b": cfg["b"],
                     "rel_residual_after": rel, "setup_s": round(t_setup, 3),
                     "launch_shape": {"fwd_split": shape["fwd_split"], "back_waves": shape["back_waves"],
                                      "tuned_ms_per_epoch": round(shape["ms"], 4),
                                      "default_ms_per_epoch": round(shape["ms_default"], 4)},
                     "tune_s": round(t_tune, 3)}
    out["roofline"] = roof
    out["kernels_ms"] = {k: round(v[0], 4) for k, v in kt.items()}
    out["kernels_note"] = "per-kernel HIP-event times from the same number of epochs run right after the timed ones"
    out["kernels_launches"] = {k: v[1] for k, v in kt.items()}
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        if g.is3d:
            # the explicit FP64 A of the full volume does not fit in memory:
            # the oracle's matrix-free mode on the same geometry, y, schedule
            out["cpu_baseline"] = cpu_baseline_matrix_free(g, y_np, ex, args.cpu_budget)
        else:
            out["cpu_baseline"] = cpu_baseline(g, y_np, ex, args.cpu_budget)
    return out


def run_batch(args):
    """64 uneven fan slices: every job solved one at a time with ct_block_epoch,
    then all of them advanced together by the batched launches (HIP graph)."""
    import torch
    from paper_1709_00953_amd import ct, inputs

    n_jobs, E, b = args.jobs, args.steps, 1.0
    rng = np.random.default_rng(4000)
    sizes = [int(v) for v in rng.choice(BATCH_SIZES, size=n_jobs)]
    t_setup = time.perf_counter()
    jobs = []
    for k, N in enumerate(sizes):
        g = inputs.slice_fan(N)
        G = ct.ct_geom_create(g)
        seed = inputs.seed_for(4, k)
        y_np, y = make_y(ct, inputs, G, g, {"noise": 0.01}, seed)
        nnz = ct.ct_geom_block_nnz(G, 1e-5 * g.vx)
        sched = ct.ct_schedule_create(G, ct.sched_params(E, 1.0, 1.0, 2, b, seed=seed), nnz)
        ex = ct.ct_schedule_export(sched)
        sol = ct.ct_solver_create(G)
        x = torch.zeros(G.N, device="cuda")
        jobs.append(dict(N=N, g=g, G=G, y=y, y_np=y_np, sched=sched, ex=ex, sol=sol, x=x,
                         upd=sum(updates_per_epoch(ex, nnz))))
        if k == 0 or (k + 1) % 16 == 0:
            print(f"[bench] job {k + 1}/{n_jobs} ready (N={N})", file=sys.stderr, flush=True)
    total_updates = sum(j["upd"] for j in jobs)

    def reset_all():
        for j in jobs:
            j["x"].zero_()
            ct.ct_solver_reset(j["sol"], j["y"])

    # warm-up: first use uploads each schedule's device tables
    reset_all()
    for j in jobs:
        ct.ct_block_epoch(j["sol"], j["sched"], 0, j["y"], j["x"])
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup

    # launch shapes: the tuner times each size class of the mix once; the jobs'
    # geometries take the batch's choice, so the one-at-a-time runs below use
    # the same shapes as the batched ones
    t_tune = time.perf_counter()
    Bt = ct.ct_batch_create(n_jobs)
    tids = [ct.ct_batch_add(Bt, j["sol"], j["sched"], j["y"], j["x"]) for j in jobs]
    shapes = ct.ct_batch_tune(Bt)
    for t in tids:
        ct.ct_batch_remove(Bt, t)
    del Bt
    t_tune = time.perf_counter() - t_tune

    def set_shapes(batch):
        for kind, t in enumerate(shapes):
            if t is not None:
                ct.ct_batch_set_tuning(batch, kind, t["fwd_split"], t["back_waves"])

    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)

    # one job at a time
    reset_all()
    torch.cuda.synchronize()
    start.record()
    for j in jobs:
        for e in range(E):
            ct.ct_block_epoch(j["sol"], j["sched"], e, j["y"], j["x"])
    stop.record()
    torch.cuda.synchronize()
    ms_plain = start.elapsed_time(stop)
    x_plain = [j["x"].clone() for j in jobs]
    res_plain = [ct.ct_true_residual(j["sol"], j["y"], j["x"]) for j in jobs]

    # batched, replayed from a HIP graph (building the batch table and the
    # graph is inside the timed region)
    reset_all()
    torch.cuda.synchronize()
    start.record()
    B = ct.ct_batch_create(n_jobs)
    set_shapes(B)
    for j in jobs:
        ct.ct_batch_add(B, j["sol"], j["sched"], j["y"], j["x"])
    for e in range(E):
        ct.ct_batch_epoch(B, graph=True)
    stop.record()
    torch.cuda.synchronize()
    ms_batch = start.elapsed_time(stop)
    same = all(torch.equal(a, j["x"]) for a, j in zip(x_plain, jobs))
    res_batch = [ct.ct_true_residual(j["sol"], j["y"], j["x"]) for j in jobs]

    # per-kernel replay of the batched epochs with events
    reset_all()
    B2 = ct.ct_batch_create(n_jobs)
    set_shapes(B2)
    for j in jobs:
        ct.ct_batch_add(B2, j["sol"], j["sched"], j["y"], j["x"])
    ct.ct_batch_profile(B2, True)
    for e in range(E):
        ct.ct_batch_epoch(B2)
    kt = ct.ct_batch_profile_read(B2)
    outs = {"back": 0, "fwd": 0}
    for j in jobs:
        o = projector_outputs(j["ex"], j["g"], range(E))
        outs["back"] += o["back"]
        outs["fwd"] += o["fwd"]
    roof = roofline_of(kt, total_updates, outs)

    out = base_record(args, total_updates / (ms_batch * 1e-3), ms_batch, E)
    out["config"] = {
        "workload": (f"{n_jobs} fan2d_curved slices, N drawn from {list(BATCH_SIZES)} (seed 4000), "
                     "pixel 256/N mm, 1.5N views/360deg, 1.5N bins over 0.768 rad, 4 view groups x "
                     "4 quadrants, alpha 1, s 2, b 1, 1% noise, epochs = steps"),
        "sizes": sizes, "total_updates": total_updates, "setup_s": round(t_setup, 3),
        "launch_shapes": {("par2d", "fan2d_flat", "fan2d_curved", "cone3d")[k]: t for k, t in enumerate(shapes)
                          if t is not None},
        "tune_s": round(t_tune, 3)}
    out["jobs_per_s"] = n_jobs / (ms_batch * 1e-3)
    out["plain"] = {"value": total_updates / (ms_plain * 1e-3), "ms": ms_plain,
                    "jobs_per_s": n_jobs / (ms_plain * 1e-3),
                    "mean_rel_residual": float(np.mean(res_plain))}
    out["batched_ms"] = ms_batch
    out["speedup_vs_plain"] = ms_plain / ms_batch
    out["mean_rel_residual"] = float(np.mean(res_batch))
    out["identical_to_plain"] = bool(same)
    out["roofline"] = roof
    out["kernels_ms"] = {k: round(v[0], 4) for k, v in kt.items()}
    out["kernels_launches"] = {k: v[1] for k, v in kt.items()}
    out["kernels_note"] = "batched launches timed with HIP events in a replay of the same epochs"
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        small = min(range(n_jobs), key=lambda k: sizes[k])
        j = jobs[small]
        out["cpu_baseline"] = cpu_baseline(j["g"], j["y_np"], j["ex"], args.cpu_budget,
                                           note=f"smallest slice of the mix (N={j['N']}): ")
    return out


def serve_stream(n_jobs, seed=5000, rate=40.0):
    """Arrival times and job kinds of the mixed serving stream."""
    rng = np.random.default_rng(seed)
    arr = np.cumsum(rng.exponential(1.0 / rate, n_jobs))
    out = []
    for k in range(n_jobs):
        if rng.random() < 0.7:
            out.append((float(arr[k]), "fan", int(rng.choice(SERVE_FAN)), int(rng.integers(2))))
        else:
            out.append((float(arr[k]), "cone", int(rng.choice(SERVE_CONE)), int(rng.integers(2))))
    return out


def run_serve(args):
    """The same Poisson stream served with the continuous-batching server
    (capacity C) and one job at a time (capacity 1).  Noise-free jobs, stop at
    true relative residual 1e-3 (checked every 10 epochs) or 500 epochs.

    Latency is measured on a stream the server drains: the first ``jobs``
    arrivals, every one run to completion in both modes, p50 / p99 over all of
    them (arrival to result).  The offered load of 40 jobs/s is far above what
    one GPU completes, so the overload figure (a fixed window of the full
    stream, with the queue left at its end) is reported separately."""
    import torch
    from paper_1709_00953_amd import ct, inputs

    n_all = max(args.jobs, 1000)
    stream = serve_stream(n_all)
    geo, pool = {}, {}
    t_setup = time.perf_counter()
    for _, kind, N, ph in stream:
        key = (kind, N)
        if key not in geo:
            geo[key] = inputs.slice_fan(N) if kind == "fan" else inputs.slice_cone(N)
        if (kind, N, ph) not in pool:
            g = geo[key]
            G = ct.ct_geom_create(g)
            xt = torch.as_tensor(inputs.phantom_for(g, inputs.seed_for(5, 100 * len(pool) + ph))
                                 .astype(np.float32), device="cuda")
            p = torch.zeros(G.M, device="cuda")
            for J in range(G.n):
                ct.ct_block_fwd(G, list(range(G.m)), J, xt, p, flags=ct.CT_ACCUMULATE if J else 0)
            pool[(kind, N, ph)] = p.cpu().numpy()
            del G, xt, p
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    print(f"[bench] serve: {len(pool)} distinct measurement sets ready in {t_setup:.1f} s",
          file=sys.stderr, flush=True)

    def params_of(i, kind):
        return (ct.sched_params(500, 1.0, 1.0, 4, 1.0, seed=inputs.seed_for(5, i)) if kind == "fan"
                else ct.sched_params(500, 1.0, 1.0, 3, 2.0, seed=inputs.seed_for(5, i)))

    def serve(capacity, n_jobs, window=None):
        # density threshold: 1e-5 of the smallest voxel pitch in the mix (0.25 mm)
        srv = ct.ct_server_create(capacity=capacity, hbm_budget=0, rel_tol=1e-3, check_every=10,
                                  tau=2.5e-6, graph=True)
        done, i, st = [], 0, None
        queue_len = []
        t0 = time.perf_counter()
        last = t0
        while True:
            now = time.perf_counter() - t0
            if window is not None and now >= window:
                break
            if window is None and len(done) >= n_jobs:
                break
            while i < n_jobs and stream[i][0] <= now:
                _, kind, N, ph = stream[i]
                ct.ct_server_submit(srv, geo[(kind, N)], params_of(i, kind), pool[(kind, N, ph)], tag=i)
                i += 1
            st = ct.ct_server_tick(srv)
            done += ct.ct_server_poll(srv)
            queue_len.append(st["queued"])
            if st["active"] == 0 and st["queued"] == 0 and i < n_jobs:
                time.sleep(max(0.0, min(0.01, stream[i][0] - (time.perf_counter() - t0))))
            if time.perf_counter() - last > 10:
                last = time.perf_counter()
                print(f"[bench] serve cap {capacity}: t={now:.0f}s submitted {i} active "
                      f"{st['active']} queued {st['queued']} done {len(done)}",
                      file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        upd = st["updates"] if st else 0
        lat = np.array([d["t_done"] - d["t_submit"] for d in done])
        wait = np.array([d["t_admit"] - d["t_submit"] for d in done])
        conv = sum(1 for d in done if d["status"] == ct.CT_OK)
        res = {"capacity": capacity, "wall_s": round(wall, 3), "submitted": i,
               "completed": len(done), "converged": conv,
               "jobs_per_s": len(done) / wall,
               "updates_per_s": upd / wall,
               "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
               "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
               "p50_queue_wait_s": float(np.percentile(wait, 50)) if len(wait) else None,
               "mean_epochs": float(np.mean([d["epochs"] for d in done])) if done else None,
               "max_rel_residual": float(max(d["rel_residual"] for d in done)) if done else None,
               "still_active": st["active"] if st else 0, "still_queued": st["queued"] if st else 0,
               "max_queue": int(max(queue_len)) if queue_len else 0}
        del srv
        return res

    n_drain = args.jobs
    served = serve(args.capacity, n_drain)
    plain = serve(1, n_drain)
    overload = serve(args.capacity, n_all, window=args.window) if args.window > 0 else None
    out = base_record(args, served["updates_per_s"], served["wall_s"] * 1e3, 1)
    out["config"] = {
        "workload": (f"the first {n_drain} arrivals of a Poisson stream, mean 40 jobs/s (seed 5000), "
                     f"every job run to completion: 70% fan slices N in {list(SERVE_FAN)} (4x4 blocks, "
                     f"alpha 1, s 4, b 1), 30% cone N in {list(SERVE_CONE)} (360 views of (1.5N)^2, "
                     "12x8 blocks, alpha 1, s 3, b 2), noise-free y from one of 2 seeded phantoms per "
                     "size, stop at true rel. residual 1e-3 (checked every 10 epochs) or 500 epochs, "
                     "HBM budget 80% of free"),
        "setup_s": round(t_setup, 3)}
    out["served"] = served
    out["plain"] = plain
    out["overload_window"] = overload
    out["jobs_per_s"] = served["jobs_per_s"]
    out["p50_latency_s"] = served["p50_latency_s"]
    out["p99_latency_s"] = served["p99_latency_s"]
    out["speedup_vs_plain"] = plain["wall_s"] / served["wall_s"]
    out["roofline"] = None
    out["cpu_baseline"] = None
    return out


def run_copy(args):
    """A plain 256 MiB device-to-device copy (torch), three times: the
    reference for scaling the HBM byte counters and a measured bandwidth."""
    import torch
    n = 64 * 1024 * 1024
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(3):
        b.copy_(a)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / 3
    gbs = 2 * 4 * n / (ms * 1e-3) / 1e9
    return {"metric": "device copy bandwidth (read + write)", "value": gbs, "unit": "GB/s",
            "n_gpus": 1, "steps": 3, "warmup": 1, "ms_per_step": ms, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "256 MiB float32 copy"},
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "traffic": 2 * 4 * n},
            "cpu_baseline": None}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cone3d_256",
                    choices=["fan2d_512", "par2d_64", "cone3d_256", "fan2d_512_parallel", "paper2d_64",
                             "paper3d_128", "batch64", "serve40",
                             "copy256"])
    ap.add_argument("--jobs", type=int, default=None,
                    help="batch64: slices (64); serve40: arrivals run to completion (48)")
    ap.add_argument("--window", type=float, default=15.0,
                    help="serve40: seconds of the overload run over the full stream (0: none)")
    ap.add_argument("--capacity", type=int, default=16, help="serve40: resident jobs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: the solver runs on one GPU only (asked for {max(args.gpus, world)}); "
              "sharding the column blocks across GPUs is not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.workload == "batch64":
        args.jobs = args.jobs or 64
        out = run_batch(args)
    elif args.workload == "copy256":
        out = run_copy(args)
    elif args.workload == "serve40":
        args.jobs = args.jobs or 48
        out = run_serve(args)
    else:
        out = run_single(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
