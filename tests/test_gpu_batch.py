"""Batched epochs: every job of a batch must produce exactly (bit for bit) what
the same job produces alone with ct_block_epoch, eagerly and when the batch
epoch is replayed from a HIP graph, while jobs join and leave between epochs.
One batch member is also checked against the FP64 oracle to the 1e-4
reconstruction tolerance.
"""
import numpy as np
import pytest

from oracle import csgd, sampler
from paper_1709_00953_amd import inputs
from tests.parity_util import GEOMS, phantom_y, rel_l2, system, tau_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ct():
    from paper_1709_00953_amd import ct as _ct
    _ct.lib()
    return _ct


# (name, geometry builder, sync, sampling, alpha, s, b, epochs, first epoch)
JOBS = [
    ("c1_par2d", GEOMS["c1_par2d"], "column", "density", 0.5, 1, 0.5, 6, 0),
    ("fan_curved", GEOMS["fan_curved"], "epoch", "density", 1.0, 2, 1.0, 4, 0),
    ("fan_flat", GEOMS["fan_flat"], "column", "mixed", 0.6, 2, 1.0, 5, 1),
    ("cone", GEOMS["cone"], "column", "density", 1.0, 3, 1.0, 3, 0),
    ("slice32", lambda: inputs.slice_fan(32), "column", "density", 1.0, 2, 1.0, 5, 0),
    ("slice48", lambda: inputs.slice_fan(48), "epoch", "uniform", 0.5, 1, 0.5, 4, 0),
    ("slice80", lambda: inputs.slice_fan(80), "column", "density", 1.0, 2, 1.0, 6, 2),
    ("fan_fine", GEOMS["fan_fine"], "column", "density", 0.5, 2, 1.0, 4, 0),
]


class Job:
    """One reconstruction: geometry, schedule, y, and two independent
    solver states (one run alone, one in a batch)."""

    def __init__(self, ct, spec, seed):
        name, build, sync, sampling, alpha, s, b, epochs, first = spec
        self.name, self.first, self.epochs = name, first, epochs
        g = build()
        self.g = g
        self.G = ct.ct_geom_create(g)
        xt = torch.as_tensor(inputs.phantom_for(g, seed).astype(np.float32), device="cuda")
        p = torch.zeros(self.G.M, device="cuda")
        for J in range(self.G.n):
            ct.ct_block_fwd(self.G, list(range(self.G.m)), J, xt, p,
                            flags=ct.CT_ACCUMULATE if J else 0)
        y = inputs.gaussian_noise(p.cpu().numpy().astype(np.float64), 0.01, seed)
        self.y = torch.as_tensor(y, device="cuda")
        nnz = ct.ct_geom_block_nnz(self.G, tau_for(g))
        smp = {"density": ct.CT_SAMPLE_DENSITY, "uniform": ct.CT_SAMPLE_UNIFORM,
               "mixed": ct.CT_SAMPLE_MIXED}[sampling]
        self.sched = ct.ct_schedule_create(
            self.G, ct.sched_params(epochs, alpha, 1.0, s, b, sampling=smp, seed=seed,
                                    theta_step=0.25), nnz)
        self.sync = ct.CT_SYNC_EPOCH if sync == "epoch" else ct.CT_SYNC_COLUMN
        self.alone = self._state(ct)
        self.batched = self._state(ct)

    def _state(self, ct):
        sol = ct.ct_solver_create(self.G, self.sync)
        x = torch.zeros(self.G.N, device="cuda")
        ct.ct_solver_reset(sol, self.y)
        return sol, x

    def run_alone(self, ct, e):
        sol, x = self.alone
        ct.ct_block_epoch(sol, self.sched, e, self.y, x)

    def assert_same(self, ct, what):
        torch.cuda.synchronize()
        (sa, xa), (sb, xb) = self.alone, self.batched
        za, ra = ct.ct_solver_state(sa)
        zb, rb = ct.ct_solver_state(sb)
        for nm, a, b in (("x", xa, xb), ("z", za, zb), ("r", ra, rb)):
            assert torch.equal(a, b), (
                f"{what}: job {self.name} {nm} differs, max |diff| "
                f"{(a - b).abs().max().item():.3e}")


def _make_jobs(ct, specs):
    jobs = []
    for k, spec in enumerate(specs):
        print(f"[batch] building job {spec[0]}", flush=True)
        jobs.append(Job(ct, spec, 4000 + k))
    return jobs


@pytest.mark.parametrize("graph,shapes", [(False, None), (True, None), (True, "tuned"), (False, "forced"),
                                          (True, "wide")])
def test_batch_matches_alone(ct, graph, shapes):
    """shapes: the default launch shapes; the tuner's (the jobs' geometries
    take the batch's choice); or forced ones set on the batch and the
    geometries alike (one piece per chord and two waves per 2D tile, or two
    pieces and sixteen waves)."""
    jobs = _make_jobs(ct, JOBS)
    B = ct.ct_batch_create(len(jobs))
    ids = {}
    for j in jobs:
        sol, x = j.batched
        ids[j.name] = ct.ct_batch_add(B, sol, j.sched, j.y, x, epoch=j.first)
    if shapes == "tuned":
        chosen = ct.ct_batch_tune(B)
        print(f"[batch] tuned shapes {chosen}", flush=True)
        for j in jobs:
            t = ct.ct_geom_get_tuning(j.G)
            c = chosen[j.g.kind]
            assert (t["fwd_split"], t["back_waves"]) == (c["fwd_split"], c["back_waves"])
    elif shapes in ("forced", "wide"):
        split, waves = (1, 2) if shapes == "forced" else (2, 16)
        for kind in range(4):
            ct.ct_batch_set_tuning(B, kind, split, 4 if kind == 3 else waves)
        for j in jobs:
            ct.ct_geom_set_tuning(j.G, split, 4 if j.g.kind == 3 else waves)
    done = {j.name: j.first for j in jobs}
    it = 0
    while True:
        print(f"[batch] graph={graph} shapes={shapes} batch epoch {it}", flush=True)
        ran = ct.ct_batch_epoch(B, graph=graph)
        expect = sum(1 for j in jobs if done[j.name] < j.epochs)
        assert ran == expect
        if ran == 0:
            break
        # the same epoch of every unfinished job, alone (eager work between replays)
        for j in jobs:
            if done[j.name] < j.epochs:
                j.run_alone(ct, done[j.name])
                done[j.name] += 1
            assert ct.ct_batch_job_epoch(B, ids[j.name]) == done[j.name]
        for j in jobs:
            j.assert_same(ct, f"batch epoch {it}")
        it += 1
    assert it == max(j.epochs - j.first for j in jobs)


def test_batch_join_and_leave(ct):
    """Continuous batching: jobs join at a later batch epoch and leave before
    their schedule ends; every member still matches its solo run."""
    specs = [JOBS[0], JOBS[4], JOBS[5], JOBS[1]]
    jobs = _make_jobs(ct, specs)
    B = ct.ct_batch_create(3)
    ids, done = {}, {}

    def join(j):
        sol, x = j.batched
        ids[j.name] = ct.ct_batch_add(B, sol, j.sched, j.y, x, epoch=j.first)
        done[j.name] = j.first

    join(jobs[0])
    join(jobs[1])
    plan = {1: ("join", jobs[2]), 2: ("leave", jobs[1]), 3: ("join", jobs[3])}
    for it in range(6):
        if it in plan:
            act, j = plan[it]
            if act == "join":
                join(j)
            else:
                ct.ct_batch_remove(B, ids.pop(j.name))
        print(f"[batch] join/leave epoch {it}: members {sorted(ids)}", flush=True)
        ct.ct_batch_epoch(B, graph=(it % 2 == 1))
        for j in jobs:
            if j.name in ids and done[j.name] < j.epochs:
                j.run_alone(ct, done[j.name])
                done[j.name] += 1
        for j in jobs:
            if j.name in done:
                j.assert_same(ct, f"join/leave epoch {it}")
    with pytest.raises(ct.CtError):
        ct.ct_batch_remove(B, 12345)


def test_batch_member_matches_oracle(ct):
    """A C1 job run inside a batch next to other jobs, against the FP64 oracle
    on the same imported schedule."""
    g, S = system("c1_par2d")
    x_true, y = phantom_y(g, S, 1000)
    P = sampler.density(S.nnz_table(tau_for(g)))
    sch = sampler.make_schedule(P, 10, 0.5, 1.0, 1, 0.5, 1000)
    ref = csgd.run(S, y.astype(np.float64), sch)
    G = ct.ct_geom_create(g)
    yd = torch.as_tensor(y, device="cuda")
    sol = ct.ct_solver_create(G)
    x = torch.zeros(G.N, device="cuda")
    ct.ct_solver_reset(sol, yd)
    sc = ct.ct_schedule_import(G, sch)
    others = _make_jobs(ct, [JOBS[4], JOBS[3]])
    B = ct.ct_batch_create(4)
    ct.ct_batch_add(B, sol, sc, yd, x)
    for j in others:
        s2, x2 = j.batched
        ct.ct_batch_add(B, s2, j.sched, j.y, x2)
    for it in range(10):
        ct.ct_batch_epoch(B, graph=True)
    torch.cuda.synchronize()
    err = rel_l2(x.cpu().numpy(), ref.x)
    print(f"[batch] oracle parity of a batch member: {err:.2e}", flush=True)
    assert err <= 1e-4


def test_batch_argument_errors(ct):
    jobs = _make_jobs(ct, [JOBS[4]])
    j = jobs[0]
    B = ct.ct_batch_create(1)
    sol, x = j.batched
    with pytest.raises(ct.CtError):
        ct.ct_batch_add(B, sol, j.sched, j.y, x, epoch=j.epochs + 1)
    ct.ct_batch_add(B, sol, j.sched, j.y, x)
    with pytest.raises(ct.CtError):             # full, and solver already a member
        ct.ct_batch_add(B, sol, j.sched, j.y, x)
    with pytest.raises(ct.CtError):
        ct.ct_batch_create(0)
    ct.ct_batch_set_tuning(B, 2, 1, 2)
    for kind, split, waves in ((3, 1, 2), (4, 1, 4), (2, 3, 4), (0, 4, 32), (3, 2, 16)):
        with pytest.raises(ct.CtError):             # 3D takes 4 waves; unknown kind; bad shapes
            ct.ct_batch_set_tuning(B, kind, split, waves)
