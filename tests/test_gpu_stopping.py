"""The stopping quantity and the whole solve against the FP64 oracle.

The tracked residual r of the method is an approximation (Sec. II-B), so a
solve stops on the true relative residual ||y - A x|| / ||y|| (reading C16).
Here the library's value (synchronous ``ct_true_residual`` and asynchronous
``ct_residual_norms``) is compared with the oracle's on the same float32 x,
and ``ct_solve``'s x, stopping value and per-epoch ||r|| with the oracle's
run of the same schedule.

Bound on the residual: the float32 forward projection differs from the
oracle's A x by at most ~1e-6 of ||A x|| (the projector parity), so the
relative residual may differ by 1e-6 max(rho, ||A x|| / ||y||).
"""
import numpy as np
import pytest

from oracle import csgd, sampler
from tests.parity_util import phantom_y, rel_l2, system, tau_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ct():
    from paper_1709_00953_amd import ct as _ct
    _ct.lib()
    return _ct


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def rho_bound(S, y, x, rho):
    ax = np.linalg.norm(S.A @ x)
    return 1e-6 * max(rho, ax / np.linalg.norm(y))


@pytest.mark.parametrize("name", ["c1_par2d", "fan_curved", "fan_split", "cone"])
def test_true_residual_matches_oracle(ct, name):
    g, S = system(name)
    G = ct.ct_geom_create(g)
    x_true, y = phantom_y(g, S, 4100)
    yd = dev(y)
    sol = ct.ct_solver_create(G)
    rng = np.random.default_rng(4101)
    # a far point, and a near one (the oracle's x after a few epochs)
    P = sampler.density(S.nnz_table(tau_for(g)))
    sch = sampler.make_schedule(P, 6, 1.0, 1.0, 2, 1.0, 4102)
    near = csgd.run(S, y.astype(np.float64), sch).x
    for label, x in (("far", rng.uniform(0, 0.2, g.n_vox)), ("near", near)):
        x32 = x.astype(np.float32)
        ref = csgd.true_rel_residual(S, y.astype(np.float64), x32.astype(np.float64))
        got = ct.ct_true_residual(sol, yd, dev(x32))
        out = torch.zeros(2, dtype=torch.float64, device="cuda")
        ct.ct_residual_norms(sol, yd, dev(x32), out)
        a, b = out.cpu().numpy()
        bound = rho_bound(S, y.astype(np.float64), x32.astype(np.float64), ref)
        print(f"[stop] {name} {label}: rho {ref:.6e} gpu {got:.6e} |d| {abs(got - ref):.2e} "
              f"(bound {bound:.2e})", flush=True)
        assert abs(got - ref) <= bound
        assert abs(np.sqrt(a / b) - ref) <= bound
        assert b == pytest.approx(float(np.sum(y.astype(np.float64) ** 2)), rel=1e-12)


@pytest.mark.parametrize("name,E,alpha,s,b,sync,seed", [
    ("c1_par2d", 21, 0.5, 1, 0.5, "column", 4200),
    ("fan_curved", 12, 1.0, 2, 1.0, "epoch", 4201),
    ("cone", 6, 1.0, 3, 1.0, "column", 4202),
])
def test_solve_matches_oracle(ct, name, E, alpha, s, b, sync, seed):
    """ct_solve with a cap and an unreachable tolerance runs exactly E epochs
    of the schedule ct_schedule_create draws from the density table; the
    oracle runs the same schedule (the samplers agree bit for bit and the
    density tables exactly)."""
    g, S = system(name)
    G = ct.ct_geom_create(g)
    _, y = phantom_y(g, S, seed)
    mode = ct.CT_SYNC_COLUMN if sync == "column" else ct.CT_SYNC_EPOCH
    params = ct.sched_params(E, alpha, 1.0, s, b, seed=seed)
    xd = torch.full((G.N,), 5.0, device="cuda")          # ct_solve starts from zero
    rc, st = ct.ct_solve(G, params, dev(y), xd, sync=mode, tau=tau_for(g), rel_tol=0.0,
                         check_every=3)
    assert rc == ct.CT_NOT_CONVERGED and st["epochs_run"] == E
    P = sampler.density(S.nnz_table(tau_for(g)))
    sch = sampler.make_schedule(P, E, alpha, 1.0, s, b, seed)
    state = csgd.State(S, y.astype(np.float64))
    r_ref = []
    for e in range(E):
        csgd.epoch(state, sch, e, sync)
        r_ref.append(np.linalg.norm(state.r))
    x = xd.cpu().numpy().astype(np.float64)
    err = rel_l2(x, state.x)
    print(f"[solve] {name}: x rel {err:.2e}", flush=True)
    assert err <= 1e-4
    # the last check (epoch E, a multiple of 3 here) against the oracle's true residual
    assert E % 3 == 0
    ref = csgd.true_rel_residual(S, y.astype(np.float64), state.x)
    assert abs(st["rel_residual"] - ref) <= 1e-4 * max(ref, 1.0)
    # per-epoch norm of the tracked residual: r within 1e-4 ||y|| of the oracle's
    yn = np.linalg.norm(y.astype(np.float64))
    assert st["r_norm"].shape == (E,)
    assert np.all(np.abs(st["r_norm"] - np.array(r_ref)) <= 1e-4 * yn)


def test_solve_argument_errors(ct):
    g, S = system("c1_par2d")
    G = ct.ct_geom_create(g)
    params = ct.sched_params(3, 0.5, 1.0, 1, 0.5, seed=1)
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(ct.CtError):
        ct.ct_solve(G, params, torch.zeros(G.M, device="cuda"), torch.zeros(G.N, device="cuda"),
                    workspace=small)
