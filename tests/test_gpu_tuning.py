"""Launch shapes of the projectors (pieces per chord of the fused forward,
waves per 2D back-projection tile) and their tuner.  Every shape computes the
same products up to the order of float32 sums, so each is held to the oracle
at the usual tolerances; the tuner must pick one of the candidates, never a
slower one than the default by its own timing, and reuse its cached table.
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


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def shapes(g):
    waves = (4,) if g.is3d else (1, 2, 4, 8, 16)
    return [(s, w) for s in (1, 2, 4) for w in waves]


@pytest.mark.parametrize("name", ["c1_par2d", "fan_curved", "fan_flat", "cone"])
def test_every_shape_matches_oracle(ct, name):
    g, S = system(name)
    G = ct.ct_geom_create(g)
    x_true, y = phantom_y(g, S, 5100)
    P = sampler.density(S.nnz_table(tau_for(g)))
    sch = sampler.make_schedule(P, 4, 1.0, 1.0, 2, 1.0, 5100)
    ref = csgd.run(S, y.astype(np.float64), sch)
    sc = ct.ct_schedule_import(G, sch)
    rng = np.random.default_rng(5101)
    r = rng.normal(0.0, 1.0, g.n_rays).astype(np.float32)
    rbs, J = [0, g.m - 1], g.n - 1
    refb = csgd.block_back(S, rbs, J, r.astype(np.float64))
    for split, waves in shapes(g):
        print(f"[shape] {name} fwd_split={split} back_waves={waves}", flush=True)
        ct.ct_geom_set_tuning(G, split, waves)
        assert ct.ct_geom_get_tuning(G)["fwd_split"] == split
        sol = ct.ct_solver_create(G)
        yd, xd = dev(y), torch.zeros(G.N, device="cuda")
        ct.ct_solver_reset(sol, yd)
        for e in range(4):
            ct.ct_block_epoch(sol, sc, e, yd, xd)
        z, rr = ct.ct_solver_state(sol)
        assert rel_l2(host(xd), ref.x) <= 1e-4, (split, waves)
        assert rel_l2(host(z), ref.z) <= 1e-4, (split, waves)
        assert np.linalg.norm(host(rr) - ref.r) <= 1e-4 * np.linalg.norm(y)
        gd = torch.zeros(G.N, device="cuda")
        ct.ct_block_back(G, rbs, J, dev(r), gd)
        assert rel_l2(host(gd)[S.vox[J]], refb) <= 1e-5, (split, waves)


@pytest.mark.parametrize("name", ["fan_curved", "cone"])
def test_tuner_picks_a_candidate_and_caches(ct, name):
    g, S = system(name)
    G = ct.ct_geom_create(g)
    nnz = ct.ct_geom_block_nnz(G, tau_for(g))
    sc = ct.ct_schedule_create(G, ct.sched_params(1, 1.0, 1.0, 2, 1.0, seed=5200), nnz)
    t1 = ct.ct_geom_tune(G, sc, refresh=True)
    print(f"[tune] {name}: {t1}", flush=True)
    assert (t1["fwd_split"], t1["back_waves"]) in shapes(g)
    assert t1["trials"] == len(shapes(g)) and not t1["cached"]
    assert 0 < t1["ms"] <= t1["ms_default"]
    got = ct.ct_geom_get_tuning(G)
    assert (got["fwd_split"], got["back_waves"]) == (t1["fwd_split"], t1["back_waves"])
    # a second geometry of the same size class takes the cached table
    G2 = ct.ct_geom_create(g)
    sc2 = ct.ct_schedule_create(G2, ct.sched_params(1, 1.0, 1.0, 2, 1.0, seed=5201), nnz)
    t2 = ct.ct_geom_tune(G2, sc2)
    assert t2["cached"] and t2["trials"] == 0
    assert (t2["fwd_split"], t2["back_waves"]) == (t1["fwd_split"], t1["back_waves"])
