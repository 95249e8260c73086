"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Tolerances: relative L2 error <= 1e-5 for every projection call and <= 1e-4
on the reconstruction after a fixed epoch count on the same inputs and the
same imported block schedule; integer block densities within 1e-4.
"""
import numpy as np
import pytest

from oracle import csgd, sampler
from paper_1709_00953_amd import inputs
from tests.parity_util import GEOMS, max_rel, phantom_y, rel_l2, system, tau_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def ct():
    from paper_1709_00953_amd import ct as _ct
    _ct.lib()
    return _ct


def _pairs(g):
    """A spread of (row blocks, column block) cases, incl. unions."""
    out = [([I], J) for I in range(g.m) for J in range(g.n)]
    out.append((list(range(g.m)), g.n - 1))
    out.append(([g.m - 1, 0], 0))
    return out


@pytest.mark.parametrize("name", list(GEOMS))
def test_block_fwd_parity(ct, name):
    g, S = system(name)
    G = ct.ct_geom_create(g)
    rng = np.random.default_rng(1)
    x = rng.uniform(0.0, 1.0, g.n_vox).astype(np.float32)
    xd = dev(x)
    worst = worst_el = 0.0
    for rbs, J in _pairs(g):
        print(f"[fwd] {name} rbs={rbs} J={J}", flush=True)
        yd = torch.full((G.M,), 7.0, device="cuda")
        ct.ct_block_fwd(G, rbs, J, xd, yd)
        y = host(yd)
        rows = S.group_rows(rbs)
        ref = csgd.block_fwd(S, rbs, J, x.astype(np.float64))
        if np.linalg.norm(ref) == 0:
            assert np.all(y[rows] == 0)
        else:
            worst = max(worst, rel_l2(y[rows], ref))
            worst_el = max(worst_el, max_rel(y[rows], ref))
        other = np.ones(G.M, bool)
        other[rows] = False
        assert np.all(y[other] == 7.0), "wrote outside the row blocks"
    assert worst <= 1e-5, worst
    assert worst_el <= 1e-5, worst_el


@pytest.mark.parametrize("name", list(GEOMS))
def test_block_back_parity(ct, name):
    g, S = system(name)
    G = ct.ct_geom_create(g)
    rng = np.random.default_rng(2)
    r = rng.normal(0.0, 1.0, g.n_rays).astype(np.float32)
    rd = dev(r)
    worst = worst_el = 0.0
    for rbs, J in _pairs(g):
        print(f"[back] {name} rbs={rbs} J={J}", flush=True)
        gd = torch.full((G.N,), -3.0, device="cuda")
        ct.ct_block_back(G, rbs, J, rd, gd)
        gv = host(gd)
        vox = S.vox[J]
        ref = csgd.block_back(S, rbs, J, r.astype(np.float64))
        if np.linalg.norm(ref) == 0:
            assert np.all(gv[vox] == 0)
        else:
            worst = max(worst, rel_l2(gv[vox], ref))
            worst_el = max(worst_el, max_rel(gv[vox], ref))
        other = np.ones(G.N, bool)
        other[vox] = False
        assert np.all(gv[other] == -3.0), "wrote outside the column block"
    assert worst <= 1e-5, worst
    assert worst_el <= 1e-5, worst_el


@pytest.mark.parametrize("name", ["c1_par2d", "cone"])
def test_accumulate_flag(ct, name):
    g, S = system(name)
    G = ct.ct_geom_create(g)
    rng = np.random.default_rng(3)
    x = dev(rng.uniform(0, 1, g.n_vox))
    r = dev(rng.normal(0, 1, g.n_rays))
    y0 = rng.normal(0, 1, g.n_rays).astype(np.float32)
    yd = dev(y0)
    ct.ct_block_fwd(G, [0], 1, x, yd, flags=ct.CT_ACCUMULATE)
    rows = S.group_rows([0])
    ref = y0[rows].astype(np.float64) + csgd.block_fwd(S, [0], 1, host(x))
    assert rel_l2(host(yd)[rows], ref) <= 1e-5
    g0 = rng.normal(0, 1, g.n_vox).astype(np.float32)
    gd = dev(g0)
    ct.ct_block_back(G, [1, 0], 0, r, gd, flags=ct.CT_ACCUMULATE)
    vox = S.vox[0]
    ref = g0[vox].astype(np.float64) + csgd.block_back(S, [1, 0], 0, host(r))
    assert rel_l2(host(gd)[vox], ref) <= 1e-5


@pytest.mark.parametrize("name", list(GEOMS))
def test_gpu_adjoint(ct, name):
    g, S = system(name)
    G = ct.ct_geom_create(g)
    rng = np.random.default_rng(4)
    x = dev(rng.uniform(0, 1, g.n_vox))
    r = dev(rng.normal(0, 1, g.n_rays))
    for I, J in [(0, 0), (g.m - 1, g.n - 1), (g.m // 2, g.n // 2)]:
        yd = torch.zeros(G.M, device="cuda")
        gd = torch.zeros(G.N, device="cuda")
        ct.ct_block_fwd(G, [I], J, x, yd)
        ct.ct_block_back(G, [I], J, r, gd)
        a = float(host(yd) @ host(r))
        b = float(host(x) @ host(gd))
        scale = float(np.abs(host(yd)) @ np.abs(host(r))) + 1e-30
        assert abs(a - b) <= 2e-6 * scale, (I, J, a, b)


@pytest.mark.parametrize("name", list(GEOMS))
def test_block_density_table(ct, name):
    g, S = system(name)
    G = ct.ct_geom_create(g)
    tau = tau_for(g)
    gpu = ct.ct_geom_block_nnz(G, tau)
    ref = S.nnz_table(tau)
    # integer work, decided on float64 lengths on both sides: exact
    assert np.array_equal(gpu, ref), np.abs(gpu - ref).sum()


def _run_pair(ct, name, epochs, alpha, gamma, s, b, seed, sync="column",
              sampling=sampler.DENSITY, noise=0.01, theta_step=1.0 / 40):
    g, S = system(name)
    G = ct.ct_geom_create(g)
    x_true, y = phantom_y(g, S, seed, noise)
    if sampling == "area":                  # the paper's projection-area densities
        from oracle import area
        P, sampling = area.area_density(g), sampler.DENSITY
    else:
        P = sampler.density(S.nnz_table(tau_for(g)))
    sch = sampler.make_schedule(P, epochs, alpha, gamma, s, b, seed, sampling, theta_step,
                                proj=sampler.projection_of(g.row_blocks))
    ref = csgd.run(S, y.astype(np.float64), sch, sync=sync)
    sc = ct.ct_schedule_import(G, sch)
    sol = ct.ct_solver_create(G, ct.CT_SYNC_COLUMN if sync == "column" else ct.CT_SYNC_EPOCH)
    yd = dev(y)
    xd = torch.zeros(G.N, device="cuda")
    ct.ct_solver_reset(sol, yd)
    for e in range(epochs):
        ct.ct_block_epoch(sol, sc, e, yd, xd)
    z, r = ct.ct_solver_state(sol)
    return g, S, ref, host(xd), host(z), host(r), x_true


@pytest.mark.parametrize("case", [
    # name, epochs, alpha, gamma, s, b, seed, sync, sampling
    ("c1_par2d", 50, 0.5, 1.0, 1, 0.5, 1000, "column", sampler.DENSITY),
    ("c1_par2d", 20, 1.0, 0.5, 2, 2.0, 1001, "column", sampler.DENSITY),
    ("c1_par2d", 20, 0.75, 1.0, 1, 1.0, 1002, "epoch", sampler.UNIFORM),
    ("fan_curved", 20, 0.5, 1.0, 1, 3.0, 2000, "column", sampler.DENSITY),
    ("fan_curved", 10, 1.0, 1.0, 3, 1.0, 2001, "column", sampler.MIXED),
    ("fan_flat", 12, 0.6, 1.0, 2, 2.0, 2100, "epoch", sampler.DENSITY),
    ("cone", 10, 1.0, 1.0, 3, 1.0, 3000, "column", sampler.DENSITY),
    ("fan_curved", 15, 0.5, 1.0, 2, 1.0, 2002, "column", "area"),
    ("fan_fine", 12, 0.5, 1.0, 2, 1.0, 2003, "column", sampler.DENSITY),
    ("cone", 6, 0.5, 1.0, 2, 1.0, 3001, "column", "area"),
    # detector split into sub-areas: mixed sampling's P_max per projection,
    # theta reaching 1 within the run
    ("fan_split", 10, 0.5, 1.0, 2, 1.0, 2004, "column", sampler.MIXED, 0.125),
    ("cone_split", 6, 0.5, 1.0, 3, 1.0, 3002, "epoch", sampler.MIXED, 0.25),
])
def test_epoch_parity(ct, case):
    name, E, a, gm, s, b, seed, sync, samp = case[:9]
    th = case[9] if len(case) > 9 else 1.0 / 40
    print(f"[epochs] {case}", flush=True)
    g, S, ref, x, z, r, x_true = _run_pair(ct, name, E, a, gm, s, b, seed, sync, samp,
                                           theta_step=th)
    err = rel_l2(x, ref.x)
    assert err <= 1e-4, err
    assert rel_l2(z, ref.z) <= 1e-4
    assert np.linalg.norm(r - ref.r) <= 1e-4 * np.linalg.norm(ref.y)
    # the reconstruction improves on the start (sanity, not parity)
    assert np.linalg.norm(x - x_true) < np.linalg.norm(x_true)


def test_reset_from_nonzero_x(ct):
    g, S = system("fan_curved")
    G = ct.ct_geom_create(g)
    rng = np.random.default_rng(9)
    x0 = rng.uniform(0, 1, g.n_vox).astype(np.float32)
    y = (S.A @ rng.uniform(0, 1, g.n_vox)).astype(np.float32)
    st = csgd.State(S, y.astype(np.float64), x0=x0.astype(np.float64))
    sol = ct.ct_solver_create(G)
    ct.ct_solver_reset(sol, dev(y), dev(x0))
    z, r = ct.ct_solver_state(sol)
    assert rel_l2(host(z), st.z) <= 1e-5
    assert rel_l2(host(r), st.r) <= 1e-5


def test_epochs_are_bitwise_reproducible(ct):
    g, S = system("c1_par2d")
    G = ct.ct_geom_create(g)
    _, y = phantom_y(g, S, 77)
    sch = sampler.make_schedule(sampler.density(S.nnz_table(tau_for(g))), 8, 0.5, 1.0, 1, 4.0, 77)
    sc = ct.ct_schedule_import(G, sch)
    outs = []
    for _ in range(2):
        sol = ct.ct_solver_create(G)
        yd, xd = dev(y), torch.zeros(G.N, device="cuda")
        ct.ct_solver_reset(sol, yd)
        for e in range(8):
            ct.ct_block_epoch(sol, sc, e, yd, xd)
        outs.append(host(xd))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("name,sync", [("fan_curved", "column"), ("fan_fine", "column"), ("cone", "epoch")])
def test_checkpoint_resume_is_bitwise(ct, name, sync):
    """A solver carries x, z and r from one epoch to the next and nothing
    else, so saving them after epoch k and restoring them into a fresh solver
    (through ct_solver_state's pointers) continues bit for bit like an
    uninterrupted run."""
    g, S = system(name)
    G = ct.ct_geom_create(g)
    _, y = phantom_y(g, S, 78)
    sch = sampler.make_schedule(sampler.density(S.nnz_table(tau_for(g))), 5, 0.5, 1.0, 2, 1.0, 78)
    sc = ct.ct_schedule_import(G, sch)
    mode = ct.CT_SYNC_COLUMN if sync == "column" else ct.CT_SYNC_EPOCH
    yd = dev(y)

    def run(sol, x, e0, e1):
        for e in range(e0, e1):
            ct.ct_block_epoch(sol, sc, e, yd, x)

    ref = ct.ct_solver_create(G, mode)
    x_ref = torch.zeros(G.N, device="cuda")
    ct.ct_solver_reset(ref, yd)
    run(ref, x_ref, 0, 5)
    z_ref, r_ref = ct.ct_solver_state(ref)

    a = ct.ct_solver_create(G, mode)
    xa = torch.zeros(G.N, device="cuda")
    ct.ct_solver_reset(a, yd)
    run(a, xa, 0, 2)
    za, ra = ct.ct_solver_state(a)
    # the checkpoint, on the host (float32 -> float64 -> float32 is exact)
    saved = tuple(host(t).astype(np.float32) for t in (xa, za, ra))
    del a, za, ra

    b = ct.ct_solver_create(G, mode)
    ct.ct_solver_reset(b, yd)
    zb, rb = ct.ct_solver_state(b)
    zb.copy_(torch.as_tensor(saved[1], device="cuda"))
    rb.copy_(torch.as_tensor(saved[2], device="cuda"))
    xb = dev(saved[0])
    run(b, xb, 2, 5)
    torch.cuda.synchronize()
    assert torch.equal(xb, x_ref) and torch.equal(zb, z_ref) and torch.equal(rb, r_ref)


def test_solve_counts_updates_and_converges(ct):
    g, S = system("c1_par2d")
    G = ct.ct_geom_create(g)
    x_true, y = phantom_y(g, S, 1000, noise=0.0)
    xd = torch.zeros(G.N, device="cuda")
    params = ct.sched_params(200, 0.5, 1.0, 1, 4.0, seed=1000)
    rc, st = ct.ct_solve(G, params, dev(y), xd, tau=tau_for(g), rel_tol=1e-2, check_every=5)
    assert rc == ct.CT_OK, st
    assert st["rel_residual"] <= 1e-2
    assert st["epochs_run"] % 5 == 0
    # the reported work is 2 * sum of the scheduled blocks' nnz
    nnz = ct.ct_geom_block_nnz(G, tau_for(g))
    sch = ct.ct_schedule_export(ct.ct_schedule_create(G, params, nnz))
    want = 0
    for e in range(st["epochs_run"]):
        for c in range(sch["epoch_col_ptr"][e], sch["epoch_col_ptr"][e + 1]):
            J = sch["cols"][c]
            for k in range(sch["group_rb_ptr"][sch["col_group_ptr"][c]],
                           sch["group_rb_ptr"][sch["col_group_ptr"][c + 1]]):
                want += 2 * nnz[sch["rbs"][k], J]
    assert st["ray_voxel_updates"] == want
    assert abs(ct.ct_true_residual(ct.ct_solver_create(G), dev(y), xd) - st["rel_residual"]) < 1e-6


def _residue_views(n_views, sid, sdd, third_axis):
    """Circular views from plain float64 cos/sin: the quarter turns keep the
    residue cos(pi/2) = 6e-17, a tilt of that size of every ray that should be
    parallel to an axis."""
    th = 2 * np.pi * np.arange(n_views) / n_views
    c, s = np.cos(th), np.sin(th)
    v = np.zeros((n_views, 12))
    v[:, 0], v[:, 1] = sid * c, sid * s
    v[:, 3], v[:, 4] = -(sdd - sid) * c, -(sdd - sid) * s
    v[:, 6], v[:, 7] = -s, c
    if third_axis:
        v[:, 11] = 1.0
    return v


@pytest.mark.parametrize("name", ["fan_flat_axis", "cone_axis"])
def test_residue_axis_rays(ct, name):
    """Rays on voxel faces whose direction carries float64 residue of an axis
    (the exact geometry puts them on the face; the oracle's float64 walk
    splits them between the two voxels at the face where the residue tilt
    crosses it, a split float32 cannot resolve).  What is unique must match:
    every other ray and voxel to 1e-5, the chord length of every ray (row sum
    of A) to 1e-5, and the back-projection of every row block keeps the total
    length of its rays (none lost or counted twice)."""
    import dataclasses
    from oracle import rays, siddon
    g0 = GEOMS[name]()
    g = dataclasses.replace(g0, views=_residue_views(g0.n_views, 100.0, 200.0, g0.is3d))
    G = ct.ct_geom_create(g)
    A = siddon.system_matrix(g).tocsr()
    S = csgd.BlockSystem(A, g)
    _, d, _ = rays.rays(g)
    ad = np.abs(d) / np.linalg.norm(d, axis=1, keepdims=True)
    degen = np.any((ad > 0) & (ad <= 1e-12), axis=1)
    assert degen.sum() > 0
    print(f"[residue] {name}: {degen.sum()} residue-tilted rays", flush=True)
    ones = dev(np.ones(g.n_vox))
    yd = torch.zeros(G.M, device="cuda")
    for J in range(g.n):
        ct.ct_block_fwd(G, list(range(g.m)), J, ones, yd, flags=ct.CT_ACCUMULATE)
    rowsum = np.asarray(A.sum(axis=1)).ravel()
    assert np.all(np.abs(host(yd) - rowsum) <= 1e-5 * rowsum.max())
    rng = np.random.default_rng(5)
    x = rng.uniform(0.0, 1.0, g.n_vox).astype(np.float32)
    r = rng.normal(0.0, 1.0, g.n_rays).astype(np.float32)
    r[degen] = 0.0
    for I in range(g.m):
        rows = S.rows[I]
        for J in range(g.n):
            yd = torch.zeros(G.M, device="cuda")
            ct.ct_block_fwd(G, [I], J, dev(x), yd)
            keep = ~degen[rows]
            ref = csgd.block_fwd(S, [I], J, x.astype(np.float64))
            assert rel_l2(host(yd)[rows][keep], ref[keep]) <= 1e-5, (I, J)
            gd = torch.zeros(G.N, device="cuda")
            ct.ct_block_back(G, [I], J, dev(r), gd)
            refb = csgd.block_back(S, [I], J, r.astype(np.float64))
            assert rel_l2(host(gd)[S.vox[J]], refb) <= 1e-5, (I, J)
        gd = torch.zeros(G.N, device="cuda")
        ri = np.zeros(g.n_rays, np.float32)
        ri[rows] = 1.0
        for J in range(g.n):
            ct.ct_block_back(G, [I], J, dev(ri), gd, flags=ct.CT_ACCUMULATE)
        tot = rowsum[rows].sum()
        assert abs(host(gd).sum() - tot) <= 1e-5 * tot, I
