"""The paper's own simulation settings (Sec. III): the 2D flat-fan case with
one row block per (view, detector half), 720 in all, at the three group sizes
and relaxations it reports (s = 1, 5, 100 with b = 100, 25, 2), and the 3D
random-sphere trajectory.  HIP path against the FP64 oracle: projections to
1e-5, epochs to 1e-4; the full 128^3 sphere case on sampled outputs.
"""
import functools

import numpy as np
import pytest

from oracle import area, csgd, rays, sampler, siddon
from paper_1709_00953_amd import inputs
from tests.parity_util import max_rel, rel_l2, tau_for

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


@functools.lru_cache(maxsize=2)
def system(name):
    g = inputs.config_paper2d() if name == "paper2d" else inputs.config_paper3d(24, 40, 360)
    return g, csgd.BlockSystem(siddon.system_matrix(g), g)


@pytest.mark.parametrize("name", ["paper2d", "paper3d_small"])
def test_paper_projectors(ct, name):
    g, S = system(name)
    G = ct.ct_geom_create(g)
    rng = np.random.default_rng(7)
    x = rng.uniform(0.0, 1.0, g.n_vox).astype(np.float32)
    r = rng.normal(0.0, 1.0, g.n_rays).astype(np.float32)
    pairs = [([int(I)], int(J)) for I, J in zip(rng.integers(0, g.m, 24), rng.integers(0, g.n, 24))]
    pairs.append((sorted(rng.choice(g.m, size=min(100, g.m), replace=False).tolist()), g.n - 1))
    for rbs, J in pairs:
        rows = S.group_rows(rbs)
        yd = torch.full((G.M,), 7.0, device="cuda")
        ct.ct_block_fwd(G, rbs, J, dev(x), yd)
        y = host(yd)
        ref = csgd.block_fwd(S, rbs, J, x.astype(np.float64))
        if np.linalg.norm(ref) > 0:
            assert rel_l2(y[rows], ref) <= 1e-5, (rbs[:4], J)
            assert max_rel(y[rows], ref) <= 1e-5, (rbs[:4], J)
        other = np.setdiff1d(np.arange(G.M), rows)
        assert np.all(y[other] == 7.0)
        gd = torch.full((G.N,), 7.0, device="cuda")
        ct.ct_block_back(G, rbs, J, dev(r), gd)
        gv = host(gd)
        refb = csgd.block_back(S, rbs, J, r.astype(np.float64))
        vox = S.vox[J]
        if np.linalg.norm(refb) > 0:
            assert rel_l2(gv[vox], refb) <= 1e-5, (rbs[:4], J)
            assert max_rel(gv[vox], refb) <= 1e-5, (rbs[:4], J)


def _epochs(ct, name, E, alpha, s, b, seed, P=None):
    g, S = system(name)
    G = ct.ct_geom_create(g)
    x_true = inputs.phantom_for(g, seed)
    y = inputs.gaussian_noise(S.A @ x_true, 0.01, seed)
    if P is None:
        P = sampler.density(S.nnz_table(tau_for(g)))
    sch = sampler.make_schedule(P, E, alpha, 1.0, s, b, seed)
    ref = csgd.run(S, y.astype(np.float64), sch)
    sc = ct.ct_schedule_import(G, sch)
    sol = ct.ct_solver_create(G)
    yd = dev(y)
    xd = torch.zeros(G.N, device="cuda")
    ct.ct_solver_reset(sol, yd)
    for e in range(E):
        ct.ct_block_epoch(sol, sc, e, yd, xd)
    z, r = ct.ct_solver_state(sol)
    return ref, host(xd), host(z), host(r), y


@pytest.mark.parametrize("s,b", [(1, 100.0), (5, 25.0), (100, 2.0)])
def test_paper2d_group_sizes(ct, s, b):
    """alpha = 0.5 over 720 row blocks per column block, the group sizes and
    relaxations of the paper's group-size comparison."""
    print(f"[paper2d] s={s} b={b}", flush=True)
    ref, x, z, r, y = _epochs(ct, "paper2d", 3, 0.5, s, b, 6000 + s)
    assert rel_l2(x, ref.x) <= 1e-4
    assert rel_l2(z, ref.z) <= 1e-4
    assert np.linalg.norm(r - ref.r) <= 1e-4 * np.linalg.norm(y)


def test_paper2d_area_sampling(ct):
    """The same with the paper's projection-area densities P_S / P_T."""
    g, _ = system("paper2d")
    ref, x, z, r, y = _epochs(ct, "paper2d", 3, 0.5, 5, 25.0, 6100, P=area.area_density(g))
    assert rel_l2(x, ref.x) <= 1e-4
    assert rel_l2(z, ref.z) <= 1e-4


def test_paper3d_sphere_epochs(ct):
    """Random-sphere trajectory (general view frames, no circular structure),
    the paper's 3D parameters: every projection a row block, groups of 90,
    b = 1, alpha = 0.5."""
    ref, x, z, r, y = _epochs(ct, "paper3d_small", 3, 0.5, 90, 1.0, 6200)
    assert rel_l2(x, ref.x) <= 1e-4
    assert rel_l2(z, ref.z) <= 1e-4
    assert np.linalg.norm(r - ref.r) <= 1e-4 * np.linalg.norm(y)


def test_paper3d_fullsize_sampled(ct):
    """128^3 voxels, 720 random views of 202^2: projections on sampled rays
    (the oracle's Siddon rows of those rays) and sampled voxels (clip lengths
    over every candidate ray)."""
    from tests.test_gpu_fullscale import clip_sum, cone_candidates, rows_of
    g = inputs.config_paper3d()
    G = ct.ct_geom_create(g)
    rng = np.random.default_rng(8)
    x = rng.uniform(0.0, 1.0, g.n_vox).astype(np.float32)
    rbs, J = [3, 17, 40, 411], 5
    yd = torch.full((G.M,), 7.0, device="cuda")
    ct.ct_block_fwd(G, rbs, J, dev(x), yd)
    got = host(yd)
    I = rows_of(g, rbs)
    smp = np.sort(rng.choice(I, size=2000, replace=False))
    org, dirn, div = rays.rays_at(g, smp)
    A_s = siddon.rows_for(g, org, dirn, div)
    xJ = np.zeros(g.n_vox)
    vox = g.col_block_vox(J)
    xJ[vox] = x[vox]
    err = rel_l2(got[smp], A_s @ xJ)
    print(f"[paper3d] forward sampled: {err:.2e}", flush=True)
    assert err <= 1e-5
    assert max_rel(got[smp], A_s @ xJ) <= 1e-5
    r = rng.normal(0.0, 1.0, g.n_rays).astype(np.float32)
    gd = torch.full((G.N,), 7.0, device="cuda")
    ct.ct_block_back(G, rbs, J, dev(r), gd)
    gv = host(gd)
    views = np.unique(np.concatenate([np.asarray(g.row_blocks[b])[:, 0] for b in rbs]))
    vsmp = np.sort(rng.choice(vox, size=40, replace=False))
    ref = []
    for v in vsmp:
        cand = cone_candidates(g, v, views)
        o, d, dv = rays.rays_at(g, cand)
        ref.append(clip_sum(g, o, d, dv, r[cand], v))
    err = rel_l2(gv[vsmp], np.array(ref))
    print(f"[paper3d] back sampled: {err:.2e}", flush=True)
    assert err <= 1e-5
    assert max_rel(gv[vsmp], np.array(ref)) <= 1e-5
