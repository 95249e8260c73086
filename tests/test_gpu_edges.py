"""Edge cases of the HIP path against the FP64 oracle: zero data (g = 0, so
mu = 0 by reading C7, and nothing moves), a column block that no ray meets
(zero density: never drawn, its voxels keep their values), and geometries
smaller than one tile (single views, one-voxel-wide blocks, boxes of a few
voxels), where every projection and two epochs must match.
"""
import numpy as np
import pytest

from oracle import csgd, sampler, siddon
from paper_1709_00953_amd import inputs
from tests.parity_util import max_rel, rel_l2, system, tau_for

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


def run_epochs(ct, g, y, sch, E, x0=None, sync="column"):
    G = ct.ct_geom_create(g)
    sc = ct.ct_schedule_import(G, sch)
    sol = ct.ct_solver_create(G, ct.CT_SYNC_COLUMN if sync == "column" else ct.CT_SYNC_EPOCH)
    yd = dev(y)
    xd = dev(x0) if x0 is not None else torch.zeros(G.N, device="cuda")
    if x0 is not None:
        ct.ct_solver_reset(sol, yd, xd)
    else:
        ct.ct_solver_reset(sol, yd)
    for e in range(E):
        ct.ct_block_epoch(sol, sc, e, yd, xd)
    z, r = ct.ct_solver_state(sol)
    return host(xd), host(z), host(r)


@pytest.mark.parametrize("name", ["c1_par2d", "fan_curved", "fan_fine", "fan_flat", "cone"])
def test_zero_data_stays_zero(ct, name):
    g, S = system(name)
    P = sampler.density(S.nnz_table(tau_for(g)))
    sch = sampler.make_schedule(P, 3, 1.0, 1.0, 2, 1.0, 11)
    x, z, r = run_epochs(ct, g, np.zeros(g.n_rays, np.float32), sch, 3)
    assert np.all(x == 0) and np.all(z == 0) and np.all(r == 0)


def geom_unreachable():
    """64^2 fan with a 9-bin detector (a fan of +-0.018 rad) and views over
    20 degrees only: every ray stays near the x axis, so the top and bottom
    rows of the 4 x 4 blocks are met by no ray."""
    return inputs.fan2d(64, 1.0, 8, 9, 4e-3, 100.0, 200.0, m=4, bx=4, by=4, span_deg=20.0)


def test_unreachable_column_block_keeps_its_values(ct):
    g = geom_unreachable()
    S = csgd.BlockSystem(siddon.system_matrix(g), g)
    nnz = S.nnz_table(tau_for(g))
    dead = np.flatnonzero(nnz.sum(axis=0) == 0)
    assert dead.size > 0
    G = ct.ct_geom_create(g)
    assert np.array_equal(ct.ct_geom_block_nnz(G, tau_for(g)), nnz)
    P = sampler.density(nnz)
    sch = sampler.make_schedule(P, 4, 1.0, 1.0, 2, 1.0, 12)
    rng = np.random.default_rng(12)
    x0 = rng.uniform(0.0, 1.0, g.n_vox)
    x_true = inputs.phantom_for(g, 12)
    y = inputs.gaussian_noise(S.A @ x_true, 0.01, 12)
    ref = csgd.run(S, y.astype(np.float64), sch, x0=x0.astype(np.float32).astype(np.float64))
    x, z, r = run_epochs(ct, g, y, sch, 4, x0=x0.astype(np.float32))
    assert rel_l2(x, ref.x) <= 1e-4
    for J in dead:
        vox = S.vox[J]
        assert np.array_equal(x[vox], x0.astype(np.float32)[vox].astype(np.float64))


def tiny_geometries():
    return {
        # 5 x 5 image in three rows of blocks (1-2 voxels tall), 2 views, 7 bins
        "par_tiny": inputs.par2d(5, 1.0, 2, 180.0, 7, 1.0, m=2, bx=1, by=3),
        # 6 x 6 curved fan, one view per row block, blocks of 2 x 3 voxels
        "fan_tiny": inputs.fan2d(6, 2.0, 3, 11, 1e-2, 50.0, 100.0, m=3, bx=3, by=2),
        # 5^3 cone, 2 views of 9^2, z blocks of 1-2 voxels
        "cone_tiny": inputs.cone3d(5, 2.0, 2, 9, 2.0, 50.0, 100.0, m=2, bz=3, bxy=2),
    }


@pytest.mark.parametrize("name", list(tiny_geometries()))
def test_tiny_geometries(ct, name):
    g = tiny_geometries()[name]
    S = csgd.BlockSystem(siddon.system_matrix(g), g)
    G = ct.ct_geom_create(g)
    rng = np.random.default_rng(13)
    x = rng.uniform(0.0, 1.0, g.n_vox).astype(np.float32)
    r = rng.normal(0.0, 1.0, g.n_rays).astype(np.float32)
    for I in range(g.m):
        for J in range(g.n):
            yd = torch.full((G.M,), 7.0, device="cuda")
            ct.ct_block_fwd(G, [I], J, dev(x), yd)
            rows = S.group_rows([I])
            ref = csgd.block_fwd(S, [I], J, x.astype(np.float64))
            got = host(yd)
            if np.linalg.norm(ref) > 0:
                assert rel_l2(got[rows], ref) <= 1e-5, (I, J)
                assert max_rel(got[rows], ref) <= 1e-5, (I, J)
            else:
                assert np.all(got[rows] == 0), (I, J)
            gd = torch.full((G.N,), -3.0, device="cuda")
            ct.ct_block_back(G, [I], J, dev(r), gd)
            refb = csgd.block_back(S, [I], J, r.astype(np.float64))
            gb = host(gd)[S.vox[J]]
            if np.linalg.norm(refb) > 0:
                assert rel_l2(gb, refb) <= 1e-5, (I, J)
                assert max_rel(gb, refb) <= 1e-5, (I, J)
            else:
                assert np.all(gb == 0), (I, J)
    nnz = S.nnz_table(tau_for(g))
    assert np.array_equal(ct.ct_geom_block_nnz(G, tau_for(g)), nnz)
    P = sampler.density(nnz)
    sch = sampler.make_schedule(P, 2, 1.0, 1.0, 1, 0.5, 14)
    y = (S.A @ rng.uniform(0.0, 1.0, g.n_vox)).astype(np.float32)
    ref = csgd.run(S, y.astype(np.float64), sch)
    x_gpu, z, rr = run_epochs(ct, g, y, sch, 2)
    assert rel_l2(x_gpu, ref.x) <= 1e-4
    assert np.linalg.norm(rr - ref.r) <= 1e-4 * np.linalg.norm(y)
