"""Parity at the full sizes of the benchmark workloads (512^2 fan beam, 256^3
cone beam), in the launch configuration the benchmark times, and at the
largest sizes of the batched and served workloads (1024^2 fan slices, 192^3
cones).

Projections are checked on sampled outputs the oracle computes one by one:
sampled rays through Siddon rows of those rays, sampled voxels through the
plain clip-length definition of A_ij summed over every candidate ray.  The
fan-beam case also runs whole epochs against the oracle (explicit FP64 A of
2.4e8 nonzeros); the cone-beam epoch, whose explicit A would need ~90 GB, is
checked through invariants that hold at any size.
"""
import functools

import numpy as np
import pytest

from oracle import csgd, rays, sampler, siddon
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
    return t.detach().cpu().numpy()


def rows_of(g, rbs):
    return np.concatenate([g.row_block_rays(b) for b in rbs])


def voxel_box(g, v):
    """Half-open box [lo, hi) of voxel index v (x fastest)."""
    ix = v % g.nx
    iy = (v // g.nx) % g.ny
    iz = v // (g.nx * g.ny)
    idx = np.stack([ix, iy, iz], axis=-1).astype(np.float64)
    h = np.array([g.vx, g.vy, g.vz])
    o = np.array([g.ox, g.oy, g.oz])
    lo = o + idx * h
    return lo, lo + h


def sampled_forward(ct, g, G, rbs, J, x, n_rays, seed):
    xd = dev(x)
    yd = torch.full((G.M,), 7.0, device="cuda")
    ct.ct_block_fwd(G, rbs, J, xd, yd)
    got = host(yd)
    rng = np.random.default_rng(seed)
    I = rows_of(g, rbs)
    smp = np.sort(rng.choice(I, size=min(n_rays, I.size), replace=False))
    org, dirn, div = rays.rays_at(g, smp)
    A_s = siddon.rows_for(g, org, dirn, div)
    vox = g.col_block_vox(J)
    xJ = np.zeros(g.n_vox)
    xJ[vox] = x[vox].astype(np.float64)
    ref = A_s @ xJ
    err = rel_l2(got[smp], ref)
    assert max_rel(got[smp], ref) <= 1e-5
    # rays outside the row blocks are not written
    outside = np.setdiff1d(rng.choice(G.M, size=20000, replace=False), I)
    assert np.all(got[outside] == 7.0)
    return err


def clip_sum(g, org, dirn, div, r, v):
    """sum_i |ray_i ∩ voxel v| r_i by the plain clip-length definition."""
    lo, hi = voxel_box(g, np.array([v]))
    D = 3 if g.is3d else 2
    K = org.shape[0]
    L = siddon.clip_length(org[:, :D], dirn[:, :D], div, np.repeat(lo[:, :D], K, 0),
                           np.repeat(hi[:, :D], K, 0))
    return float(L @ r.astype(np.float64))


# 2D cases: the benchmark's 512^2 fan, and the largest slice of the batched
# and served workloads (1024^2 at 0.25 mm, 1536 views of 1536 bins)
FAN_CASES = {
    "fan512": (inputs.config_c2, (([0, 1, 2, 3, 4, 5, 6, 7], 5), ([2], 0), ([7, 3], 6)),
               (([2], 0), ([7, 3], 6))),
    "slice1024": (lambda: inputs.slice_fan(1024), (([0, 1, 2, 3], 3), ([1], 0), ([3, 0], 2)),
                  (([1], 0), ([3, 0], 2))),
}


@pytest.mark.parametrize("name", list(FAN_CASES))
def test_fan_projectors_sampled(ct, name):
    make, fwd_cases, back_cases = FAN_CASES[name]
    g = make()
    G = ct.ct_geom_create(g)
    rng = np.random.default_rng(11)
    x = rng.uniform(0.0, 1.0, g.n_vox).astype(np.float32)
    for rbs, J in fwd_cases:
        err = sampled_forward(ct, g, G, list(rbs), J, x, 3000, 12 + J)
        print(f"[full] {name} forward rbs={rbs} J={J}: rel {err:.2e}", flush=True)
        assert err <= 1e-5
    r = rng.normal(0.0, 1.0, g.n_rays).astype(np.float32)
    org_all, dir_all, div = rays.rays(g)
    for rbs, J in back_cases:
        rbs = list(rbs)
        gd = torch.full((G.N,), 7.0, device="cuda")
        ct.ct_block_back(G, rbs, J, dev(r), gd)
        got = host(gd)
        I = rows_of(g, rbs)
        vox = g.col_block_vox(J)
        smp = np.sort(rng.choice(vox, size=300, replace=False))
        ref = np.array([clip_sum(g, org_all[I], dir_all[I], div, r[I], v) for v in smp])
        err = rel_l2(got[smp], ref)
        print(f"[full] {name} back rbs={rbs} J={J}: rel {err:.2e}", flush=True)
        assert err <= 1e-5
        assert max_rel(got[smp], ref) <= 1e-5
        other = np.setdiff1d(rng.choice(G.N, size=5000, replace=False), vox)
        assert np.all(got[other] == 7.0)


@functools.lru_cache(maxsize=1)
def fan512_system():
    g = inputs.config_c2()
    A = siddon.system_matrix(g)
    return g, csgd.BlockSystem(A, g)


@pytest.mark.parametrize("sync,gamma", [("column", 1.0), ("epoch", 0.5)])
def test_fan512_epochs_match_oracle(ct, sync, gamma):
    """Two epochs of the benchmark's fan-beam configuration (alpha 0.5, s 1,
    b 1, density sampling) on the oracle's schedule and y; also in the
    fully parallel reading (r refreshed once per epoch, Sec. II-B) with half
    of the column blocks per epoch (gamma 0.5, Sec. III-C)."""
    g, S = fan512_system()
    A = S.A
    x_true = inputs.phantom_for(g, 2000)
    y = inputs.gaussian_noise(A @ x_true, 0.01, 2000)
    P = sampler.density(S.nnz_table(tau_for(g)))
    sch = sampler.make_schedule(P, 2, 0.5, gamma, 1, 1.0, 2000)
    st = csgd.State(S, y.astype(np.float64))
    for e in range(2):
        csgd.epoch(st, sch, e, sync)
    G = ct.ct_geom_create(g)
    sol = ct.ct_solver_create(G, ct.CT_SYNC_COLUMN if sync == "column" else ct.CT_SYNC_EPOCH)
    yd = dev(y)
    x = torch.zeros(G.N, device="cuda")
    ct.ct_solver_reset(sol, yd)
    sc = ct.ct_schedule_import(G, sch)
    for e in range(2):
        ct.ct_block_epoch(sol, sc, e, yd, x)
    z, r = ct.ct_solver_state(sol)
    ex = rel_l2(host(x), st.x)
    ez = rel_l2(host(z).ravel(), np.concatenate([st.z[j] for j in range(g.n)]))
    er = np.linalg.norm(host(r) - st.r) / np.linalg.norm(y)
    print(f"[full] fan512 2 epochs ({sync}, gamma {gamma}): x {ex:.2e} z {ez:.2e} r {er:.2e}", flush=True)
    assert ex <= 1e-4 and ez <= 1e-4 and er <= 1e-4


def cone_candidates(g, v, views):
    """Rays of `views` whose bin lies within two bins of voxel v's projected
    corners (every ray meeting the voxel is among them)."""
    lo, hi = voxel_box(g, np.array([v]))
    corners = np.array([[lo[0, 0] if (c & 1) == 0 else hi[0, 0],
                         lo[0, 1] if (c & 2) == 0 else hi[0, 1],
                         lo[0, 2] if (c & 4) == 0 else hi[0, 2]] for c in range(8)])
    V = np.asarray(g.views, dtype=np.float64)[views]
    a, c, eu, ev = V[:, 0:3], V[:, 3:6], V[:, 6:9], V[:, 9:12]
    n = c - a
    sdd = np.linalg.norm(n, axis=1)
    n = n / sdd[:, None]
    w = corners[None, :, :] - a[:, None, :]
    dep = np.einsum("vkc,vc->vk", w, n)
    u = sdd[:, None] * np.einsum("vkc,vc->vk", w, eu) / dep / g.pu + 0.5 * (g.nu - 1)
    vv = sdd[:, None] * np.einsum("vkc,vc->vk", w, ev) / dep / g.pv + 0.5 * (g.nv - 1)
    out = []
    for k, view in enumerate(views):
        u0, u1 = max(0, int(np.floor(u[k].min())) - 2), min(g.nu - 1, int(np.ceil(u[k].max())) + 2)
        v0, v1 = max(0, int(np.floor(vv[k].min())) - 2), min(g.nv - 1, int(np.ceil(vv[k].max())) + 2)
        iu, iv = np.meshgrid(np.arange(u0, u1 + 1), np.arange(v0, v1 + 1))
        out.append(((view * g.nv + iv) * g.nu + iu).ravel())
    return np.concatenate(out)


# 3D cases: the benchmark's 256^3 cone and the largest served cone (192^3,
# 360 views of 288^2)
CONE_CASES = {
    "cone256": (inputs.config_c3, (([0, 1, 2], 4), ([11], 0), ([5, 9, 6], 7)), (([0, 1, 2], 4), ([5, 9, 6], 7))),
    "cone192": (lambda: inputs.slice_cone(192), (([0, 1, 2], 3), ([11], 0), ([4, 8], 6)), (([0, 1, 2], 3), ([4, 8], 6))),
}


@pytest.mark.parametrize("name", list(CONE_CASES))
def test_cone_projectors_sampled(ct, name):
    make, fwd_cases, back_cases = CONE_CASES[name]
    g = make()
    G = ct.ct_geom_create(g)
    rng = np.random.default_rng(21)
    x = rng.uniform(0.0, 1.0, g.n_vox).astype(np.float32)
    for rbs, J in fwd_cases:
        err = sampled_forward(ct, g, G, list(rbs), J, x, 2000, 22 + J)
        print(f"[full] {name} forward rbs={rbs} J={J}: rel {err:.2e}", flush=True)
        assert err <= 1e-5
    del x
    r = rng.normal(0.0, 1.0, g.n_rays).astype(np.float32)
    for rbs, J in back_cases:
        rbs = list(rbs)
        gd = torch.full((G.N,), 7.0, device="cuda")
        ct.ct_block_back(G, rbs, J, dev(r), gd)
        got = host(gd)
        views = np.unique(np.concatenate([np.asarray(g.row_blocks[b])[:, 0] for b in rbs]))
        vox = g.col_block_vox(J)
        smp = np.sort(rng.choice(vox, size=48, replace=False))
        ref = []
        for v in smp:
            cand = cone_candidates(g, v, views)
            org, dirn, div = rays.rays_at(g, cand)
            ref.append(clip_sum(g, org, dirn, div, r[cand], v))
        err = rel_l2(got[smp], np.array(ref))
        print(f"[full] {name} back rbs={rbs} J={J}: rel {err:.2e}", flush=True)
        assert err <= 1e-5
        assert max_rel(got[smp], np.array(ref)) <= 1e-5
        other = np.setdiff1d(rng.choice(G.N, size=5000, replace=False), vox)
        assert np.all(got[other] == 7.0)


def test_cone256_epoch_invariants(ct):
    """One epoch of the benchmark's cone configuration (alpha 1, s 3, sync
    per column block): every ray is touched, so afterwards r = y - sum_j z^j
    holds exactly in the kernels' float32 order; the residual falls; and
    z^j after a reset from x equals the oracle's A^j x_J on sampled rays."""
    g = inputs.config_c3()
    G = ct.ct_geom_create(g)
    rng = np.random.default_rng(31)
    x0 = inputs.phantom_for(g, 3000).astype(np.float32)
    x0d = dev(x0)
    p = torch.zeros(G.M, device="cuda")
    for J in range(G.n):
        ct.ct_block_fwd(G, list(range(G.m)), J, x0d, p, flags=ct.CT_ACCUMULATE if J else 0)
    yd = p.clone()
    nnz = ct.ct_geom_block_nnz(G, tau_for(g))
    sc = ct.ct_schedule_create(G, ct.sched_params(1, 1.0, 1.0, 3, 1.0, seed=3000), nnz)
    sol = ct.ct_solver_create(G)

    # reset from a nonzero x: z^j = A^j x_J, checked against the oracle's rows
    xs = rng.uniform(0.0, 1.0, g.n_vox).astype(np.float32)
    xd = dev(xs)
    ct.ct_solver_reset(sol, yd, xd)
    z, r = ct.ct_solver_state(sol)
    smp = np.sort(rng.choice(g.n_rays, size=1500, replace=False))
    org, dirn, div = rays.rays_at(g, smp)
    A_s = siddon.rows_for(g, org, dirn, div)
    zs = host(z[:, torch.as_tensor(smp, device="cuda")])
    for J in (0, 3, 7):
        vox = g.col_block_vox(J)
        xJ = np.zeros(g.n_vox)
        xJ[vox] = xs[vox]
        err = rel_l2(zs[J], A_s @ xJ)
        print(f"[full] cone256 reset z^{J}: rel {err:.2e}", flush=True)
        assert err <= 1e-5
        assert max_rel(zs[J], A_s @ xJ) <= 1e-5

    x = torch.zeros(G.N, device="cuda")
    ct.ct_solver_reset(sol, yd)
    ct.ct_block_epoch(sol, sc, 0, yd, x)
    z, r = ct.ct_solver_state(sol)
    smp = torch.as_tensor(np.sort(rng.choice(g.n_rays, size=1 << 20, replace=False)), device="cuda")
    zs, rs, ys = host(z[:, smp]), host(r[smp]), host(yd[smp])
    s = np.zeros(zs.shape[1], dtype=np.float32)
    for j in range(g.n):
        s = s + zs[j]
    assert np.array_equal(rs, ys - s)
    rel = ct.ct_true_residual(sol, yd, x)
    print(f"[full] cone256 one epoch: true residual {rel:.4f}", flush=True)
    assert np.isfinite(host(x)).all()
    assert 0.0 < rel < 0.9


# The fused forward of the solver's epoch, the kernel the benchmark times, at
# full size: the 2D cases walk slab by slab, the 3D ones run their chunks in
# per-XCD runs.
FUSED_CASES = {
    "fan512": inputs.config_c2,
    "slice1024": lambda: inputs.slice_fan(1024),
    "cone256": inputs.config_c3,
    "cone192": lambda: inputs.slice_cone(192),
}


@pytest.mark.parametrize("name", list(FUSED_CASES))
def test_fused_forward_sampled(ct, name):
    """After a reset from x0, y is set to the float32 sum of the z^j in the
    kernels' order, so the reset gives r = 0 exactly; with r refreshed once per
    epoch every g and mu of the next epoch is then 0 (reading C7), x stays x0
    and each visited z^J is the fused forward's A_{I_G}^J x0_J, checked on
    sampled rays against the oracle's Siddon rows."""
    g = FUSED_CASES[name]()
    G = ct.ct_geom_create(g)
    rng = np.random.default_rng(31)
    x0 = rng.uniform(0.0, 1.0, g.n_vox).astype(np.float32)
    xd = dev(x0)
    sol = ct.ct_solver_create(G, ct.CT_SYNC_EPOCH)
    ct.ct_solver_reset(sol, torch.zeros(G.M, device="cuda"), xd)
    z, r = ct.ct_solver_state(sol)
    zz = z.view(g.n, G.M)
    y = zz[0].clone()
    for j in range(1, g.n):
        y = y + zz[j]
    ct.ct_solver_reset(sol, y, xd)
    torch.cuda.synchronize()
    assert torch.count_nonzero(r).item() == 0
    P = np.full((g.m, g.n), 1.0 / g.m)
    sch = sampler.make_schedule(P, 1, 0.5, 1.0, 2, 1.0, 31)
    x = xd.clone()
    ct.ct_block_epoch(sol, ct.ct_schedule_import(G, sch), 0, y, x)
    torch.cuda.synchronize()
    # x_J = the mean over its groups of x0_J + 0 g: x0 up to the rounding of
    # the mean
    assert rel_l2(host(x).astype(np.float64), x0.astype(np.float64)) <= 1e-6
    cols = sch.cols[sch.epoch_col_ptr[0]:sch.epoch_col_ptr[1]]
    for k, J in enumerate(cols[:3]):
        c = sch.epoch_col_ptr[0] + k
        groups = range(sch.col_group_ptr[c], sch.col_group_ptr[c + 1])
        rbs = [int(b) for q in groups for b in sch.rbs[sch.group_rb_ptr[q]:sch.group_rb_ptr[q + 1]]]
        I = rows_of(g, rbs)
        smp = np.sort(rng.choice(I, size=min(1500, I.size), replace=False))
        org, dirn, div = rays.rays_at(g, smp)
        vox = g.col_block_vox(int(J))
        xJ = np.zeros(g.n_vox)
        xJ[vox] = x0[vox].astype(np.float64)
        ref = siddon.rows_for(g, org, dirn, div) @ xJ
        got = zz[int(J)][torch.as_tensor(smp, device="cuda")].cpu().numpy().astype(np.float64)
        err = rel_l2(got, ref)
        print(f"[full] {name} fused forward J={int(J)} ({len(rbs)} row blocks): rel {err:.2e}", flush=True)
        assert err <= 1e-5
        assert max_rel(got, ref) <= 1e-5
