"""CPU check of the float32 ray distance that the curved-fan back-projection
uses in place of a float64 product per candidate.

On an equi-angular detector, bin b's ray is the reference bin kr's ray
turned by e = pu (b - kr).  A point at lateral offset X and depth R from the
reference ray is then at signed distance X cos e - R sin e from ray b, with
cos e ~ 1 - e^2/2 and sin e ~ e - e^3/6 for |e| <= 2e-2.  The test forms X
and R in float32 from the tile centre's float64 values and the voxel's small
offsets, exactly as the back-projection does, and compares with the float64
distance cos(g_b) B - sin(g_b) A of the view frame (Sec. II-A geometry) over
random tiles of the 512^2 fan (0.5 mm pixels, 1e-3 rad bins, source at
500 mm), eight bins around each voxel's shadow.  No GPU needed.
"""
import numpy as np

f32 = np.float32


def _fma32(a, b, c):
    """float32 fused multiply-add: the exact product and sum, rounded once."""
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(f32)


def test_reference_bin_distance_matches_float64():
    rng = np.random.default_rng(7)
    sid, pu, nu, vx = 500.0, 1e-3, 768, 0.5
    c0 = 0.5 * (nu - 1)
    n_tiles = 300
    th = rng.uniform(0.0, 2.0 * np.pi, n_tiles)
    s17 = rng.choice([-1.0, 1.0], n_tiles)
    eA = np.stack([np.cos(th), np.sin(th)], 1)
    eB = s17[:, None] * np.stack([-np.sin(th), np.cos(th)], 1)
    w17 = eA[:, 0] * eB[:, 1] - eA[:, 1] * eB[:, 0]
    q0 = rng.uniform(-125.0, 125.0, (n_tiles, 2)) + sid * eA        # tile centre from the source
    Ac, Bc = (q0 * eA).sum(1), (q0 * eB).sum(1)
    ax, ay, bx, by = eA[:, 0] * vx, eA[:, 1] * vx, eB[:, 0] * vx, eB[:, 1] * vx
    bc = np.arctan2(Bc, Ac) / pu + c0
    kr = np.clip(np.floor(bc + 0.5), 0, nu - 1)
    g = (kr - c0) * pu
    p, q = w17 * np.cos(g), w17 * np.sin(g)
    Xx, Xy = f32(p * bx - q * ax), f32(p * by - q * ay)
    Yx, Yy = f32(p * ax + q * bx), f32(p * ay + q * by)
    Xc, Rc = f32(p * Bc - q * Ac), f32(p * Ac + q * Bc)
    # voxel offsets from the tile centre (8 x 8 tile) and bins around each shadow
    off = np.arange(8, dtype=f32) - f32(3.5)
    lx, ly = [a.ravel() for a in np.meshgrid(off, off, indexing="ij")]
    lx, ly = lx[None, :, None], ly[None, :, None]
    T = lambda a: a[:, None, None]                                       # noqa: E731
    A = T(Ac) + lx.astype(np.float64) * T(ax) + ly.astype(np.float64) * T(ay)
    B = T(Bc) + lx.astype(np.float64) * T(bx) + ly.astype(np.float64) * T(by)
    ub = np.floor(np.arctan2(B, A) / pu + c0)
    b = ub + np.arange(-3, 5)[None, None, :]
    gb = (b - c0) * pu
    ref = T(w17) * (np.cos(gb) * B - np.sin(gb) * A)
    # the kernel's float32 operations
    Xs = T(Xc) + _fma32(np.broadcast_to(ly, (n_tiles, 64, 1)), np.broadcast_to(T(Xy), (n_tiles, 64, 1)),
                        (lx * T(Xx)).astype(f32))
    Rs = T(Rc) + _fma32(np.broadcast_to(ly, (n_tiles, 64, 1)), np.broadcast_to(T(Yy), (n_tiles, 64, 1)),
                        (lx * T(Yx)).astype(f32))
    e = ((b - T(kr)).astype(f32) * f32(pu)).astype(f32)
    assert np.abs(e).max() <= 2e-2
    e2 = (e * e).astype(f32)
    sn = (e * _fma32(e2, np.full_like(e2, f32(-1.0 / 6.0)), np.ones_like(e2))).astype(f32)
    cs = _fma32(e2, np.full_like(e2, f32(-0.5)), np.ones_like(e2))
    got = _fma32(cs, np.broadcast_to(Xs, e.shape), (-(sn * np.broadcast_to(Rs, e.shape))).astype(f32))
    err = np.abs(got.astype(np.float64) - ref)
    # a few 1e-7 of the 0.5 mm pixel: far below the 1e-5 parity tolerance
    assert err.max() <= 1.5e-6, err.max()


def test_turned_next_bin_distance_matches_float64():
    """Where a voxel has at most two candidate bins, the second's distance is
    the first's turned by one pitch: X' = X cos pu - Y sin pu with the depth
    Y = X sin e + R cos e in the first bin's frame, in float32 as the kernel
    forms it, against the float64 distance of bin b + 1."""
    rng = np.random.default_rng(8)
    sid, pu, nu, vx = 500.0, 1e-3, 768, 0.5
    c0 = 0.5 * (nu - 1)
    n = 20000
    th = rng.uniform(0.0, 2.0 * np.pi, n)
    s17 = rng.choice([-1.0, 1.0], n)
    eA = np.stack([np.cos(th), np.sin(th)], 1)
    eB = s17[:, None] * np.stack([-np.sin(th), np.cos(th)], 1)
    w17 = eA[:, 0] * eB[:, 1] - eA[:, 1] * eB[:, 0]
    q = rng.uniform(-125.0, 125.0, (n, 2)) + sid * eA                   # voxel centre from the source
    A, B = (q * eA).sum(1), (q * eB).sum(1)
    bc = np.arctan2(B, A) / pu + c0
    kr = np.clip(np.floor(bc + 0.5) + rng.integers(-3, 4, n), 0, nu - 1)   # reference bin near the shadow
    g = (kr - c0) * pu
    p, qq = w17 * np.cos(g), w17 * np.sin(g)
    Xs, Rs = f32(p * B - qq * A), f32(p * A + qq * B)                    # float32 X, R (rounded once)
    b0 = np.floor(bc + rng.uniform(-0.7, 0.7, n))
    e = ((b0 - kr).astype(f32) * f32(pu)).astype(f32)
    assert np.abs(e).max() <= 2e-2
    one = np.ones(n, dtype=f32)
    e2 = (e * e).astype(f32)
    sn = (e * _fma32(e2, np.full(n, f32(-1.0 / 6.0)), one)).astype(f32)
    cs = _fma32(e2, np.full(n, f32(-0.5)), one)
    d0 = _fma32(cs, Xs, (-(sn * Rs)).astype(f32))
    y0 = _fma32(sn, Xs, (cs * Rs).astype(f32))
    cp, sp = np.full(n, f32(np.cos(pu))), f32(np.sin(pu))
    d1 = _fma32(d0, cp, (-(y0 * sp)).astype(f32))
    for bb, got in ((b0, d0), (b0 + 1, d1)):
        gb = (bb - c0) * pu
        ref = w17 * (np.cos(gb) * B - np.sin(gb) * A)
        err = np.abs(got.astype(np.float64) - ref)
        assert err.max() <= 1.5e-6, err.max()


def test_polynomial_angle_bound():
    """The cubic sine and quadratic cosine at |e| <= 2e-2 against float64."""
    e = np.linspace(-2e-2, 2e-2, 100001)
    assert np.abs(e - e ** 3 / 6 - np.sin(e)).max() <= 3e-11
    assert np.abs(1 - e ** 2 / 2 - np.cos(e)).max() <= 7e-9
