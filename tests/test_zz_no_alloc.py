"""The no-allocation density entry point (ct_geom_block_nnz_static) against
ct_geom_block_nnz, through the C ABI: the same counts, exactly, on two calls
in a row, the second with a smaller geometry (the static counter array keeps
the last call's contents, so the second call must clear what it uses)."""
import numpy as np
import pytest

from paper_1709_00953_amd import inputs
from tests.parity_util import tau_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ct():
    from paper_1709_00953_amd import ct as _ct
    _ct.lib()
    return _ct


def test_static_nnz_equals_nnz_on_two_calls(ct):
    big = inputs.config_p3()                                   # 12 x 8 blocks, 48^3, 360 views
    small = inputs.cone3d(12, 2.0, 30, 20, 3.0, 500.0, 1000.0, m=3, bz=2, bxy=1)   # 3 x 2 blocks
    assert big.m * big.n > small.m * small.n
    for g in (big, small):
        G = ct.ct_geom_create(g)
        ref = ct.ct_geom_block_nnz(G, tau_for(g))             # also puts the tables on the device
        out = np.full((g.m, g.n), -7, dtype=np.int64)
        got = ct.ct_geom_block_nnz_static(G, tau_for(g), out=out)
        assert got is out
        print(f"[noalloc] {g.m}x{g.n} blocks, {int(ref.sum())} pairs", flush=True)
        np.testing.assert_array_equal(got, ref)
        assert ref.sum() > 0


def test_static_nnz_needs_resident_tables(ct):
    g = inputs.config_c1()
    G = ct.ct_geom_create(g)
    with pytest.raises(ct.CtError):
        ct.ct_geom_block_nnz_static(G, tau_for(g))             # tables not uploaded yet
    ref = ct.ct_geom_block_nnz(G, tau_for(g))
    np.testing.assert_array_equal(ct.ct_geom_block_nnz_static(G, tau_for(g)), ref)
