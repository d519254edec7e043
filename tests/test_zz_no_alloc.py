"""The allocation-free site readout (lb_read_sites_noalloc) through the C ABI
against the allocating one (lb_read_sites): bitwise the same populations on
two calls in a row, the second with fewer sites, after steps in between; the
site-count limit and the call-order rule are reported as errors."""
import numpy as np
import pytest

from lbcase import ks_case

pytestmark = pytest.mark.gpu

lbm = pytest.importorskip("paper_0809_4958_amd.lbm")


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("storage", [lbm.STORE_F64, lbm.STORE_F32, lbm.STORE_F16DEV])
def test_noalloc_sites_match_allocating_readout(storage):
    say("case no-alloc site readout, storage", storage)
    cases = [ks_case(n, 40, dt=20, res=9, n_beads=6, config_idx=2, box_idx=i)
             for i, n in enumerate([24, 32])]
    ctx = lbm.Context([c.dims for c in cases], collision=lbm.MRT, tau=0.6, tau_bulk=0.6,
                      storage=storage, reduce_every=10)
    for k, c in enumerate(cases):
        c.add_to(ctx, k)
    # the device tables are built by the first step or readout
    with pytest.raises(lbm.LBError) as e:
        ctx.read_sites_noalloc(0, [[1, 1, 1]])
    assert e.value.status == lbm.ERR_STATE
    rng = np.random.default_rng(12)
    ctx.step(15)
    for box, n_sites in ((1, 20000), (0, 777)):
        n = cases[box].dims[0]
        xyz = rng.integers(1, n - 1, size=(n_sites, 3)).astype(np.int32)
        a = ctx.read_sites(box, xyz)
        b = ctx.read_sites_noalloc(box, xyz)
        say(f"box {box}: {n_sites} sites, max |diff| {np.abs(a - b).max():.3e}")
        assert np.array_equal(a, b)
        ctx.step(5)
    with pytest.raises(lbm.LBError) as e:
        ctx.read_sites_noalloc(0, np.ones((32769, 3), dtype=np.int32))
    assert e.value.status == lbm.ERR_ARG
    assert ctx.read_sites_noalloc(0, np.zeros((0, 3), dtype=np.int32)).shape == (0, 19)
    ctx.close()
