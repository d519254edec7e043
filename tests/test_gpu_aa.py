"""In-place streaming (one population buffer, LB_STREAM_AA): parity with the
oracle in every storage, with and without chains, on walled, periodic and
mixed boxes; equality with the two-buffer step on the same tile items (FP16
bit for bit, FP32 to a few ulp), after even and odd step counts; checkpoint/resume at even and odd
steps; graph replay; the extended collision (body force, thermal noise); half
the population memory; and the 512^3 large box against its oracle values."""
import os

import numpy as np
import pytest

import oracle
from lbcase import Case, ks_case
from paper_0809_4958_amd import inputs
from test_gpu_parity import STORE, check, compare

pytestmark = pytest.mark.gpu

lbm = pytest.importorskip("paper_0809_4958_amd.lbm")


def say(*a):
    print(*a, flush=True)


def ctx_for(cases, storage, streaming, **kw):
    c0 = cases[0]
    ctx = lbm.Context([c.dims + (c.pmask,) for c in cases], collision=c0.collision, tau=c0.tau,
                      tau_bulk=c0.tau_bulk, ghost_rate=c0.ghost_rate, storage=STORE[storage],
                      reduce_every=c0.reduce_every, streaming=streaming, **kw)
    for k, c in enumerate(cases):
        c.add_to(ctx, k)
    return ctx


def two_buffer_tiles(cases, storage, **kw):
    """A two-buffer context whose boxes all run as tile items."""
    os.environ["LBM_NO_VEC"] = "1"
    try:
        return ctx_for(cases, storage, lbm.STREAM_AB, **kw)
    finally:
        del os.environ["LBM_NO_VEC"]


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_aa_ks_box_with_chain_against_oracle(storage):
    steps = 61
    case = ks_case(28, steps, dt=20, res=9, tau=0.6, n_beads=10, f32_samples=storage != "f64")
    case.reduce_every = 20
    say("case in-place KS 28^3 chain,", storage)
    ob = case.oracle_box()
    assert ob.step(steps) == 0
    ctx = ctx_for([case], storage, lbm.STREAM_AA)
    ctx.step(steps)
    check(compare(ctx, ob, case, storage), storage, "in-place KS")
    mm_o, mm_g = ob.mass_mom(), ctx.read(0, lbm.F_MASS_MOM)
    assert mm_o[0] == mm_g[0] == 60
    assert abs(mm_g[1] - mm_o[1]) < {"f64": 1e-12, "f32": 1e-6, "f16": 1e-5}[storage] * mm_o[1]
    ctx.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_aa_equals_two_buffer_tiles(storage):
    """Same step on the same tile items: FP16 bit for bit; FP32 to a few
    units in the last place of the largest population.  In-place streaming
    runs its own kernel instantiation, and the fused multiply-adds the
    compiler forms there may round differently from the two-buffer one
    (measured: 1 ulp on the 8 interior corner nodes after the first step,
    spreading to ~2% of the nodes at the same size after 7 steps).  An
    addressing mistake moves whole populations, orders of magnitude above
    this bound."""
    cases = [ks_case(n, 40, dt=20, res=9, n_beads=6, config_idx=2, box_idx=i)
             for i, n in enumerate([20, 27])]
    for c in cases:
        c.reduce_every = 10
    say("case in-place vs two buffers, tiles,", storage)
    aa = ctx_for(cases, storage, lbm.STREAM_AA)
    ab = two_buffer_tiles(cases, storage)
    for n in (13, 14):   # odd, then even step counts
        aa.step(n)
        ab.step(n)
        for k, c in enumerate(cases):
            pa, pb = aa.read(k, lbm.F_POP_DEV), ab.read(k, lbm.F_POP_DEV)
            ba, bb = aa.read(k, lbm.F_BEAD_POS, n_beads=6), ab.read(k, lbm.F_BEAD_POS, n_beads=6)
            if storage == "f16":
                assert np.array_equal(pa, pb), (n, k)
                assert np.array_equal(ba, bb)
            else:
                ulp = np.spacing(np.float32(np.abs(pb).max()))
                say(f"after {n} steps box {k}: max |diff| {np.abs(pa - pb).max() / ulp:.1f} ulp, "
                    f"nodes differing {int(np.any(pa != pb, axis=0).sum())}")
                assert np.abs(pa - pb).max() <= 8 * ulp, (n, k)
                assert np.abs(ba - bb).max() < 1e-6
            ma, mb = aa.read(k, lbm.F_MASS_MOM), ab.read(k, lbm.F_MASS_MOM)
            # FP32: ulp differences of the populations reach the FP64 mass sum
            assert ma[0] == mb[0] and abs(ma[1] - mb[1]) < (1e-12 if storage == "f16" else 1e-9) * mb[1]
    aa.close()
    ab.close()


def test_aa_periodic_and_mixed_fp64():
    rng = np.random.default_rng(21)
    dims_p = (12, 10, 14)
    pos, _ = inputs.chain_init(6, [5.5, 4.5, 6.5], rng)
    per = Case(dims_p, collision=oracle.MRT, tau=0.8, tau_bulk=0.9, ghost_rate=1.2, periodic_mask=7,
               u0=1e-2 * rng.standard_normal(dims_p[::-1] + (3,)),
               chains=[dict(pos=pos, vel=1e-2 * rng.standard_normal((6, 3)), fix_com=False,
                            zeta=3.0, anchor=[5.5, 4.5, 6.5])], reduce_every=5)
    dims_m = (17, 13, 6)
    mixed = Case(dims_m, collision=oracle.MRT, tau=0.8, tau_bulk=0.9, ghost_rate=1.2, periodic_mask=5,
                 bc=(oracle.BC_AFFINE, inputs.ou_strain(41, rng, 20.0, 1e-3), 0, 1, 0),
                 u0=1e-3 * rng.standard_normal(dims_m[::-1] + (3,)), reduce_every=5)
    say("case in-place periodic + mixed, fp64")
    ctx = ctx_for([per, mixed], "f64", lbm.STREAM_AA)
    ctx.step(35)
    for k, c in enumerate((per, mixed)):
        ob = c.oracle_box()
        assert ob.step(35) == 0
        check(compare(ctx, ob, c, "f64", box=k), "f64", f"in-place box {k}")
    ctx.close()


@pytest.mark.parametrize("storage", ["f64", "f16"])
def test_aa_extended_collision(storage):
    steps = 40
    case = ks_case(24, steps, dt=20, res=9, tau=0.6, n_beads=8, f32_samples=storage != "f64")
    case.body = (2e-6 * np.random.default_rng(3).standard_normal((9, 3)), 0, 5)
    case.kT, case.seed = 2e-6, 77
    say("case in-place body force + thermal,", storage)
    ob = case.oracle_box()
    assert ob.step(steps) == 0
    ctx = ctx_for([case], storage, lbm.STREAM_AA)
    ctx.set_thermal(case.kT, case.seed)
    ctx.step(steps)
    check(compare(ctx, ob, case, storage), storage, "in-place extended")
    ctx.close()


@pytest.mark.parametrize("restart", [30, 31])
@pytest.mark.parametrize("storage", ["f64", "f16"])
def test_aa_checkpoint_resume_and_graphs_bitwise(storage, restart):
    case = ks_case(20, 60, dt=20, res=9, n_beads=6, config_idx=4)
    full = ctx_for([case], storage, lbm.STREAM_AA)
    full.step(60)
    ref = full.read(0, lbm.F_POP_DEV)
    ref_p = full.read(0, lbm.F_BEAD_POS, n_beads=6)
    graphed = ctx_for([case], storage, lbm.STREAM_AA, graph_steps=7)
    graphed.step(60)
    assert np.array_equal(graphed.read(0, lbm.F_POP_DEV), ref)
    half = ctx_for([case], storage, lbm.STREAM_AA)
    half.step(restart)
    pop = half.read(0, lbm.F_POP_DEV)
    bp = half.read(0, lbm.F_BEAD_REL, n_beads=6)
    bv = half.read(0, lbm.F_BEAD_VEL, n_beads=6)
    fresh = ctx_for([case], storage, lbm.STREAM_AA)
    fresh.write_state(0, lbm.F_POP_DEV, pop)      # uploaded at step 0, then moved
    fresh.write_state(0, lbm.F_STEP, restart)     # to the restart's parity
    fresh.write_state(0, lbm.F_BEAD_REL, bp)
    fresh.write_state(0, lbm.F_BEAD_VEL, bv)
    assert np.array_equal(fresh.read(0, lbm.F_POP_DEV), pop)
    fresh.step(60 - restart)
    assert fresh.read(0, lbm.F_STEP) == 60
    assert np.array_equal(fresh.read(0, lbm.F_POP_DEV), ref)
    assert np.array_equal(fresh.read(0, lbm.F_BEAD_POS, n_beads=6), ref_p)
    for c in (full, graphed, half, fresh):
        c.close()
    with pytest.raises(lbm.LBError) as e:
        ctx_for([case], storage, lbm.STREAM_AA).autotune(1)
    assert e.value.status == lbm.ERR_STATE


def test_aa_halves_the_population_memory():
    import torch
    n = 160
    sizes = {}
    for streaming in (lbm.STREAM_AB, lbm.STREAM_AA):
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        ctx = lbm.Context([(n, n, n)], collision=lbm.MRT, tau=0.6, tau_bulk=0.6,
                          storage=lbm.STORE_F16DEV, torch_alloc=True, streaming=streaming)
        sizes[streaming] = torch.cuda.memory_allocated() - before
        ctx.close()
    pop = 19 * n ** 3 * 2
    say("context memory: two buffers", sizes[lbm.STREAM_AB], "one buffer", sizes[lbm.STREAM_AA],
        "population set", pop)
    assert sizes[lbm.STREAM_AB] - sizes[lbm.STREAM_AA] >= pop
    assert sizes[lbm.STREAM_AA] < 1.1 * pop
