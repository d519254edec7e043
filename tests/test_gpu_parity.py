"""GPU parity: the HIP library against the FP64 oracle on identical seeded inputs.

Tolerances (relative L2 over the interior, velocity u = j/rho):
FP64 storage 1e-12, FP32 storage 1e-5, FP16-deviation storage 1e-3.
"""
import sys

import numpy as np
import pytest

import oracle
from lbcase import CHAIN_BOND, Case, bead_errors, cfg0_case, ks_case, max_rel, rel_l2
from paper_0809_4958_amd import inputs

pytestmark = pytest.mark.gpu

lbm = pytest.importorskip("paper_0809_4958_amd.lbm")

STORE = {"f64": 0, "f32": 1, "f16": 2}
TOL_U = {"f64": 1e-12, "f32": 1e-5, "f16": 1e-3}
# Population deviations f_i - w_i rho0 in FP64 mode.  The oracle stores
# absolute f_i (magnitude up to 1/3) and so carries an absolute rounding of
# about eps * 1/3 = 4e-17 per operation, while the deviations it is compared
# on are O(w_i u) ~ 1e-5..1e-4; over a few hundred steps that alone gives
# relative differences of ~1e-12..1e-11 (the library computes on deviations
# and is the more accurate side).  The bound 1e-10 leaves a 10x margin.
TOL_POP_F64 = 1e-10


# Bounds of every compared field, per storage.  rel-L2 norms (u, population
# deviations, beads): the relative velocity tolerances of the precision
# targets, TOL_U (FP64 population deviations: TOL_POP_F64).  Per-node
# max-norms (largest error of any node, axis or bead over the field's largest
# magnitude): TOL_MAX.  In FP64 they share the rel-L2 bounds.  In FP16 one
# rounding of a stored deviation h = (f/w - rho0) 2^10 is up to 2^-11 = 4.9e-4
# of it; the node with the largest error has taken several roundings of the
# same sign, so the max-norm bound is 8 half-ulps, 3.9e-3 -> 4e-3 (measured:
# up to 1.3e-3, 2-4x the rel-L2).  In FP32 the largest errors sit on the
# nodes next to extended chains, set by FP32 bead coordinates (ulp 2^-24 x
# 40 = 2.4e-6 lattice units, accumulated over the substeps) in the
# interpolation and spreading weights and by the impulse m(V' - V): 1e-4
# (measured: up to 1.5e-5, 10x the rel-L2).
TOL_MAX = {"f64": 1e-12, "f32": 1e-4, "f16": 4e-3}
FIELDS = ("u", "pop", "bead_pos", "bead_vel")
TOL = {}
for _st in TOL_U:
    TOL[_st] = {}
    for _f in FIELDS:
        l2 = TOL_POP_F64 if _st == "f64" and _f == "pop" else TOL_U[_st]
        TOL[_st][_f] = l2
        TOL[_st][_f + "_max"] = l2 if _st == "f64" else TOL_MAX[_st]


def check(r, storage, label="", skip=()):
    """Prints every error of a comparison and asserts each against its bound."""
    say(label, storage, {k: f"{v:.3e}" for k, v in r.items()})
    bad = {k: v for k, v in r.items() if k in TOL[storage] and k not in skip and not v < TOL[storage][k]}
    assert not bad, f"{label} {storage}: over the bound: {bad}"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_ctx(case, storage="f64", **kw):
    ctx = lbm.Context([case.dims + (case.pmask,)], collision=case.collision, tau=case.tau,
                      tau_bulk=case.tau_bulk, ghost_rate=case.ghost_rate, storage=STORE[storage],
                      reduce_every=case.reduce_every, **kw)
    case.add_to(ctx, 0)
    return ctx


def compare(ctx, ob, case, storage, box=0, strict=True):
    """Errors of every field of one box against the oracle (strict=False: the
    context holds a latched error and its fields are those of the last good
    step)."""
    def rd(field, **kw):
        return ctx.read(box, field, **kw) if strict else ctx.read(box, field, strict=False, **kw)[0]

    mask = ob.interior_mask()
    _, u_o = ob.rho_u()
    u_g = rd(lbm.F_U)
    f_o = ob.pop()
    f_g = rd(lbm.F_POP)
    _, w = oracle.lattice()
    dev_o = f_o - w[:, None, None, None]
    dev_g = f_g - w[:, None, None, None]
    res = {"u": rel_l2(u_g, u_o, mask), "pop": rel_l2(dev_g[:, mask], dev_o[:, mask]),
           "u_max": max_rel(u_g[mask], u_o[mask]), "pop_max": max_rel(dev_g[:, mask], dev_o[:, mask])}
    if case.n_beads:
        p_o, v_o = ob.beads()
        p_g = rd(lbm.F_BEAD_POS, n_beads=case.n_beads)
        v_g = rd(lbm.F_BEAD_VEL, n_beads=case.n_beads)
        res.update(bead_errors(p_g, v_g, p_o, v_o, case.chains, np.abs(u_o[mask]).max()))
    return res


def test_cfg0_fp64_full_run():
    """32^3 BGK tau 0.8, affine OU boundary, 16-bead chain, 200 steps: 1e-12."""
    case = cfg0_case()
    say("case cfg0 fp64 32^3 200 steps")
    ob = case.oracle_box()
    assert ob.step(200) == 0
    ctx = make_ctx(case, "f64")
    ctx.step(200)
    ctx.sync()
    assert ctx.read(0, lbm.F_STEP) == 200
    r = compare(ctx, ob, case, "f64")
    check(r, "f64", "cfg0")
    mm_o = ob.mass_mom()
    mm_g = ctx.read(0, lbm.F_MASS_MOM)
    assert mm_g[0] == mm_o[0] == 200
    assert abs(mm_g[1] - mm_o[1]) / mm_o[1] < 1e-13
    assert np.abs(mm_g[2:] - mm_o[2:]).max() < 1e-12 * mm_o[1]


@pytest.mark.parametrize("coll", [oracle.BGK, oracle.MRT])
def test_ks_sampled_fp64(coll):
    """KS-driven sampled boundary, ragged tiles (26^3), MRT/BGK, chain: 1e-12."""
    case = ks_case(26, 60, dt=20, res=9, tau=0.6, n_beads=8, collision=coll, f32_samples=False)
    say("case ks fp64", coll)
    ob = case.oracle_box()
    assert ob.step(60) == 0
    ctx = make_ctx(case, "f64")
    ctx.step(60)
    r = compare(ctx, ob, case, "f64")
    check(r, "f64", f"ks coll {coll}")


def test_periodic_and_mixed_axes_fp64():
    """Periodic x and z with equilibrium walls in y (odd sizes), chain without
    the centre-of-mass pin crossing no wall."""
    rng = np.random.default_rng(5)
    dims = (17, 13, 6)
    u0 = 1e-3 * rng.standard_normal(dims[::-1] + (3,))
    A = inputs.ou_strain(41, rng, corr_steps=20.0, rms=1e-3)
    pos, vel = inputs.chain_init(5, [8.3, 6.1, 2.7], rng)
    chain = dict(pos=pos, vel=1e-3 * rng.standard_normal((5, 3)), fix_com=False, anchor=[8.3, 6.1, 2.7])
    case = Case(dims, collision=oracle.MRT, tau=0.7, tau_bulk=0.9, ghost_rate=1.2, periodic_mask=5,
                bc=(oracle.BC_AFFINE, A, 0, 1, 0), u0=u0, chains=[chain], reduce_every=7)
    say("case periodic-mixed fp64")
    ob = case.oracle_box()
    assert ob.step(40) == 0
    ctx = make_ctx(case, "f64")
    ctx.step(40)
    r = compare(ctx, ob, case, "f64")
    check(r, "f64", "periodic-mixed")
    mm_o, mm_g = ob.mass_mom(), ctx.read(0, lbm.F_MASS_MOM)
    assert mm_g[0] == mm_o[0] == 35
    assert abs(mm_g[1] - mm_o[1]) < 1e-12 * mm_o[1]


def test_fully_periodic_conservation_fp64():
    rng = np.random.default_rng(8)
    dims = (12, 10, 14)
    u0 = 1e-2 * rng.standard_normal(dims[::-1] + (3,))
    pos, _ = inputs.chain_init(6, [5.5, 4.5, 6.5], rng)
    chain = dict(pos=pos, vel=1e-2 * rng.standard_normal((6, 3)), fix_com=False, zeta=3.0,
                 anchor=[5.5, 4.5, 6.5])
    case = Case(dims, collision=oracle.BGK, tau=0.9, periodic_mask=7, u0=u0, chains=[chain])
    say("case fully periodic fp64")
    ob = case.oracle_box()
    assert ob.step(30) == 0
    ctx = make_ctx(case, "f64")
    ctx.step(30)
    r = compare(ctx, ob, case, "f64")
    check(r, "f64", "fully periodic")


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_periodic_and_walled_boxes_with_chains(storage):
    """One context holding a fully periodic box, whose chain's spread force the
    step kernel gathers, and a walled box, whose chain couples through the
    force pass (which skips the periodic box's chain but still ends the
    step): each box against its own oracle box, check records included.  In
    FP32 and FP16 storage the walled box, which alone would be a row box,
    runs as a tile box beside the periodic one."""
    rng = np.random.default_rng(11)
    dp = (12, 10, 14)
    posp, _ = inputs.chain_init(6, [5.5, 4.5, 6.5], rng)
    per = Case(dp, collision=oracle.BGK, tau=0.9, periodic_mask=7,
               u0=1e-2 * rng.standard_normal(dp[::-1] + (3,)),
               chains=[dict(pos=posp, vel=1e-2 * rng.standard_normal((6, 3)), fix_com=False,
                            zeta=3.0, anchor=[5.5, 4.5, 6.5])], reduce_every=5)
    dw = (16, 14, 12)
    xc = [7.5, 6.5, 5.5]
    posw, velw = inputs.chain_init(8, xc, rng, bond=CHAIN_BOND)
    walled = Case(dw, collision=oracle.BGK, tau=0.9,
                  bc=(oracle.BC_AFFINE, inputs.ou_strain(41, rng, corr_steps=20.0, rms=1e-3), 0, 1, 0),
                  u0=1e-3 * rng.standard_normal(dw[::-1] + (3,)),
                  chains=[dict(pos=posw, vel=velw, anchor=xc)], reduce_every=5)
    cases = [per, walled]
    say("case periodic + walled boxes with chains,", storage)
    ctx = lbm.Context([c.dims + (c.pmask,) for c in cases], collision=oracle.BGK, tau=0.9,
                      tau_bulk=0.9, storage=STORE[storage], reduce_every=5)
    for k, c in enumerate(cases):
        c.add_to(ctx, k)
    ctx.step(40)
    assert ctx.sync_status() == lbm.OK
    assert ctx.read(0, lbm.F_STEP) == 40
    for k, c in enumerate(cases):
        ob = c.oracle_box()
        assert ob.step(40) == 0
        r = compare(ctx, ob, c, storage, box=k)
        check(r, storage, f"box {k} {c.dims}")
        mm_o, mm_g = ob.mass_mom(), ctx.read(k, lbm.F_MASS_MOM)
        assert mm_g[0] == mm_o[0] == 40
        assert abs(mm_g[1] - mm_o[1]) < {"f64": 1e-12, "f32": 1e-6, "f16": 1e-5}[storage] * mm_o[1]
    ctx.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_reduced_precision_storage(storage):
    """FP32 compute with FP32 / FP16-deviation storage vs the FP64 oracle."""
    case = ks_case(32, 400, dt=20, res=17, tau=0.6, n_beads=16)
    say("case ks", storage, "32^3 400 steps")
    ob = case.oracle_box()
    assert ob.step(400) == 0
    ctx = make_ctx(case, storage)
    ctx.step(400)
    r = compare(ctx, ob, case, storage)
    check(r, storage, "ks 32^3 400 steps")


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("layout", ["one_chain", "three_chains"])
def test_row_gather_many_beads(storage, layout):
    """Spreading into row items from many beads near the same rows of a 40^3
    KS box: "one_chain" has one 200-bead chain at the centre (four 64-record
    chunks per wavefront), "three_chains" three 120-bead chains at the same
    centre (several chains per item, 360 records).  Bead masses keep the
    whole load at half a fluid node."""
    n, steps = 40, 100
    units, u0, faces = inputs.ks_box_inputs(1, 3, n=n, tau=0.6, n_steps=steps, dt=20, res=17)
    xc = np.full(3, (n - 1) / 2.0)
    sizes = [200] if layout == "one_chain" else [120, 120, 120]
    chains = []
    for k, nb in enumerate(sizes):
        pos, vel = inputs.chain_init(nb, xc, inputs.rng(1, 10 + k), bond=CHAIN_BOND)
        chains.append(dict(pos=pos, vel=vel, anchor=xc, mass=0.5 / sum(sizes)))
    case = Case((n, n, n), collision=oracle.MRT, tau=0.6, tau_bulk=0.6, ghost_rate=1.0,
                bc=(oracle.BC_SAMPLED, faces.astype(np.float32), 0, 20, 17), u0=u0, chains=chains)
    say("case gather", layout, storage, f"{n}^3 {steps} steps, chains {sizes}")
    ob = case.oracle_box()
    assert ob.step(steps) == 0
    ctx = make_ctx(case, storage)
    ctx.step(steps)
    r = compare(ctx, ob, case, storage)
    check(r, storage, layout)


def test_edge_shapes_fp64():
    """Smallest box (one interior node), long thin and ragged boxes in one batch."""
    rng = np.random.default_rng(3)
    cases = []
    for dims in [(3, 3, 3), (40, 4, 5), (7, 33, 9)]:
        A = inputs.ou_strain(11, rng, corr_steps=10.0, rms=1e-2)
        cases.append(Case(dims, collision=oracle.MRT, tau=0.75, tau_bulk=1.1,
                          bc=(oracle.BC_AFFINE, A, 0, 2, 0)))
    ctx = lbm.Context([c.dims for c in cases], collision=lbm.MRT, tau=0.75, tau_bulk=1.1,
                      storage=0)
    for k, c in enumerate(cases):
        c.add_to(ctx, k)
    ctx.step(20)
    for k, c in enumerate(cases):
        ob = c.oracle_box()
        assert ob.step(20) == 0
        r = compare(ctx, ob, c, "f64", box=k)
        check(r, "f64", f"edge {c.dims}")


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_batched_equals_single_bitwise(storage):
    """Uneven boxes in one launch give bitwise the same populations and beads
    as each box run alone."""
    cases = [ks_case(n, 40, dt=20, res=9, n_beads=6, config_idx=2, box_idx=i)
             for i, n in enumerate([20, 32, 24])]
    batch = lbm.Context([c.dims for c in cases], collision=lbm.MRT, tau=0.6, tau_bulk=0.6,
                        storage=STORE[storage], reduce_every=10)
    for k, c in enumerate(cases):
        c.add_to(batch, k)
    batch.step(40)
    for k, c in enumerate(cases):
        single = make_ctx(c, storage)
        single.step(40)
        a = batch.read(k, lbm.F_POP)
        b = single.read(0, lbm.F_POP)
        assert np.array_equal(a, b), f"box {k}"
        pa = batch.read(k, lbm.F_BEAD_POS, n_beads=c.n_beads)
        pb = single.read(0, lbm.F_BEAD_POS, n_beads=c.n_beads)
        assert np.array_equal(pa, pb)
        single.close()


def test_graph_replay_and_determinism_bitwise():
    case = ks_case(24, 60, dt=20, res=9, n_beads=8, config_idx=3)
    runs = []
    for graph_steps, timed in ((0, False), (0, False), (7, False), (7, True), (0, True)):
        ctx = make_ctx(case, "f16", graph_steps=graph_steps)
        ctx.step(25)
        # timed: per-step HIP events (inside the two alternating graphs when
        # graph_steps > 0); the timed steps must compute the same state
        ctx.set_timing(timed)
        ctx.step(35)
        if timed:
            t = ctx.timing()
            assert t[1] > 0 and t[2] > 0 and t[0] >= t[1]
        runs.append((ctx.read(0, lbm.F_POP), ctx.read(0, lbm.F_BEAD_POS, n_beads=8),
                     ctx.read(0, lbm.F_MASS_MOM)))
        ctx.close()
    for r in runs[1:]:
        assert np.array_equal(r[0], runs[0][0])
        assert np.array_equal(r[1], runs[0][1])
        assert np.array_equal(r[2], runs[0][2])


def test_check_steps_with_graph_phases_bitwise():
    """Mass/momentum checks fall on the same steps whether the steps run one
    by one or from graphs captured for one check phase (graph length a
    multiple of the check interval, leaving the other steps' check launches
    out), with the starting phase changing between calls; the state and
    every check record are bitwise the same, and each record belongs to the
    last check step."""
    case = ks_case(20, 60, dt=20, res=9, n_beads=6, config_idx=4)
    case.reduce_every = 5
    calls = (3, 20, 4, 10, 13)  # starting phases 0, 3, 3, 2, 2 (mod 5)
    runs = []
    for gs in (0, 10, 5):
        ctx = make_ctx(case, "f16", graph_steps=gs)
        recs, done = [], 0
        for n in calls:
            ctx.step(n)
            done += n
            mm = ctx.read(0, lbm.F_MASS_MOM)
            recs.append(mm)
            if done >= 5:
                assert mm[0] == 5 * (done // 5), (gs, done, mm[0])
        runs.append((recs, ctx.read(0, lbm.F_POP), ctx.sync_status()))
        ctx.close()
    assert runs[0][2] == lbm.OK
    for recs, pop, status in runs[1:]:
        assert status == lbm.OK
        for a, b in zip(recs, runs[0][0]):
            assert np.array_equal(a, b)
        assert np.array_equal(pop, runs[0][1])
    # and the last record is the oracle's mass and momentum at that step (FP16
    # storage: the state itself differs from the FP64 one at the 1e-4 level)
    ob = case.oracle_box()
    assert ob.step(sum(calls)) == 0
    mm_o, mm_g = ob.mass_mom(), runs[0][0][-1]
    assert mm_o[0] == mm_g[0] == 50
    assert abs(mm_g[1] - mm_o[1]) / mm_o[1] < 1e-5
    assert np.abs(mm_g[2:] - mm_o[2:]).max() < 1e-2 * np.abs(mm_o[2:]).max() + 1e-9


def test_tune_cache_round_trip(tmp_path):
    """The autotuner's launch shape (item sizes per box size, grid) written to
    the cache is what a new context over the same boxes reads back, and the
    two compute the same state bitwise."""
    case = ks_case(32, 40, dt=20, res=9, n_beads=8, config_idx=2)
    cache = str(tmp_path / "tune.jsonl")
    a = make_ctx(case, "f16", tune_cache=cache)
    a.autotune(1)
    a.step(20)
    desc_a = a.describe()
    b = make_ctx(case, "f16", tune_cache=cache)
    b.step(20)
    desc_b = b.describe()
    say("tuned:", desc_a, "| from cache:", desc_b)
    assert desc_a == desc_b
    assert np.array_equal(a.read(0, lbm.F_POP), b.read(0, lbm.F_POP))
    a.close()
    b.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_checkpoint_resume_bitwise(storage):
    case = ks_case(20, 60, dt=20, res=9, n_beads=6, config_idx=4)
    full = make_ctx(case, storage)
    full.step(60)
    ref = full.read(0, lbm.F_POP)
    ref_p = full.read(0, lbm.F_BEAD_POS, n_beads=6)
    half = make_ctx(case, storage)
    half.step(30)
    pop = half.read(0, lbm.F_POP_DEV)
    bp = half.read(0, lbm.F_BEAD_REL, n_beads=6)
    bv = half.read(0, lbm.F_BEAD_VEL, n_beads=6)
    fresh = make_ctx(case, storage)
    fresh.write_state(0, lbm.F_STEP, 30)
    fresh.write_state(0, lbm.F_POP_DEV, pop)
    fresh.write_state(0, lbm.F_BEAD_REL, bp)
    fresh.write_state(0, lbm.F_BEAD_VEL, bv)
    fresh.step(30)
    assert fresh.read(0, lbm.F_STEP) == 60
    assert np.array_equal(fresh.read(0, lbm.F_POP), ref)
    assert np.array_equal(fresh.read(0, lbm.F_BEAD_POS, n_beads=6), ref_p)
    # the absolute-population round trip is exact up to the rounding of w_i rho0 + d_i
    again = make_ctx(case, storage)
    again.write_state(0, lbm.F_STEP, 30)
    again.write_state(0, lbm.F_POP, half.read(0, lbm.F_POP))
    again.write_state(0, lbm.F_BEAD_POS, half.read(0, lbm.F_BEAD_POS, n_beads=6))
    again.write_state(0, lbm.F_BEAD_VEL, bv)
    again.step(30)
    assert np.abs(again.read(0, lbm.F_POP) - ref).max() < {"f64": 1e-14, "f32": 1e-7, "f16": 1e-5}[storage]


def test_error_codes_match_oracle():
    # bead stencil leaves the interior at the first step
    n = 12
    A = np.zeros((30, 9))
    pos = np.array([[9.6, 5.0, 5.0], [10.2, 5.1, 5.0]])
    c = Case((n, n, n), bc=(oracle.BC_AFFINE, A, 0, 1, 0),
             chains=[dict(pos=pos, fix_com=False, anchor=pos.mean(0))])
    ob = c.oracle_box()
    assert ob.step(5) == oracle.ERR_BEAD_OUT
    ctx = make_ctx(c)
    ctx.step(5)
    assert ctx.sync_status() == lbm.ERR_BEAD_OUT
    assert ctx.read(0, lbm.F_STEP, strict=False)[0] == ob.error()[1] == 0
    assert ctx.step_status(1) == lbm.ERR_BEAD_OUT
    # overstretched bond
    pos = np.array([[5.0, 5.0, 5.0], [7.01, 5.0, 5.0]])
    c = Case((n, n, n), bc=(oracle.BC_AFFINE, A, 0, 1, 0),
             chains=[dict(pos=pos, fix_com=True, anchor=pos.mean(0))])
    ob = c.oracle_box()
    assert ob.step(5) == oracle.ERR_FENE
    ctx = make_ctx(c)
    ctx.step(5)
    assert ctx.sync_status() == lbm.ERR_FENE
    # non-finite state caught by the mass check at t_2 (K = 2), frozen at t_1
    c = Case((n, n, n), bc=(oracle.BC_AFFINE, A, 0, 1, 0), reduce_every=2)
    ob = c.oracle_box()
    f = ob.pop()
    f[3, 5, 5, 5] = np.nan
    ob.set_populations(f)
    assert ob.step(5) == oracle.ERR_UNSTABLE
    assert ob.error() == (oracle.ERR_UNSTABLE, 1)
    ctx = make_ctx(c)
    ctx.write_state(0, lbm.F_POP, f)
    ctx.step(5)
    assert ctx.sync_status() == lbm.ERR_UNSTABLE
    assert ctx.read(0, lbm.F_STEP, strict=False)[0] == 1
    # stepping beyond the samples is refused on the host
    c = Case((n, n, n), bc=(oracle.BC_AFFINE, A[:3], 0, 1, 0))
    ctx = make_ctx(c)
    assert ctx.step_status(3) == 0
    assert ctx.step_status(1) == lbm.ERR_ARG


def zigzag_chain(n_beads, bond, centre, angle=0.5):
    """Planar zigzag of n_beads with every bond of the given length, centred
    (centre of mass) on ``centre``."""
    pos = np.zeros((n_beads, 3))
    for j in range(1, n_beads):
        a = angle if j % 2 else -angle
        pos[j] = pos[j - 1] + bond * np.array([np.cos(a), np.sin(a), 0.0])
    return pos + np.asarray(centre, dtype=np.float64) - pos.mean(axis=0)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_fene_near_full_extension(storage):
    """A chain pre-stretched to r^2/R0^2 = 0.856 (bonds 1.85, R0 = 2) in a
    walled box under a weak affine strain, with FP32 and FP16 population
    storage (the chain arithmetic is FP64 in every storage): the FENE factor
    1/(1 - r^2/R0^2) amplifies a separation's error sevenfold there; a small
    spring constant (3e-5) keeps every bond in 0.81 < r^2/R0^2 < 0.9 for the
    whole run.  Fluid and beads against the oracle."""
    n, steps = 24, 100
    xc = np.full(3, (n - 1) / 2.0)
    pos = zigzag_chain(8, 1.85, xc)
    A = inputs.ou_strain(steps + 1, inputs.rng(7, 0), corr_steps=50.0, rms=2e-4)
    case = Case((n, n, n), collision=oracle.MRT, tau=0.6, tau_bulk=0.6,
                bc=(oracle.BC_AFFINE, A, 0, 1, 0),
                chains=[dict(pos=pos, anchor=xc, fene_k=3e-5, fene_r0=2.0)], reduce_every=20)
    say("case FENE near full extension,", storage)
    ob = case.oracle_box()
    assert ob.step(steps) == 0
    p_o, _ = ob.beads()
    r2 = np.sum(np.diff(p_o, axis=0) ** 2, axis=1) / 4.0
    assert r2.min() > 0.81 and r2.max() < 0.9, r2  # near full extension throughout
    ctx = make_ctx(case, storage)
    ctx.step(steps)
    r = compare(ctx, ob, case, storage)
    check(r, storage, "FENE near full extension")
    ctx.close()


def _latch_case(kind):
    """A run that latches an error at step 3 with a wide margin: a dimer
    pulled apart by its initial velocities (bond 2.0041 > R0 = 2 at t_3), or
    one bead carried toward the -x wall (x = 0.994 < 1 at t_3, its stencil
    leaves the interior)."""
    n = 16
    xc = np.full(3, (n - 1) / 2.0)
    A = np.zeros((40, 9))
    if kind == "fene":
        pos = np.array([xc - [0.85, 0, 0], xc + [0.85, 0, 0]])
        vel = np.array([[-0.1, 0, 0], [0.1, 0, 0]])
        ch = dict(pos=pos, vel=vel, mass=1.0, zeta=0.5, fene_k=1e-6, fene_r0=2.0, anchor=xc,
                  fix_com=True)
    else:
        pos = np.array([[1.3, 7.2, 7.7]])
        ch = dict(pos=pos, vel=np.array([[-0.2, 0, 0]]), mass=1.0, zeta=0.5, anchor=pos[0],
                  fix_com=False)
    return Case((n, n, n), collision=oracle.MRT, tau=0.6, tau_bulk=0.6,
                bc=(oracle.BC_AFFINE, A, 0, 1, 0), chains=[ch], reduce_every=1)


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("kind", ["fene", "bead_out"])
def test_error_latch_reduced_precision(storage, kind):
    """FENE and BEAD_OUT latch at the oracle's step in FP32 and FP16 storage,
    and the state stays frozen at the last good step: fluid, beads and the
    mass/momentum record equal the oracle's at that step, and further steps
    return the latched error without changing them."""
    case = _latch_case(kind)
    code = {"fene": (oracle.ERR_FENE, lbm.ERR_FENE), "bead_out": (oracle.ERR_BEAD_OUT, lbm.ERR_BEAD_OUT)}[kind]
    say("case error latch", kind, storage)
    ob = case.oracle_box()
    assert ob.step(10) == code[0]
    assert ob.error() == (code[0], 3)
    ctx = make_ctx(case, storage)
    ctx.step(10)
    assert ctx.sync_status() == code[1]
    assert ctx.read(0, lbm.F_STEP, strict=False)[0] == 3
    r = compare(ctx, ob, case, storage, strict=False)
    # The last good step of the FENE case runs its final substeps at
    # 1 - r^2/R0^2 ~ 1e-3: there the FP32 bead coordinates (ulp 1.2e-7) set
    # the FENE force to ~1e-4 relative, which the friction update hands on to
    # the bead velocities (measured 1.8e-5 of them in FP32); their bound in
    # this case is 1e-3.
    skip = ("bead_vel", "bead_vel_max") if kind == "fene" else ()
    check(r, storage, f"frozen at the {kind} latch", skip=skip)
    assert r["bead_vel_max"] < 1e-3
    mm_o = ob.mass_mom()
    mm_g, st = ctx.read(0, lbm.F_MASS_MOM, strict=False)
    assert st == code[1] and mm_g[0] == mm_o[0] == 3
    pop = ctx.read(0, lbm.F_POP_DEV, strict=False)[0]
    assert ctx.step_status(5) == code[1]
    assert ctx.read(0, lbm.F_STEP, strict=False)[0] == 3
    assert np.array_equal(ctx.read(0, lbm.F_POP_DEV, strict=False)[0], pop)
    ctx.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_extended_overlapping_chains(storage):
    """Three 24-bead chains with bonds of 0.8 (random walks spanning 3-6 nodes
    per axis) whose anchors lie 2-3 nodes apart, so their stencil boxes
    overlap in part, in a walled 40^3 KS box: the force pass re-collides
    nodes that beads of several chains spread onto.  Spring constant 0.003
    keeps the fluid velocity at the per-mille level.  Against the oracle."""
    n, steps = 40, 100
    units, u0, faces = inputs.ks_box_inputs(1, 5, n=n, tau=0.6, n_steps=steps, dt=20, res=17)
    xc = np.full(3, (n - 1) / 2.0)
    chains = []
    for k, off in enumerate(([0, 0, 0], [2.5, 1.5, 0.5], [-1.5, 2.0, -2.5])):
        a = xc + np.asarray(off, dtype=np.float64)
        pos, vel = inputs.chain_init(24, a, inputs.rng(1, 20 + k), bond=0.8)
        chains.append(dict(pos=pos, vel=vel, anchor=a, mass=0.5 / 72, fene_k=0.003))
    case = Case((n, n, n), collision=oracle.MRT, tau=0.6, tau_bulk=0.6, ghost_rate=1.0,
                bc=(oracle.BC_SAMPLED, faces.astype(np.float32), 0, 20, 17), u0=u0, chains=chains,
                reduce_every=50)
    say("case extended overlapping chains,", storage)
    ob = case.oracle_box()
    assert ob.step(steps) == 0
    ctx = make_ctx(case, storage)
    ctx.step(steps)
    r = compare(ctx, ob, case, storage)
    check(r, storage, "extended chains")
    ctx.close()
